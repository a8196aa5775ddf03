"""GPU parity of the recipe family R(n, F, G) (dct_codec_recipe) against the
oracle's recipe mode, bit for bit: reconstruction, int16 quantized values and
SSE, for every built recipe, at several quality scales, ragged sizes and padded
strides, and at 2048 x 2048."""
import sys

import numpy as np
import pytest


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

RECIPES = [(n, F, G) for n in (4, 6, 8, 10, 12) for F, G in ((8, 8), (12, 12), (16, 12))]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hip():
    from paper_1306_1373_amd import codec
    codec.load()
    return codec


def to_dev(img, stride=None, fill=0xA5):
    import torch
    H, W = img.shape
    stride = stride or ((W + 7) // 8) * 8
    buf = torch.full((H, stride), fill, dtype=torch.uint8, device="cuda")
    buf[:, :W] = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    return buf[:, :W]


def synth(W, H, seed, sigma=5.0):
    from paper_1306_1373_amd.synth import synth_image
    return synth_image(W, H, seed, sigma)


def check(hip, oracle_mod, recipe, img, qs, stride=None):
    H, W = img.shape
    src = to_dev(img, stride)
    dst, sse, q = hip.dct_codec_recipe(src, recipe, qs, want_qcoef=True)
    orec, osse, oq = oracle_mod.recipe_codec(*recipe, img, qs, want_q=True)
    assert np.array_equal(q.cpu().numpy(), oq), (recipe, qs, "qcoef")
    assert np.array_equal(dst.cpu().numpy(), orec), (recipe, qs, "reconstruction")
    assert int(sse.cpu()[0]) == osse, (recipe, qs, "sse")
    # the variant without the quantized output gives the same pixels and SSE
    dst2, sse2 = hip.dct_codec_recipe(src, recipe, qs)
    assert np.array_equal(dst2.cpu().numpy(), orec) and int(sse2.cpu()[0]) == osse
    return osse


@pytest.mark.parametrize("recipe", RECIPES, ids=lambda r: "R%d_%d_%d" % r)
def test_recipe_bit_exact_512(hip, oracle_mod, recipe):
    for seed, qs in ((0, 4), (1, 1), (2, 16), (3, 1024)):
        s = check(hip, oracle_mod, recipe, synth(512, 512, seed), qs)
        say(f"[gpu] R{recipe} seed {seed} qs {qs}: sse {s}")


@pytest.mark.parametrize("recipe", [(4, 16, 12), (8, 8, 8), (12, 12, 12)], ids=lambda r: "R%d_%d_%d" % r)
def test_recipe_ragged_and_strided(hip, oracle_mod, recipe):
    rng = np.random.default_rng(71)
    for W, H in ((1, 1), (7, 9), (13, 5), (1000, 1), (1024, 814), (200, 200)):
        check(hip, oracle_mod, recipe, synth(W, H, 5), 4, stride=((W + 7) // 8) * 8 + 8)
    # adversarial: 0 / 255 checkerboards of every basis sign pattern
    import scipy.fft as sf
    C8 = sf.dct(np.eye(8), type=2, norm="ortho", axis=0)
    C64 = np.kron(C8, C8)
    blocks = [np.where(s * C64[k] > 0, 255, 0).astype(np.uint8).reshape(8, 8) for k in range(64) for s in (1, -1)]
    img = np.ascontiguousarray(np.concatenate(blocks, axis=1))
    for qs in (1, 2, 7, 64, 1024):
        check(hip, oracle_mod, recipe, img, qs)
    check(hip, oracle_mod, recipe, rng.integers(0, 256, (96, 136), dtype=np.uint8), 3)


def test_default_recipe_is_dct_codec(hip, oracle_mod):
    img = synth(640, 480, 4)
    src = to_dev(img)
    a, sa, qa = hip.dct_codec(src, 4, want_qcoef=True)
    b, sb, qb = hip.dct_codec_recipe(src, (10, 12, 12), 4, want_qcoef=True)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    assert np.array_equal(qa.cpu().numpy(), qb.cpu().numpy())
    assert int(sa.cpu()[0]) == int(sb.cpu()[0])


def test_every_recipe_2048(hip, oracle_mod):
    from oracle import bands  # noqa: F401  (the oracle's recipe mode is whole-image)
    img = synth(2048, 2048, 6, sigma=4.0)
    src = to_dev(img)
    for recipe in RECIPES:
        dst, sse = hip.dct_codec_recipe(src, recipe, 4)
        orec, osse = oracle_mod.recipe_codec(*recipe, img, 4)
        assert int(sse.cpu()[0]) == osse, recipe
        assert np.array_equal(dst.cpu().numpy(), orec), recipe
        say(f"[gpu] 2048^2 R{recipe}: PSNR {oracle_mod.psnr_from_sse(osse, 2048, 2048):.4f}")


def test_unsupported_recipe_raises(hip):
    src = to_dev(synth(16, 16, 1))
    with pytest.raises(hip.DctError):
        hip.dct_codec_recipe(src, (5, 12, 12), 4)
