"""GPU checks of the floating-point forms (FP32 Loeffler, FP16 / BF16 matrix form
on the matrix cores) against the FP64 definition, and of the YCbCr conversion.

The matrix forms round C (x) C once to FP16 / BF16 and accumulate in FP32, so
every coefficient must lie within sum_k |x_k| |K^_jk - K_jk| + (64 u) sum_k |x_k K^_jk|
of the exact value, with K^ the rounded matrix (computed here independently)
and u = 2^-24: a rigorous per-coefficient bound that a wrong lane layout or a
wrong matrix entry breaks.  The FP32 Loeffler form is held to 2e-3 (about thirty
rounded operations of 2^-24 relative error on values up to 2^13).  Whole codecs
must reproduce the FP64 codec's PSNR to 0.01 dB.
"""
import math
import sys

import numpy as np
import pytest
import scipy.fft as sf


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

C8 = sf.dct(np.eye(8), type=2, norm="ortho", axis=0)
K = np.kron(C8, C8)   # K[j][k], j = 8u + v, k = 8i + jj


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def bf16_round(x):
    """Round float64 values to the nearest bfloat16 (8 significant bits, ties to even)."""
    m, e = np.frexp(x)                 # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(m * 256.0) / 256.0, e)


K_HAT = {"f16": np.float16(K).astype(np.float64), "bf16": bf16_round(K)}


@pytest.fixture(scope="module")
def hip():
    from paper_1306_1373_amd import codec
    codec.load()
    return codec


def to_dev(img, stride=None):
    import torch
    H, W = img.shape
    stride = stride or ((W + 7) // 8) * 8
    buf = torch.full((H, stride), 0x5A, dtype=torch.uint8, device="cuda")
    buf[:, :W] = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    return buf[:, :W]


def blocks_of(img):
    H, W = img.shape
    Hp, Wp = -(-H // 8) * 8, -(-W // 8) * 8
    p = np.pad(img, ((0, Hp - H), (0, Wp - W)), mode="edge").astype(np.float64) - 128
    return p.reshape(Hp // 8, 8, Wp // 8, 8).transpose(0, 2, 1, 3).reshape(-1, 64)


def synth(W, H, seed, sigma=5.0):
    from paper_1306_1373_amd.synth import synth_image
    return synth_image(W, H, seed, sigma)


def check_forward(hip, oracle_mod, img, form):
    got = hip.dct_forward_float(to_dev(img), form).cpu().numpy().astype(np.float64)
    exact = oracle_mod.exact_forward(img)
    err = np.abs(got - exact)
    if form == "f32":
        assert err.max() < 2e-3, err.max()
    else:
        X = np.abs(blocks_of(img))
        bound = X @ np.abs(K_HAT[form] - K).T + 64 * 2.0 ** -24 * (X @ np.abs(K_HAT[form]).T) + 1e-6
        assert np.all(err <= bound), (err - bound).max()
    return err.max()


@pytest.mark.parametrize("form", ["f32", "f16", "bf16"])
def test_forward_within_bound(hip, oracle_mod, form):
    rng = np.random.default_rng(51)
    for img in (synth(512, 512, 0), rng.integers(0, 256, (64, 96), dtype=np.uint8),
                synth(37, 29, 3), np.full((16, 16), 255, np.uint8)):
        e = check_forward(hip, oracle_mod, img, form)
        say(f"[gpu] forward {form} {img.shape}: max abs err {e:.3g}")


@pytest.mark.parametrize("form", ["f32", "f16", "bf16"])
def test_basis_images(hip, oracle_mod, form):
    # each block of the image is one (scaled, integer-rounded) basis function
    blocks = []
    for k in range(64):
        b = np.clip(np.rint(128 + 100 * sf.idctn(np.eye(64)[k].reshape(8, 8), type=2, norm="ortho") * 8),
                    0, 255).astype(np.uint8)
        blocks.append(b)
    img = np.ascontiguousarray(np.concatenate(blocks, axis=1))
    check_forward(hip, oracle_mod, img, form)


@pytest.mark.parametrize("form", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("qs", [2, 4, 8, 16])
def test_codec_psnr_matches_fp64(hip, oracle_mod, form, qs):
    for seed in (0, 1):
        img = synth(512, 512, seed)
        dst, sse = hip.dct_codec_float(to_dev(img), form, qs)
        rec = dst.cpu().numpy()
        s = int(sse.cpu()[0])
        assert s == oracle_mod.sse(img, rec)          # the device SSE is exact for its output
        p_gpu = oracle_mod.psnr_from_sse(s, 512, 512)
        p_ref = oracle_mod.psnr(img, oracle_mod.exact_codec(img, qs))
        say(f"[gpu] codec {form} qs {qs} seed {seed}: PSNR {p_gpu:.5f} vs FP64 {p_ref:.5f}")
        assert abs(p_gpu - p_ref) <= 0.01


@pytest.mark.parametrize("form", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("W,H", [(1024, 814), (13, 5), (200, 200), (1, 1), (9, 17)])
def test_codec_ragged(hip, oracle_mod, form, W, H):
    # An edge block reads the nearest pixel past W / H, so a ragged image codes
    # exactly like its edge-replicated extension to the block grid, cropped.
    img = synth(W, H, 7)
    src = to_dev(img, stride=((W + 7) // 8) * 8 + 16)
    dst = hip.new_plane(W, H, "cuda", stride=((W + 7) // 8) * 8 + 24)
    base = dst.as_strided((H, dst.stride(0)), (dst.stride(0), 1))
    base.fill_(0x33)
    _, sse = hip.dct_codec_float(src, form, 4, dst=dst)
    full = base.cpu().numpy()
    assert np.all(full[:, W:] == 0x33)                 # pad bytes untouched
    rec = full[:, :W]
    Wp, Hp = -(-W // 8) * 8, -(-H // 8) * 8
    padded = np.pad(img, ((0, Hp - H), (0, Wp - W)), mode="edge")
    rec_p, _ = hip.dct_codec_float(to_dev(padded), form, 4)
    assert np.array_equal(rec, rec_p.cpu().numpy()[:H, :W])
    assert int(sse.cpu()[0]) == oracle_mod.sse(img, rec)
    if W * H >= 40000:
        ref = oracle_mod.exact_codec(img, 4)
        assert abs(oracle_mod.psnr(img, rec) - oracle_mod.psnr(img, ref)) <= 0.02


# largest coefficient / pixel error of each form against FP64, with margin
FORM_TOL = {"f32": 2e-3, "f16": 0.06}


@pytest.mark.parametrize("form", ["f32", "f16"])
@pytest.mark.parametrize("W,H,qs", [(512, 512, 4), (1024, 814, 8), (256, 256, 1)])
def test_codec_tie_aware_pixels(hip, oracle_mod, form, W, H, qs):
    # Where the FP64 codec is decided with room to spare the form must agree with
    # it exactly; only values within the form's error of a rounding tie (of the
    # quantizer or of the reconstruction) may go either way.
    tol = FORM_TOL[form]
    img = synth(W, H, 11)
    dst, _ = hip.dct_codec_float(to_dev(img), form, qs)
    rec = dst.cpu().numpy()
    Fx = oracle_mod.exact_forward(img)                     # [nblocks, 64]
    Q = oracle_mod.qtable(qs).reshape(64).astype(np.float64)
    r = np.abs(Fx) / Q
    ambiguous = np.abs(r - np.floor(r) - 0.5) < tol / Q
    q = np.sign(Fx) * np.floor(r + 0.5)
    bw, bh = oracle_mod.grid(W, H)
    checked = 0
    for b in np.flatnonzero(~ambiguous.any(axis=1)):
        by, bx = divmod(int(b), bw)
        x = oracle_mod.idct8x8((q[b] * Q).reshape(8, 8)) + 128.0
        lo, hi = np.clip(np.floor(x + 0.5 - tol), 0, 255), np.clip(np.floor(x + 0.5 + tol), 0, 255)
        h, w = min(8, H - by * 8), min(8, W - bx * 8)
        got = rec[by * 8:by * 8 + h, bx * 8:bx * 8 + w]
        assert np.all((got >= lo[:h, :w]) & (got <= hi[:h, :w])), (b, form)
        checked += 1
    say(f"[gpu] {form} {W}x{H} qs {qs}: {checked} of {bw * bh} blocks decided, all agree")
    assert checked >= 0.25 * bw * bh


def test_ycbcr_bit_exact(hip, oracle_mod):
    import torch
    rng = np.random.default_rng(52)
    # packed rows of odd width (byte path), packed rows of width 256 (8-pixel path),
    # and rows padded to an 8-byte multiple with a ragged tail (both paths)
    for (H, W, pitch) in ((97, 131, None), (50, 256, None), (41, 131, 408), (3, 8, 24), (1, 1, None)):
        rgb = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
        if pitch is None:
            dev = torch.from_numpy(rgb).cuda()
        else:
            buf = torch.zeros((H, pitch), dtype=torch.uint8, device="cuda")
            buf[:, :3 * W] = torch.from_numpy(rgb.reshape(H, 3 * W)).cuda()
            dev = buf.as_strided((H, W, 3), (pitch, 3, 1))
        planes = hip.dct_rgb_to_ycbcr(dev)
        for got, ref in zip(planes, oracle_mod.rgb_to_ycbcr(rgb)):
            assert np.array_equal(got.cpu().numpy(), ref), (H, W, pitch)


def test_precision_workload_image(hip, oracle_mod):
    # one image of the precision workload: 2048 x 2048 RGB -> YCbCr -> each plane
    # through every form; PSNR within 0.01 dB of the FP64 codec on every plane
    import torch
    from oracle import bands
    from paper_1306_1373_amd.synth import synth_rgb
    rgb = synth_rgb(2048, 2048, 5)
    planes = hip.dct_rgb_to_ycbcr(torch.from_numpy(rgb).cuda())
    host_planes = oracle_mod.rgb_to_ycbcr(rgb)
    for name, dev, ref_plane in zip("Y Cb Cr".split(), planes, host_planes):
        assert np.array_equal(dev.cpu().numpy(), ref_plane)
        ref = bands.exact_codec_bands(ref_plane, 8, threads=16)
        p_ref = oracle_mod.psnr(ref_plane, ref)
        for form in ("f32", "f16", "bf16"):
            dst, sse = hip.dct_codec_float(dev, form, 8)
            p = oracle_mod.psnr_from_sse(int(sse.cpu()[0]), 2048, 2048)
            say(f"[gpu] 2048^2 {name} {form}: PSNR {p:.5f} vs FP64 {p_ref:.5f}")
            assert abs(p - p_ref) <= 0.01


def test_invalid_form(hip):
    import torch
    src = to_dev(synth(16, 16, 1))
    with pytest.raises(hip.DctError):
        hip.dct_forward_float(src, 7)
    with pytest.raises(hip.DctError):
        hip.dct_codec_float(src, "f16", 0)


@pytest.mark.parametrize("form", ["f16", "bf16"])
def test_fused_rgb_codec_matches_separate_steps(hip, form):
    # dct_codec_rgb_float == dct_rgb_to_ycbcr followed by dct_codec_float per plane, bit for bit
    import torch
    from paper_1306_1373_amd.synth import synth_rgb
    rng = np.random.default_rng(53)
    cases = [(synth_rgb(200, 136, 21), None), (synth_rgb(131, 97, 22), None), (synth_rgb(131, 41, 23), 400),
             (rng.integers(0, 256, (16, 24, 3), dtype=np.uint8), None), (synth_rgb(5, 3, 24), None)]
    for rgb, pitch in cases:
        H, W, _ = rgb.shape
        if pitch is None:
            dev = torch.from_numpy(rgb).cuda()
        else:
            buf = torch.zeros((H, pitch), dtype=torch.uint8, device="cuda")
            buf[:, :3 * W] = torch.from_numpy(rgb.reshape(H, 3 * W)).cuda()
            dev = buf.as_strided((H, W, 3), (pitch, 3, 1))
        fused, sse = hip.dct_codec_rgb_float(dev, form, 8)
        planes = hip.dct_rgb_to_ycbcr(dev)
        for c in range(3):
            ref, s1 = hip.dct_codec_float(planes[c], form, 8)
            assert np.array_equal(fused[c].cpu().numpy(), ref.cpu().numpy()), (W, H, pitch, c)
            assert int(sse[c].cpu()) == int(s1.cpu()[0]), (W, H, pitch, c)


def test_fused_rgb_rejects_f32(hip):
    import torch
    rgb = torch.zeros((8, 8, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(hip.DctError):
        hip.dct_codec_rgb_float(rgb, "f32", 8)
