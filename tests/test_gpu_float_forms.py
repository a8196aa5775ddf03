"""GPU checks of the floating-point forms (FP32 Loeffler, FP16 / BF16 matrix form
on the matrix cores) against the FP64 definition, and of the YCbCr conversion.

Every coefficient and every pixel is held to its own rigorous rounding bound
(u = 2^-24, gamma_m = m u / (1 - m u)):

  * The matrix forms round K = C (x) C once to FP16 / BF16 (K^, computed here
    independently) and accumulate 64 exact products in FP32:
    |F^_j - F_j| <= sum_k |X_k| |K^_jk - K_jk| + gamma_64 sum_k |K^_jk X_k|.  The
    inverse starts its FP32 sum at 128.5 and takes the dequantized values d
    rounded to the operand type (exact in FP16, 2^-9 relative in BF16):
    |x^_k - x_k| <= sum_j |d_j| |K^_jk - K_jk| + sum_j |K^_jk| |d^_j - d_j|
                    + gamma_65 (128.5 + sum_j |K^_jk d^_j|).
  * The FP32 Loeffler form runs the flow graph with FP32 constants; the longest
    path through two passes meets 14 roundings (operations and constants), so
    the error is at most gamma_14 times the graph with every constant replaced
    by its magnitude and every subtraction by an addition, applied to |X|
    (computed here from the graph of Sec. 2.5.2); the inverse likewise, plus
    the rounding of the + 128.5.

A codec output is then checked against the FP64 codec block by block.  A
quantizer decision floor(|F| / Q + 1/2) whose exact value lies within the
coefficient bound (plus the quantizer's own three roundings) of a tie may go
either way: for an integer image the DC coefficient is sum / 8, a rational
that lands exactly on a tie for some blocks, and the FP64 codec decides such
a tie by its own rounding (the reading of the paper that lets FP ties go
either way).  Both sides of every such decision are tried; the block must
match one of them.  A reconstructed pixel floor(x + 128 + 1/2) whose exact
value lies within the pixel bound of an integer may likewise be either
neighbour; every other pixel must agree exactly.  Whole codecs must also
reproduce the FP64 codec's PSNR to 0.01 dB on images large enough for PSNR
to be meaningful.
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

from float_form_bounds import (K, K_HAT, U, blocks_of, bf16_round, check_codec_blocks, coef_bound,  # noqa: F401
                               pixel_bound)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


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


def synth(W, H, seed, sigma=5.0):
    from paper_1306_1373_amd.synth import synth_image
    return synth_image(W, H, seed, sigma)


def check_forward(hip, oracle_mod, img, form):
    got = hip.dct_forward_float(to_dev(img), form).cpu().numpy().astype(np.float64)
    exact = oracle_mod.exact_forward(img)
    err = np.abs(got - exact)
    bound = coef_bound(form, blocks_of(img))
    assert np.all(err <= bound), (err / bound).max()
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
    # Every block of a ragged image against the FP64 codec; in addition, an edge
    # block reads the nearest pixel past W / H, so the image codes exactly like its
    # edge-replicated extension to the block grid, cropped.
    img = synth(W, H, 7)
    src = to_dev(img, stride=((W + 7) // 8) * 8 + 16)
    dst = hip.new_plane(W, H, "cuda", stride=((W + 7) // 8) * 8 + 24)
    base = dst.as_strided((H, dst.stride(0)), (dst.stride(0), 1))
    base.fill_(0x33)
    _, sse = hip.dct_codec_float(src, form, 4, dst=dst)
    full = base.cpu().numpy()
    assert np.all(full[:, W:] == 0x33)                 # pad bytes untouched
    rec = full[:, :W]
    assert int(sse.cpu()[0]) == oracle_mod.sse(img, rec)
    nb, namb, nties = check_codec_blocks(oracle_mod, img, rec, form, 4)
    say(f"[gpu] ragged {form} {W}x{H}: {nb} blocks match the FP64 codec ({namb} with a quantizer decision "
        f"within reach of rounding, {nties} pixels at a reconstruction boundary)")
    Wp, Hp = -(-W // 8) * 8, -(-H // 8) * 8
    padded = np.pad(img, ((0, Hp - H), (0, Wp - W)), mode="edge")
    rec_p, _ = hip.dct_codec_float(to_dev(padded), form, 4)
    assert np.array_equal(rec, rec_p.cpu().numpy()[:H, :W])
    if W * H >= 40000:
        ref = oracle_mod.exact_codec(img, 4)
        assert abs(oracle_mod.psnr(img, rec) - oracle_mod.psnr(img, ref)) <= 0.01


@pytest.mark.parametrize("form", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("W,H,qs", [(512, 512, 4), (1024, 814, 8), (256, 256, 1), (96, 64, 16)])
def test_codec_blocks_match_fp64(hip, oracle_mod, form, W, H, qs):
    img = synth(W, H, 11)
    dst, _ = hip.dct_codec_float(to_dev(img), form, qs)
    nb, namb, nties = check_codec_blocks(oracle_mod, img, dst.cpu().numpy(), form, qs)
    say(f"[gpu] {form} {W}x{H} qs {qs}: {nb} blocks match the FP64 codec ({namb} with a quantizer decision "
        f"within reach of rounding, {nties} pixels at a reconstruction boundary)")


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
