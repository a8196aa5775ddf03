"""GPU parity: every entry point of the C ABI against the CPU oracle, bit for bit.

The HIP path (through paper_1306_1373_amd.codec, which only marshals
pointers) and the oracle see the same seeded synthetic bytes.  The integer
recipe is exact, so every comparison is equality: coefficients, quantized
values, reconstructed pixels and SSE.  Sizes span one block up to the full
8192 x 8192 workload, ragged edges, padded strides, every quality scale, and
adversarial inputs.
"""
import math
import sys

import numpy as np
import pytest



def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hip():
    import torch
    from paper_1306_1373_amd import codec
    codec.load()
    torch.cuda.init()
    return codec


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def to_dev(img, stride=None, fill=0xA5):
    """Upload a (H, W) uint8 array into a device plane with the given row pitch;
    pad bytes hold `fill`."""
    import torch
    H, W = img.shape
    stride = stride or ((W + 7) // 8) * 8
    buf = torch.full((H, stride), fill, dtype=torch.uint8, device="cuda")
    buf[:, :W] = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    return buf[:, :W]


def host(t):
    return t.cpu().numpy()


def synth(W, H, seed, sigma=5.0):
    from paper_1306_1373_amd.synth import synth_image
    return synth_image(W, H, seed, sigma)


def check_all_stages(hip, oracle_mod, img, qs, stride=None):
    """Staged and fused paths against the oracle on one image."""
    import torch
    H, W = img.shape
    src = to_dev(img, stride)
    coef = hip.dct_forward(src)
    ocoef = oracle_mod.cordic_forward(img)
    assert np.array_equal(host(coef), ocoef), "forward"
    q = hip.dct_quantize(coef, qs)
    oq = oracle_mod.cordic_quantize(ocoef, qs)
    assert np.array_equal(host(q), oq), "quantize"
    dst = hip.new_plane(W, H, "cuda", stride=stride)
    pad_before = host(dst.as_strided((H, dst.stride(0)), (dst.stride(0), 1))) if stride else None
    hip.dct_inverse(q, qs, W, H, dst)
    orec = oracle_mod.cordic_inverse(oq, qs, W, H)
    assert np.array_equal(host(dst), orec), "inverse"
    if stride:
        pad_after = host(dst.as_strided((H, dst.stride(0)), (dst.stride(0), 1)))
        assert np.array_equal(pad_after[:, W:], pad_before[:, W:]), "pad bytes written"
    psnr, sse = hip.dct_psnr(src, dst)
    osse = oracle_mod.sse(img, orec)
    assert sse == osse, "psnr sse"
    assert psnr == oracle_mod.psnr_from_sse(osse, W, H) or (math.isinf(psnr) and osse == 0)
    # fused
    fdst, fsse, fq = hip.dct_codec(src, qs, want_qcoef=True)
    frec, fs, foq = oracle_mod.cordic_codec(img, qs, want_q=True)
    assert np.array_equal(host(fq), foq), "fused qcoef"
    assert np.array_equal(host(fdst), frec), "fused dst"
    assert int(host(fsse)[0]) == fs, "fused sse"
    assert fs == osse and np.array_equal(frec, orec)
    return fs


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_staged_and_fused_512(hip, oracle_mod, seed):
    say(f"[gpu] 512x512 seed {seed} qs 4")
    check_all_stages(hip, oracle_mod, synth(512, 512, seed), 4)


@pytest.mark.parametrize("qs", [1, 2, 8, 16, 1024])
def test_quality_scales_512(hip, oracle_mod, qs):
    say(f"[gpu] 512x512 seed 0 qs {qs}")
    check_all_stages(hip, oracle_mod, synth(512, 512, 0), qs)


def test_golden_oracle_record(hip, oracle_mod):
    # the GPU reproduces the oracle's recorded SSE for the 512x512 workload
    import json
    import os
    rec = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_codec_512.json")))
    for c in rec["cases"]:
        _, sse = hip.dct_codec(to_dev(synth(512, 512, c["seed"])), c["qs"])
        assert int(host(sse)[0]) == c["sse"], c


def test_every_quality_scale_fused(hip, oracle_mod):
    # all 1024 quality scales on a small image: the fused quantizer's division
    # constants for every table entry, against plain integer division
    say("[gpu] qs sweep 1..1024 on 64x48")
    img = synth(64, 48, 5, 8.0)
    src = to_dev(img)
    for qs in range(1, 1025):
        dst, sse, q = hip.dct_codec(src, qs, want_qcoef=True)
        rec, s, oq = oracle_mod.cordic_codec(img, qs, want_q=True)
        assert np.array_equal(host(q), oq), qs
        assert np.array_equal(host(dst), rec), qs
        assert int(host(sse)[0]) == s, qs


@pytest.mark.parametrize("W,H", [(1, 1), (7, 9), (9, 7), (13, 5), (1, 1000), (1000, 1), (200, 200),
                                 (1024, 814), (513, 257), (64, 8), (8, 64)])
def test_ragged_sizes(hip, oracle_mod, W, H):
    say(f"[gpu] ragged {W}x{H}")
    img = synth(W, H, W * 7 + H, 6.0)
    check_all_stages(hip, oracle_mod, img, 4)


@pytest.mark.parametrize("W,H,extra", [(37, 29, 24), (512, 64, 64), (1023, 17, 8)])
def test_padded_strides(hip, oracle_mod, W, H, extra):
    say(f"[gpu] padded {W}x{H} + {extra}")
    stride = ((W + 7) // 8) * 8 + extra
    check_all_stages(hip, oracle_mod, synth(W, H, 11, 5.0), 8, stride=stride)


def test_worst_case_blocks(hip, oracle_mod):
    # 0/255 along the sign of every DCT basis function: the largest intermediates
    import scipy.fft as sf
    C8 = sf.dct(np.eye(8), type=2, norm="ortho", axis=0)
    C64 = np.kron(C8, C8)
    blocks = [np.where(C64[k] > 0, 255, 0).astype(np.uint8).reshape(8, 8) for k in range(64)]
    blocks += [255 - b for b in blocks]
    img = np.ascontiguousarray(np.concatenate(blocks, axis=1))
    for qs in (1, 4, 64):
        check_all_stages(hip, oracle_mod, img, qs)


def test_constant_images(hip, oracle_mod):
    img = np.repeat(np.arange(256, dtype=np.uint8), 64).reshape(256, 8, 8)
    img = np.ascontiguousarray(img.transpose(1, 0, 2).reshape(8, 256 * 8))
    for qs in (1, 3, 16):
        check_all_stages(hip, oracle_mod, img, qs)


def test_inverse_arbitrary_int16(hip, oracle_mod, torch_mod):
    # any int16 input: dequantized values clamp to [-2048, 2047] before the inverse
    rng = np.random.default_rng(21)
    W, H = 96, 40
    nb = (W // 8) * (H // 8)
    q = rng.integers(-32768, 32768, (nb, 64), dtype=np.int64).astype(np.int16)
    q[0] = 32767
    q[1] = -32768
    q[2, ::2] = 32767
    q[2, 1::2] = -32768
    q[3:10] = rng.integers(-300, 300, (7, 64)).astype(np.int16)
    for qs in (1, 7, 1024):
        dst = hip.dct_inverse(torch_mod.from_numpy(q).cuda(), qs, W, H)
        assert np.array_equal(host(dst), oracle_mod.cordic_inverse(q, qs, W, H)), qs


def test_quantize_arbitrary_int32(hip, oracle_mod, torch_mod):
    # any int32 input: nearest integer, ties away from zero, int16 saturation
    rng = np.random.default_rng(22)
    rand = rng.integers(-(2 ** 31), 2 ** 31, (500, 64), dtype=np.int64)
    rand[0, :5] = [2 ** 31 - 1, -(2 ** 31), 0, 1, -1]
    for qs in (1, 5, 1024):
        # every tie point (and its neighbours) of every table entry, placed in a
        # slot (u, v) whose entry is that Q
        parts = [rand]
        for s in range(15):
            Q = 1 + (1 + s) * qs
            D = Q << 15
            m = np.arange(0, min(64, (2 ** 31 - 1) // D - 1))
            ties = np.concatenate([m * D + D // 2 + d for d in (-1, 0, 1)] +
                                  [m * D + d for d in (-1, 0, 1)])
            ties = np.concatenate([ties, -ties])
            u = min(s, 7)
            blk = np.zeros((ties.size, 64), np.int64)
            blk[:, u * 8 + (s - u)] = ties
            parts.append(blk)
        allc = np.concatenate(parts)
        assert allc.min() >= -(2 ** 31) and allc.max() < 2 ** 31
        allc = np.ascontiguousarray(allc.astype(np.int32))
        q = hip.dct_quantize(torch_mod.from_numpy(allc).cuda(), qs)
        assert np.array_equal(host(q), oracle_mod.cordic_quantize(allc, qs)), qs


def test_psnr_variants(hip, oracle_mod):
    rng = np.random.default_rng(23)
    a = rng.integers(0, 200, (77, 131), dtype=np.uint8)
    b = rng.integers(0, 256, (77, 131), dtype=np.uint8)
    da, db = to_dev(a, 136), to_dev(b, 160)
    p, s = hip.dct_psnr(da, db)
    assert s == oracle_mod.sse(a, b) and p == oracle_mod.psnr(a, b)
    p0, s0 = hip.dct_psnr(da, db, peak=0)
    assert s0 == s and abs(p0 - oracle_mod.psnr(a, b, peak=0)) < 1e-12
    pi, si = hip.dct_psnr(da, da)
    assert si == 0 and math.isinf(pi)


def test_psnr_grid_strides(hip, oracle_mod):
    # a width of three workgroups of segments with a ragged last segment, and more
    # rows than the grid has in y, so every stride of the SSE kernel is taken
    rng = np.random.default_rng(29)
    H, W = 1401, 5003
    a = rng.integers(0, 251, (H, W), dtype=np.uint8)
    b = rng.integers(0, 256, (H, W), dtype=np.uint8)
    a[H - 1, W - 1] = 253          # the largest pixel sits in the last, ragged segment
    # pad bytes that would change both the SSE and the maximum if they were read
    da, db = to_dev(a, 5008, fill=254), to_dev(b, 5016, fill=1)
    p, s = hip.dct_psnr(da, db)
    assert s == oracle_mod.sse(a, b) and p == oracle_mod.psnr(a, b)
    p0, s0 = hip.dct_psnr(da, db, peak=0)
    assert s0 == s and abs(p0 - oracle_mod.psnr(a, b, peak=0)) < 1e-12


def test_determinism_and_streams(hip, oracle_mod, torch_mod):
    img = synth(640, 360, 9)
    src = to_dev(img)
    d1, s1, q1 = hip.dct_codec(src, 4, want_qcoef=True)
    side = torch_mod.cuda.Stream()
    with torch_mod.cuda.stream(side):
        d2, s2, q2 = hip.dct_codec(src, 4, want_qcoef=True)
    side.synchronize()
    torch_mod.cuda.synchronize()
    assert torch_mod.equal(d1, d2) and torch_mod.equal(s1, s2) and torch_mod.equal(q1, q2)


def test_accumulate_over_bands(hip, oracle_mod, torch_mod):
    # dct_codec_accumulate over two block-aligned bands of one image (two planes
    # that are views of one buffer): the reconstruction and the summed SSE equal
    # the whole image's, and a second pass adds the same SSE again
    W, H, cut = 1000, 620, 312
    img = synth(W, H, 12)
    src = to_dev(img)
    rec, osse, oq = oracle_mod.cordic_codec(img, 6, want_q=True)
    dst = hip.new_plane(W, H, "cuda")
    sse = torch_mod.zeros(1, dtype=torch_mod.int64, device="cuda")
    for rep in (1, 2):
        _, _, q_top = hip.dct_codec_accumulate(src[:cut], 6, sse, dst=dst[:cut], want_qcoef=True)
        _, _, q_bot = hip.dct_codec_accumulate(src[cut:], 6, sse, dst=dst[cut:], want_qcoef=True)
        torch_mod.cuda.synchronize()
        assert int(host(sse)[0]) == rep * osse
        assert np.array_equal(host(dst), rec)
        assert np.array_equal(np.concatenate([host(q_top), host(q_bot)]), oq)


@pytest.mark.parametrize("W,H,qs", [(512, 512, 4), (1, 1, 4), (13, 5, 2), (1024, 814, 8), (333, 97, 16),
                                    (2048, 1536, 4)])
def test_block_mapping_bit_exact(hip, oracle_mod, W, H, qs):
    # the lane-per-block codec (transpose in registers) against the oracle, with
    # padded strides; dct_codec itself (one lane per block row) is checked by
    # every other test here
    img = synth(W, H, 40 + W % 7)
    src = to_dev(img, stride=((W + 7) // 8) * 8 + 16)
    dst, sse, q = hip.dct_codec_blocks(src, qs, want_qcoef=True)
    rec, osse, oq = oracle_mod.cordic_codec(img, qs, want_q=True)
    assert int(host(sse)[0]) == osse
    assert np.array_equal(host(q), oq)
    assert np.array_equal(host(dst), rec)


def test_invalid_arguments_raise(hip, torch_mod):
    src = to_dev(synth(16, 16, 1))
    with pytest.raises(hip.DctError) as e:
        hip.dct_codec(src, 0)
    assert e.value.status == hip.DCT_ERR_INVALID
    with pytest.raises(hip.DctError):
        hip.dct_quantize(torch_mod.zeros((4, 64), dtype=torch_mod.int32, device="cuda"), 2000)
    empty = torch_mod.zeros((0, 64), dtype=torch_mod.int32, device="cuda")
    assert hip.dct_quantize(empty, 4).numel() == 0


def test_full_size_8192(hip, oracle_mod):
    # the 8192 x 8192 workload in the launch configuration the benchmark times:
    # fused codec and all staged entry points, whole image, bit for bit
    from oracle import bands
    from paper_1306_1373_amd.synth import sigma_for_seed
    seed = 3
    say(f"[gpu] 8192x8192 seed {seed} sigma {sigma_for_seed(seed):.3f} qs 4: generating")
    img = synth(8192, 8192, seed, sigma_for_seed(seed))
    src = to_dev(img)
    say("[gpu] 8192x8192 fused codec")
    dst, sse, q = hip.dct_codec(src, 4, want_qcoef=True)
    rec_h, sse_h, q_h = host(dst), int(host(sse)[0]), host(q)
    say("[gpu] 8192x8192 oracle (band-parallel)")
    orec, osse, oq = bands.codec_bands(img, 4, threads=16, want_q=True)
    assert sse_h == osse
    assert np.array_equal(q_h, oq)
    assert np.array_equal(rec_h, orec)
    say("[gpu] 8192x8192 fused codec, lane-per-block mapping")
    d_blk, s_blk, q_blk = hip.dct_codec_blocks(src, 4, want_qcoef=True)
    assert int(host(s_blk)[0]) == osse
    assert np.array_equal(host(d_blk), orec)
    assert np.array_equal(host(q_blk), oq)
    del d_blk, q_blk
    say("[gpu] 8192x8192 fused codec, accumulating entry point (the benchmark's)")
    import torch
    acc = torch.zeros(1, dtype=torch.int64, device="cuda")
    dst3 = hip.new_plane(8192, 8192, "cuda")
    hip.dct_codec_accumulate(src, 4, acc, dst=dst3)
    hip.dct_codec_accumulate(src, 4, acc, dst=dst3)
    assert int(host(acc)[0]) == 2 * osse
    assert np.array_equal(host(dst3), orec)
    del dst3
    say("[gpu] 8192x8192 staged path")
    coef = hip.dct_forward(src)
    assert np.array_equal(host(coef), bands.forward_bands(img, threads=16))
    q2 = hip.dct_quantize(coef, 4)
    assert np.array_equal(host(q2), oq)
    del coef
    d2 = hip.dct_inverse(q2, 4, 8192, 8192)
    assert np.array_equal(host(d2), orec)
    p, s2 = hip.dct_psnr(src, d2)
    assert s2 == osse
    assert p == oracle_mod.psnr_from_sse(osse, 8192, 8192)
