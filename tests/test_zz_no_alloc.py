"""GPU test of dct_psnr_noalloc, the SSE entry point that allocates nothing.

It is called through the C ABI (ctypes on the library, no Python wrapper) and
its {SSE, largest pixel} must equal what dct_psnr reports for the same planes,
and the oracle's exact SSE, on two calls in a row: the second on a smaller
image, so a partial left in the shared scratch by the first call would show.
Ragged widths exercise the byte-wise tail of the SSE pass.
"""
import ctypes as C
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


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def plane(img, stride, fill):
    import torch
    H, W = img.shape
    buf = torch.full((H, stride), fill, dtype=torch.uint8, device="cuda")
    buf[:, :W] = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    return buf


def pair(W, H, seed, qs):
    """A source image and its codec reconstruction, both from the oracle."""
    import oracle
    from paper_1306_1373_amd.synth import synth_image
    img = synth_image(W, H, seed, 5.0)
    rec, _ = oracle.cordic_codec(img, qs)
    return img, rec


def run_pair(lib, img, rec, result):
    import torch
    H, W = img.shape
    stride = ((W + 7) // 8) * 8 + 8
    a, b = plane(img, stride, 0xFF), plane(rec, stride, 0x00)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib.dct_psnr_noalloc(C.c_void_p(a.data_ptr()), stride, C.c_void_p(b.data_ptr()), stride, W, H,
                              C.c_void_p(result.data_ptr()), stream)
    assert st == 0, f"dct_psnr_noalloc status {st}"
    torch.cuda.synchronize()
    got = [int(v) for v in result.cpu().numpy().view(np.uint64)]
    psnr, sse = C.c_double(), C.c_uint64()
    st = lib.dct_psnr(C.c_void_p(a.data_ptr()), stride, C.c_void_p(b.data_ptr()), stride, W, H, C.c_double(0.0),
                      C.byref(psnr), C.byref(sse), stream)
    assert st == 0, f"dct_psnr status {st}"
    return got, int(sse.value), psnr.value


@pytest.mark.parametrize("first,second", [((1024, 776, 1), (40, 24, 2)), ((813, 601, 3), (13, 5, 4))])
def test_noalloc_matches_dct_psnr(first, second):
    import torch

    import oracle
    from paper_1306_1373_amd import codec
    lib = codec.load()
    result = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    for W, H, seed in (first, second):
        say(f"dct_psnr_noalloc {W}x{H} seed {seed}")
        img, rec = pair(W, H, seed, 8)
        got, sse, psnr = run_pair(lib, img, rec, result)
        assert got[0] == sse == oracle.sse(img, rec), (W, H, got, sse)
        assert got[1] == oracle.max_pixel(img)
        mine = C.c_double()
        assert lib.dct_psnr_from_sse(got[0], W * H, float(got[1]), C.byref(mine)) == 0
        assert mine.value == psnr


def test_noalloc_rejects_bad_arguments():
    import torch
    from paper_1306_1373_amd import codec
    lib = codec.load()
    a = torch.zeros((8, 16), dtype=torch.uint8, device="cuda")
    r = torch.zeros(2, dtype=torch.int64, device="cuda")
    p, pr = C.c_void_p(a.data_ptr()), C.c_void_p(r.data_ptr())
    assert lib.dct_psnr_noalloc(p, 16, p, 16, 16, 8, None, None) == codec.DCT_ERR_INVALID
    assert lib.dct_psnr_noalloc(p, 12, p, 16, 12, 8, pr, None) == codec.DCT_ERR_INVALID  # stride % 8
    assert lib.dct_psnr_noalloc(p, 16, p, 16, 17, 8, pr, None) == codec.DCT_ERR_INVALID  # W > stride
    assert lib.dct_psnr_noalloc(p, 16, p, 16, 16, 8, C.c_void_p(r.data_ptr() + 4), None) == codec.DCT_ERR_INVALID
