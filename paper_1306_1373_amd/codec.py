"""Python binding of the C ABI in include/dctcodec.h.

Argument marshalling only: each function checks tensor dtypes, shapes and
devices, allocates missing outputs with torch (device memory is torch's), and
passes raw pointers and the current HIP stream to the library.  Every step of
the codec runs in the library's HIP kernels; there is no fallback path, and a
missing or unloadable library raises.

Planes are 2-D uint8 CUDA (HIP) tensors of shape (H, W) whose rows are
contiguous (``stride(1) == 1``); a row pitch larger than W (a column slice of
a wider buffer) is passed through as the plane's stride.
"""
import ctypes as C
import os

from . import build as _build

_lib = None

DCT_OK = 0
DCT_ERR_INVALID = -1
DCT_ERR_UNSUPPORTED = -2
DCT_ERR_DEVICE = -3
DCT_ERR_NOMEM = -4

DCT_FORM_F32_LOEFFLER = 1
DCT_FORM_MFMA_F16 = 2
DCT_FORM_MFMA_BF16 = 3
FORMS = {"f32": DCT_FORM_F32_LOEFFLER, "f16": DCT_FORM_MFMA_F16, "bf16": DCT_FORM_MFMA_BF16}

# prototypes of include/dctcodec.h
_PROTOS = {
    "dct_forward": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "dct_quantize": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p]),
    "dct_inverse": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                              C.c_void_p]),
    "dct_psnr": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                           C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_uint64), C.c_void_p]),
    "dct_codec": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                            C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dct_codec_accumulate": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                       C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dct_codec_blocks": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                 C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dct_forward_float": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                    C.c_void_p, C.c_void_p]),
    "dct_codec_float": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                  C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "dct_codec_rgb_float": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "dct_rgb_to_ycbcr": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_int32, C.c_void_p]),
    "dct_codec_recipe": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                   C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.c_void_p]),
    "dct_recipe_supported": (C.c_int, [C.c_int32, C.c_int32, C.c_int32]),
    "dct_recipe_list": (C.c_int, [C.POINTER(C.c_int32), C.c_int32]),
    "dct_recipe_tables_n": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "dct_batch_workspace_size": (C.c_size_t, [C.c_void_p, C.c_int32, C.c_int32]),
    "dct_batch_plan": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_size_t,
                                 C.POINTER(C.c_int64), C.c_void_p]),
    "dct_batch_run": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "dct_batch_run_threads": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "dct_batch_release": (C.c_int, [C.c_void_p]),
    "dct_deblock_nparam": (C.c_int32, []),
    "dct_deblock_workspace_size": (C.c_size_t, [C.c_int64, C.c_int32]),
    "dct_deblock_apply": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p]),
    "dct_deblock_apply_stack": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                          C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p]),
    "dct_deblock_forward": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                                      C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                      C.c_void_p]),
    "dct_deblock_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                   C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_size_t, C.c_void_p]),
    "dct_deblock_adam": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float,
                                   C.c_float, C.c_float, C.c_float, C.c_void_p]),
    "dct_deblock_init": (C.c_int, [C.c_uint64, C.c_void_p, C.c_void_p]),
    "dct_deblock_select": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_double),
                                     C.POINTER(C.c_int32), C.c_void_p]),
    "dct_psnr_from_sse": (C.c_int, [C.c_uint64, C.c_int64, C.c_double, C.POINTER(C.c_double)]),
    "dct_psnr_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                   C.c_void_p, C.c_void_p]),
    "dct_recipe_info": (C.c_int, [C.POINTER(C.c_int32)] * 3),
    "dct_recipe_tables": (C.c_int, [C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "dct_probe_copy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "dct_status_string": (C.c_char_p, [C.c_int]),
    "dct_shutdown": (C.c_int, []),
}


class DctImage(C.Structure):
    """dct_image of the C ABI: one image of a batch."""
    _fields_ = [("src", C.c_void_p), ("dst", C.c_void_p), ("W", C.c_int32), ("H", C.c_int32),
                ("src_stride", C.c_int32), ("dst_stride", C.c_int32), ("qs", C.c_int32),
                ("reserved", C.c_int32)]


class DctError(RuntimeError):
    """A dct_* call returned a status other than DCT_OK."""

    def __init__(self, status: int, where: str):
        self.status = status
        msg = load().dct_status_string(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {msg} (status {status})")


def library_path() -> str:
    return os.environ.get("DCTCODEC_LIB", _build.LIB)


def load() -> C.CDLL:
    """Load libdctcodec.so (built by ``python -m paper_1306_1373_amd.build``).

    torch is imported first so that the HIP runtime the library links against
    is the one torch already loaded (both use the soname libamdhip64.so.7)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime first)
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run python -m paper_1306_1373_amd.build")
    L = C.CDLL(path)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status: int, where: str):
    if status != DCT_OK:
        raise DctError(status, where)


def _stream(t) -> int:
    import torch
    return torch.cuda.current_stream(t.device).cuda_stream


def _plane(t, name: str):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or t.dim() != 2:
        raise TypeError(f"{name} must be a 2-D uint8 tensor")
    if not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.stride(1) != 1:
        raise TypeError(f"{name} rows must be contiguous")
    H, W = t.shape
    stride = t.stride(0) if H > 1 else max(W, ((W + 7) // 8) * 8)
    return t.data_ptr(), int(W), int(H), int(stride)


def grid(W: int, H: int):
    """(blocks per row, block rows) of a W x H image."""
    return (W + 7) // 8, (H + 7) // 8


def nblocks(W: int, H: int) -> int:
    bw, bh = grid(W, H)
    return bw * bh


def new_plane(W: int, H: int, device, stride: int = None):
    """A (H, W) uint8 device plane whose rows are ``stride`` bytes apart
    (default: W rounded up to a multiple of 8)."""
    import torch
    stride = stride or ((W + 7) // 8) * 8
    buf = torch.empty((H, stride), dtype=torch.uint8, device=device)
    return buf[:, :W]


def dct_forward(src, coef=None):
    """a1-a4: int32 coefficients [nblocks, 64] of a uint8 plane (value / 2^15)."""
    import torch
    p, W, H, s = _plane(src, "src")
    nb = nblocks(W, H)
    if coef is None:
        coef = torch.empty((nb, 64), dtype=torch.int32, device=src.device)
    if coef.dtype != torch.int32 or not coef.is_contiguous() or coef.numel() != nb * 64:
        raise TypeError("coef must be a contiguous int32 tensor of nblocks * 64 elements")
    _check(load().dct_forward(p, W, H, s, coef.data_ptr(), _stream(src)), "dct_forward")
    return coef


def dct_quantize(coef, qs: int, qcoef=None):
    """a5: int16 quantized values of int32 coefficients, table Q = 1 + (1 + u + v) qs."""
    import torch
    if coef.dtype != torch.int32 or not coef.is_contiguous() or coef.numel() % 64:
        raise TypeError("coef must be a contiguous int32 tensor of whole blocks")
    nb = coef.numel() // 64
    if qcoef is None:
        qcoef = torch.empty((nb, 64), dtype=torch.int16, device=coef.device)
    if qcoef.dtype != torch.int16 or not qcoef.is_contiguous() or qcoef.numel() != nb * 64:
        raise TypeError("qcoef must be a contiguous int16 tensor of nblocks * 64 elements")
    _check(load().dct_quantize(coef.data_ptr(), nb, int(qs), qcoef.data_ptr(), _stream(coef)),
           "dct_quantize")
    return qcoef


def dct_inverse(qcoef, qs: int, W: int, H: int, dst=None):
    """a6-a8: W x H uint8 reconstruction of int16 quantized values."""
    import torch
    if qcoef.dtype != torch.int16 or not qcoef.is_contiguous() or qcoef.numel() != nblocks(W, H) * 64:
        raise TypeError("qcoef must be a contiguous int16 tensor matching the block grid")
    if dst is None:
        dst = new_plane(W, H, qcoef.device)
    p, dW, dH, s = _plane(dst, "dst")
    if (dW, dH) != (W, H):
        raise ValueError("dst shape does not match W, H")
    _check(load().dct_inverse(qcoef.data_ptr(), int(qs), W, H, p, s, _stream(qcoef)), "dct_inverse")
    return dst


def dct_psnr(a, b, peak: float = 255.0):
    """(psnr, sse) of plane b against plane a (waits for the stream)."""
    pa, W, H, sa = _plane(a, "a")
    pb, W2, H2, sb = _plane(b, "b")
    if (W, H) != (W2, H2):
        raise ValueError("planes differ in shape")
    out = C.c_double()
    sse = C.c_uint64()
    _check(load().dct_psnr(pa, sa, pb, sb, W, H, float(peak), C.byref(out), C.byref(sse),
                           _stream(a)), "dct_psnr")
    return out.value, int(sse.value)


def dct_psnr_noalloc(a, b, result=None):
    """Enqueue the SSE of plane b against plane a without any allocation in the
    library; returns a two-element int64 device tensor {SSE, largest pixel of a}
    (``result`` if given).  Does not wait for the stream."""
    import torch
    pa, W, H, sa = _plane(a, "a")
    pb, W2, H2, sb = _plane(b, "b")
    if (W, H) != (W2, H2):
        raise ValueError("planes differ in shape")
    if result is None:
        result = torch.empty(2, dtype=torch.int64, device=a.device)
    if result.dtype != torch.int64 or not result.is_contiguous() or result.numel() < 2:
        raise TypeError("result must be a contiguous int64 tensor of two elements")
    _check(load().dct_psnr_noalloc(pa, sa, pb, sb, W, H, result.data_ptr(), _stream(a)), "dct_psnr_noalloc")
    return result


def dct_codec(src, qs: int, dst=None, qcoef=None, sse=None, want_qcoef: bool = False):
    """a1-a9 in one pass.  Returns (dst, sse_tensor) or (dst, sse_tensor, qcoef);
    sse_tensor is a one-element int64 device tensor holding the uint64 SSE."""
    return _codec(src, qs, dst, qcoef, sse, want_qcoef, None)


def dct_codec_accumulate(src, qs: int, sse, dst=None, qcoef=None, want_qcoef: bool = False):
    """dct_codec that adds the SSE into ``sse`` (a one-element int64 device tensor the
    caller has zeroed) instead of overwriting it; returns as dct_codec."""
    return _codec(src, qs, dst, qcoef, sse, want_qcoef, "accumulate")


def dct_codec_blocks(src, qs: int, dst=None, qcoef=None, sse=None, want_qcoef: bool = False):
    """dct_codec with the lane-per-block mapping (the transpose in registers); returns as dct_codec."""
    return _codec(src, qs, dst, qcoef, sse, want_qcoef, "blocks")


def dct_codec_recipe(src, recipe, qs: int, dst=None, qcoef=None, sse=None, want_qcoef: bool = False):
    """dct_codec under recipe (n, F, G); returns as dct_codec."""
    n, F, G = (int(v) for v in recipe)
    return _codec(src, qs, dst, qcoef, sse, want_qcoef, (n, F, G))


def _codec(src, qs, dst, qcoef, sse, want_qcoef, recipe):
    import torch
    p, W, H, s = _plane(src, "src")
    if dst is None:
        dst = new_plane(W, H, src.device)
    pd, dW, dH, ds = _plane(dst, "dst")
    if (dW, dH) != (W, H):
        raise ValueError("dst shape does not match src")
    if want_qcoef and qcoef is None:
        qcoef = torch.empty((nblocks(W, H), 64), dtype=torch.int16, device=src.device)
    if qcoef is not None and (qcoef.dtype != torch.int16 or not qcoef.is_contiguous()
                              or qcoef.numel() != nblocks(W, H) * 64):
        raise TypeError("qcoef must be a contiguous int16 tensor matching the block grid")
    if sse is None:
        sse = torch.empty(1, dtype=torch.int64, device=src.device)
    qptr = None if qcoef is None else qcoef.data_ptr()
    if recipe is None:
        _check(load().dct_codec(p, W, H, s, int(qs), pd, ds, qptr, sse.data_ptr(), _stream(src)),
               "dct_codec")
    elif recipe == "blocks":
        _check(load().dct_codec_blocks(p, W, H, s, int(qs), pd, ds, qptr, sse.data_ptr(), _stream(src)),
               "dct_codec_blocks")
    elif recipe == "accumulate":
        if sse.dtype != torch.int64 or sse.numel() < 1 or not sse.is_cuda:
            raise TypeError("sse must be an int64 device tensor")
        _check(load().dct_codec_accumulate(p, W, H, s, int(qs), pd, ds, qptr, sse.data_ptr(), _stream(src)),
               "dct_codec_accumulate")
    else:
        _check(load().dct_codec_recipe(p, W, H, s, *recipe, int(qs), pd, ds, qptr, sse.data_ptr(),
                                       _stream(src)), "dct_codec_recipe")
    return (dst, sse, qcoef) if qcoef is not None else (dst, sse)


def _form(form) -> int:
    return FORMS[form] if isinstance(form, str) else int(form)


def dct_forward_float(src, form, coef=None):
    """Orthonormal float32 coefficients [nblocks, 64] in a floating-point form
    ('f32' Loeffler, 'f16' or 'bf16' matrix form on the matrix cores)."""
    import torch
    p, W, H, s = _plane(src, "src")
    nb = nblocks(W, H)
    if coef is None:
        coef = torch.empty((nb, 64), dtype=torch.float32, device=src.device)
    if coef.dtype != torch.float32 or not coef.is_contiguous() or coef.numel() != nb * 64:
        raise TypeError("coef must be a contiguous float32 tensor of nblocks * 64 elements")
    _check(load().dct_forward_float(p, W, H, s, _form(form), coef.data_ptr(), _stream(src)),
           "dct_forward_float")
    return coef


def dct_codec_float(src, form, qs: int, dst=None, sse=None):
    """The codec with a floating-point transform; returns (dst, sse_tensor)."""
    import torch
    p, W, H, s = _plane(src, "src")
    if dst is None:
        dst = new_plane(W, H, src.device)
    pd, dW, dH, ds = _plane(dst, "dst")
    if (dW, dH) != (W, H):
        raise ValueError("dst shape does not match src")
    if sse is None:
        sse = torch.empty(1, dtype=torch.int64, device=src.device)
    _check(load().dct_codec_float(p, W, H, s, _form(form), int(qs), pd, ds, sse.data_ptr(),
                                  _stream(src)), "dct_codec_float")
    return dst, sse


def dct_rgb_to_ycbcr(rgb, planes=None):
    """(Y, Cb, Cr) uint8 planes of an (H, W, 3) uint8 RGB device tensor."""
    import torch
    if not isinstance(rgb, torch.Tensor) or rgb.dtype != torch.uint8 or rgb.dim() != 3 \
            or rgb.shape[2] != 3 or not rgb.is_cuda:
        raise TypeError("rgb must be an (H, W, 3) uint8 device tensor")
    if rgb.stride(2) != 1 or rgb.stride(1) != 3:
        raise TypeError("rgb pixels must be interleaved and contiguous within a row")
    H, W, _ = rgb.shape
    if planes is None:
        planes = tuple(new_plane(W, H, rgb.device) for _ in range(3))
    ptrs, strides = [], set()
    for t in planes:
        pt, pW, pH, ps = _plane(t, "plane")
        if (pW, pH) != (W, H):
            raise ValueError("plane shape does not match rgb")
        ptrs.append(pt)
        strides.add(ps)
    if len(strides) != 1:
        raise ValueError("the three planes must share one row pitch")
    rs = rgb.stride(0) if H > 1 else 3 * W
    _check(load().dct_rgb_to_ycbcr(rgb.data_ptr(), int(W), int(H), int(rs), *ptrs, strides.pop(),
                                   _stream(rgb)), "dct_rgb_to_ycbcr")
    return planes


class Batch:
    """A planned batch (dct_batch_plan) and its device workspace; run() codes every
    image with one launch.  srcs / dsts are 2-D uint8 device planes; qs is an int
    or one int per image."""

    def __init__(self, srcs, dsts, qs, chunk: int = 512):
        import torch
        if len(srcs) != len(dsts) or not srcs:
            raise ValueError("need matching, non-empty source and destination lists")
        qs_list = [int(qs)] * len(srcs) if isinstance(qs, int) else [int(q) for q in qs]
        if len(qs_list) != len(srcs):
            raise ValueError("one qs per image")
        arr = (DctImage * len(srcs))()
        for k, (a, b, q) in enumerate(zip(srcs, dsts, qs_list)):
            pa, W, H, sa = _plane(a, "src")
            pb, Wb, Hb, sb = _plane(b, "dst")
            if (W, H) != (Wb, Hb):
                raise ValueError(f"image {k}: dst shape does not match src")
            arr[k] = DctImage(pa, pb, W, H, sa, sb, q, 0)
        L = load()
        n = len(srcs)
        size = L.dct_batch_workspace_size(arr, n, int(chunk))
        if size == 0:
            raise DctError(DCT_ERR_INVALID, "dct_batch_workspace_size")
        dev = srcs[0].device
        self.workspace = torch.empty(size + 256, dtype=torch.uint8, device=dev)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = self.workspace.data_ptr() + off
        total = C.c_int64()
        _check(L.dct_batch_plan(arr, n, int(chunk), self._ws_ptr, size, C.byref(total), _stream(srcs[0])),
               "dct_batch_plan")
        self.n_images, self.chunk, self.total_chunks = n, int(chunk), total.value
        self.sse = torch.zeros(n, dtype=torch.int64, device=dev)
        self._keep = (list(srcs), list(dsts))

    def run(self, grid: int = 0, sse=None, threads: int = None):
        """Code the batch (threads lanes per workgroup: None for min(chunk, 512));
        returns the int64 device tensor of per-image SSEs."""
        out = self.sse if sse is None else sse
        if threads is None:
            _check(load().dct_batch_run(self._ws_ptr, int(grid), out.data_ptr(), _stream(out)), "dct_batch_run")
        else:
            _check(load().dct_batch_run_threads(self._ws_ptr, int(grid), int(threads), out.data_ptr(), _stream(out)),
                   "dct_batch_run_threads")
        return out

    def release(self):
        if self._ws_ptr is not None:
            load().dct_batch_release(self._ws_ptr)
            self._ws_ptr = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Deblocker:
    """The learned deblocking post-filter (dct_deblock_*): FP32 master parameters
    and Adam moments on the device, and workspaces sized on demand.  Crops are
    given as an int32 device tensor [n, 2] of top-left (row, col) positions in a
    decoded plane (and the matching original plane) of the same pitch.

    params: a host array of 19105 values, or None for the library's initial
    parameters of `seed` (dct_deblock_init)."""

    def __init__(self, params=None, device="cuda", seed: int = 0):
        import numpy as np
        import torch
        n = load().dct_deblock_nparam()
        if params is None:
            self.params = torch.empty(n, dtype=torch.float32, device=device)
            _check(load().dct_deblock_init(int(seed), self.params.data_ptr(), _stream(self.params)),
                   "dct_deblock_init")
        else:
            params = np.asarray(params, dtype=np.float32)
            if params.size != n:
                raise ValueError(f"expected {n} parameters")
            self.params = torch.from_numpy(params.copy()).to(device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)
        self.step_count = 0
        self._ws = {}

    def _workspace(self, npix: int, training: bool):
        import torch
        key = (int(npix), bool(training))
        if key not in self._ws:
            size = load().dct_deblock_workspace_size(int(npix), int(training))
            if size == 0:
                raise DctError(DCT_ERR_INVALID, "dct_deblock_workspace_size")
            buf = torch.empty(size + 256, dtype=torch.uint8, device=self.params.device)
            off = (-buf.data_ptr()) % 256
            self._ws = {key: (buf, buf.data_ptr() + off, size)}
        return self._ws[key]

    def apply(self, decoded, out=None):
        """The filtered plane (uint8) of a decoded plane."""
        p, W, H, s = _plane(decoded, "decoded")
        if out is None:
            out = new_plane(W, H, decoded.device)
        po, Wo, Ho, so = _plane(out, "out")
        if (Wo, Ho) != (W, H):
            raise ValueError("out shape does not match")
        _, ws, size = self._workspace(W * H, False)
        _check(load().dct_deblock_apply(p, W, H, s, self.params.data_ptr(), po, so, ws, size,
                                        _stream(decoded)), "dct_deblock_apply")
        return out

    def apply_stack(self, decoded, n: int, out=None):
        """The filtered planes (uint8) of n images of equal height stacked
        vertically in the decoded plane, in one launch."""
        p, W, rows, s = _plane(decoded, "decoded")
        if n < 1 or rows % n:
            raise ValueError("the plane's rows must hold n images of equal height")
        if out is None:
            out = new_plane(W, rows, decoded.device)
        po, Wo, Ho, so = _plane(out, "out")
        if (Wo, Ho) != (W, rows):
            raise ValueError("out shape does not match")
        H = rows // n
        _, ws, size = self._workspace(W * H, False)
        _check(load().dct_deblock_apply_stack(p, W, H, int(n), s, self.params.data_ptr(), po, so, ws, size,
                                              _stream(decoded)), "dct_deblock_apply_stack")
        return out

    def forward(self, decoded, pos, h: int, w: int):
        """y (float32, [n, h, w]) of the crops of a decoded plane."""
        import torch
        p, W, H, s = _plane(decoded, "decoded")
        n = 1 if pos is None else int(pos.shape[0])
        y = torch.empty((n, h, w), dtype=torch.float32, device=decoded.device)
        _, ws, size = self._workspace(n * h * w, True)
        _check(load().dct_deblock_forward(p, W, H, s, None if pos is None else pos.data_ptr(), n, h, w,
                                          self.params.data_ptr(), y.data_ptr(), ws, size, _stream(decoded)),
               "dct_deblock_forward")
        return y

    def compute_grad(self, decoded, original, pos, h: int, w: int):
        """Gradient (into self.grad) and mean squared error (self.loss) of the crops."""
        p, W, H, s = _plane(decoded, "decoded")
        po, Wo, Ho, so = _plane(original, "original")
        if (Wo, Ho, so) != (W, H, s):
            raise ValueError("decoded and original planes must have the same shape and pitch")
        n = 1 if pos is None else int(pos.shape[0])
        _, ws, size = self._workspace(n * h * w, True)
        _check(load().dct_deblock_grad(p, po, W, H, s, None if pos is None else pos.data_ptr(), n, h, w,
                                       self.params.data_ptr(), self.grad.data_ptr(), self.loss.data_ptr(), ws,
                                       size, _stream(decoded)), "dct_deblock_grad")
        return self.grad, self.loss

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.step_count += 1
        _check(load().dct_deblock_adam(self.params.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                                       self.grad.data_ptr(), self.step_count, lr, beta1, beta2, eps,
                                       _stream(self.params)), "dct_deblock_adam")

    def train_step(self, decoded, original, pos, h: int, w: int, lr: float):
        self.compute_grad(decoded, original, pos, h, w)
        self.adam(lr)
        return self.loss

    def select(self, sse_plain, sse_filtered):
        """The fallback rule (dct_deblock_select): keep the trained filter only if
        it raises the mean PSNR of a validation set, else zero its output layer.
        sse_plain / sse_filtered: int64 device tensors of per-image SSEs of the
        decoded and the filtered planes.  Returns (mean gain in dB, kept)."""
        import torch
        for t in (sse_plain, sse_filtered):
            if t.dtype != torch.int64 or not t.is_contiguous() or not t.is_cuda:
                raise TypeError("SSEs must be contiguous int64 device tensors")
        if sse_plain.numel() != sse_filtered.numel():
            raise ValueError("one SSE of each kind per image")
        gain, kept = C.c_double(), C.c_int32()
        _check(load().dct_deblock_select(sse_plain.data_ptr(), sse_filtered.data_ptr(), int(sse_plain.numel()),
                                         self.params.data_ptr(), C.byref(gain), C.byref(kept),
                                         _stream(self.params)), "dct_deblock_select")
        return gain.value, bool(kept.value)


def dct_codec_rgb_float(rgb, form, qs: int, planes=None, sse=None):
    """The matrix-form codec of the Y, Cb, Cr planes of an (H, W, 3) uint8 device RGB
    tensor in one pass; returns ((y, cb, cr) reconstructions, sse tensor [3])."""
    import torch
    if not isinstance(rgb, torch.Tensor) or rgb.dtype != torch.uint8 or rgb.dim() != 3 \
            or rgb.shape[2] != 3 or not rgb.is_cuda:
        raise TypeError("rgb must be an (H, W, 3) uint8 device tensor")
    if rgb.stride(2) != 1 or rgb.stride(1) != 3:
        raise TypeError("rgb pixels must be interleaved and contiguous within a row")
    H, W, _ = rgb.shape
    if planes is None:
        planes = tuple(new_plane(W, H, rgb.device) for _ in range(3))
    ptrs, strides = [], set()
    for t in planes:
        pt, pW, pH, ps = _plane(t, "plane")
        if (pW, pH) != (W, H):
            raise ValueError("plane shape does not match rgb")
        ptrs.append(pt)
        strides.add(ps)
    if len(strides) != 1:
        raise ValueError("the three planes must share one row pitch")
    if sse is None:
        sse = torch.empty(3, dtype=torch.int64, device=rgb.device)
    rs = rgb.stride(0) if H > 1 else 3 * W
    _check(load().dct_codec_rgb_float(rgb.data_ptr(), int(W), int(H), int(rs), _form(form), int(qs), *ptrs,
                                      strides.pop(), sse.data_ptr(), _stream(rgb)), "dct_codec_rgb_float")
    return planes, sse


def psnr_from_sse(sse: int, W: int, H: int, peak: float = 255.0) -> float:
    """PSNR (eq. (23)) of an SSE that dct_codec left in device memory (dct_psnr_from_sse)."""
    out = C.c_double()
    _check(load().dct_psnr_from_sse(int(sse), int(W) * int(H), float(peak), C.byref(out)), "dct_psnr_from_sse")
    return out.value


def recipe_info():
    n, f, p = C.c_int32(), C.c_int32(), C.c_int32()
    _check(load().dct_recipe_info(C.byref(n), C.byref(f), C.byref(p)), "dct_recipe_info")
    return n.value, f.value, p.value


def recipe_tables(n: int = None):
    """(directions[3][n], gains[4]) of the default recipe, or of the built recipes with n."""
    if n is None:
        n = recipe_info()[0]
        d = (C.c_int32 * (3 * n))()
        g = (C.c_int32 * 4)()
        _check(load().dct_recipe_tables(d, g), "dct_recipe_tables")
    else:
        d = (C.c_int32 * (3 * n))()
        g = (C.c_int32 * 4)()
        _check(load().dct_recipe_tables_n(int(n), d, g), "dct_recipe_tables_n")
    return [[d[r * n + i] for i in range(n)] for r in range(3)], list(g)


def recipe_list():
    """The built recipes as (n, F, G) triples, the default first."""
    L = load()
    count = L.dct_recipe_list(None, 0)
    buf = (C.c_int32 * (3 * count))()
    L.dct_recipe_list(buf, count)
    return [(buf[3 * i], buf[3 * i + 1], buf[3 * i + 2]) for i in range(count)]


def recipe_supported(n: int, F: int, G: int) -> bool:
    return bool(load().dct_recipe_supported(int(n), int(F), int(G)))


def probe_copy(src, dst):
    """Measurement aid, not an operation of the codec: copies the bytes of the
    contiguous device tensor src into dst (same byte count, 16-byte aligned, a
    multiple of 16 bytes) with the library's plain non-temporal copy, on the
    current stream.  Timed, it gives the HBM bandwidth a pure stream reaches."""
    for t, name in ((src, "src"), (dst, "dst")):
        if not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous device tensor")
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n:
        raise ValueError("src and dst differ in size")
    _check(load().dct_probe_copy(src.data_ptr(), dst.data_ptr(), n, _stream(src)), "dct_probe_copy")


def status_string(status: int) -> str:
    return load().dct_status_string(status).decode()


def shutdown():
    _check(load().dct_shutdown(), "dct_shutdown")
