"""CPU parity oracle for the blockwise 8x8 Cordic-based Loeffler DCT codec.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the product library never does, and
this package never touches the product library.

The arithmetic lives in ``oracle.c`` (plain C, FP64 / int64); this module only
marshals NumPy arrays through ctypes.  Each function names the passage of the
paper it follows (Sec. 2.5.1 eq. (6)-(7) for the DCT, Sec. 2.5.2 for the
Loeffler graph with CORDIC rotation blocks, Sec. 3.2 for the quantizer, Sec. 4.1
eq. (23)-(24) for PSNR).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

N_ITER = 10   # CORDIC micro-rotations per rotation block
FRAC = 12     # fractional bits of the fixed-point samples
PBITS = 15    # fractional bits of the gain constants

ROT_PI_16, ROT_3PI_16, ROT_6PI_16 = 0, 1, 2

_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i16p = np.ctypeslib.ndpointer(dtype=np.int16, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_intp = np.ctypeslib.ndpointer(dtype=np.intc, flags="C_CONTIGUOUS")


def lib():
    """Load (building first if needed) liboracle.so."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("ORACLE_LIB_OVERRIDE")  # the mutation tests load planted mistakes
    if not path:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
    L = C.CDLL(path)
    sig = {
        "or_fdct8x8_f64": (None, [_f64p, _f64p]),
        "or_idct8x8_f64": (None, [_f64p, _f64p]),
        "or_exact_forward": (None, [_u8p, C.c_int, C.c_int, C.c_int, _f64p]),
        "or_exact_codec": (None, [_u8p, C.c_int, C.c_int, C.c_int, C.c_int, _u8p, C.c_int,
                                  C.c_void_p]),
        "or_sse": (C.c_uint64, [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_int]),
        "or_max_pixel": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int]),
        "or_psnr_from_sse": (C.c_double, [C.c_uint64, C.c_int, C.c_int, C.c_double]),
        "or_recipe_info": (None, [C.POINTER(C.c_int)] * 3),
        "or_recipe_tables": (None, [_intp, _i64p]),
        "or_cordic_forward": (C.c_int64, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p]),
        "or_cordic_quantize": (None, [C.c_void_p, C.c_int64, C.c_int, C.c_void_p]),
        "or_cordic_inverse": (C.c_int64, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p,
                                          C.c_int]),
        "or_cordic_codec": (C.c_uint64, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                         C.c_void_p, C.c_int, C.c_void_p]),
        "or_cordic_forward_block": (C.c_int64, [_i64p, _i64p]),
        "or_cordic_inverse_block": (C.c_int64, [_i64p, _i64p]),
        "or_cordic_rotate_pair": (None, [C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_int,
                                         C.c_int]),
        "or_recipe_quantize": (C.c_int64, [C.c_int64, C.c_int64]),
        "or_recipe_dequantize": (C.c_int64, [C.c_int64, C.c_int64]),
        "or_recipe_reconstruct": (C.c_int, [C.c_int64]),
        "or_rgb_to_ycbcr": (None, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_int]),
        "or_recipe_valid": (C.c_int, [C.c_int, C.c_int, C.c_int]),
        "or_recipe_tables_n": (None, [C.c_int, _intp, _i64p]),
        "or_recipe_codec": (C.c_uint64, [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int,
                                         C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p]),
        "or_recipe_forward_block": (C.c_int64, [C.c_int, C.c_int, C.c_int, _i64p, _i64p]),
        "or_recipe_inverse_block": (C.c_int64, [C.c_int, C.c_int, C.c_int, _i64p, _i64p]),
        "or_recipe_peaks": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int,
                                      C.c_int, C.c_int, C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64)]),
        "or_db_nparam": (C.c_int, []),
        "or_conv3x3": (None, [_f64p, C.c_int, C.c_int, C.c_int, _f64p, C.c_void_p, C.c_int, _f64p]),
        "or_conv3x3_bwd": (None, [_f64p, C.c_int, C.c_int, C.c_int, _f64p, C.c_int, _f64p, C.c_void_p,
                                  C.c_void_p, C.c_void_p]),
        "or_db_forward": (None, [_f64p, _f64p, C.c_int, C.c_int, _f64p, C.c_void_p]),
        "or_db_loss_grad": (C.c_double, [_f64p, _f64p, _f64p, C.c_int, C.c_int, C.c_int, C.c_void_p]),
        "or_adam_step": (None, [_f64p, _f64p, _f64p, _f64p, C.c_long, C.c_double, C.c_double, C.c_double,
                                C.c_double, C.c_int]),
        "or_loeffler_forward_f64": (None, [_f64p, _f64p]),
        "or_loeffler_inverse_f64": (None, [_f64p, _f64p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _plane(img: np.ndarray):
    """(array, W, H, stride) of a 2-D uint8 plane whose rows may be padded."""
    if img.dtype != np.uint8 or img.ndim != 2:
        raise TypeError("expected a 2-D uint8 plane")
    if img.strides[1] != 1:
        raise TypeError("plane rows must be contiguous")
    return img, img.shape[1], img.shape[0], img.strides[0]


def grid(W: int, H: int):
    """Block grid (blocks per row, block rows) of a W x H image."""
    return (W + 7) // 8, (H + 7) // 8


def qtable(qs: int) -> np.ndarray:
    """Quantization table Q[u][v] = 1 + (1 + u + v) * qs (int64, 8x8)."""
    u = np.arange(8)[:, None]
    v = np.arange(8)[None, :]
    return (1 + (1 + u + v) * qs).astype(np.int64)


# ---- O1 / O2: exact DCT ----------------------------------------------------

def fdct8x8(block) -> np.ndarray:
    """Orthonormal 2-D DCT-II of one 8x8 block by the O(N^4) definition (eq. (6))."""
    f = np.ascontiguousarray(block, dtype=np.float64).reshape(64)
    out = np.empty(64, np.float64)
    lib().or_fdct8x8_f64(f, out)
    return out.reshape(8, 8)


def idct8x8(coef) -> np.ndarray:
    """Orthonormal 2-D DCT-III (the inverse of eq. (6)) of one 8x8 block."""
    F = np.ascontiguousarray(coef, dtype=np.float64).reshape(64)
    out = np.empty(64, np.float64)
    lib().or_idct8x8_f64(F, out)
    return out.reshape(8, 8)


def exact_forward(img: np.ndarray) -> np.ndarray:
    """Exact FP64 coefficients [nblocks, 64] of (img - 128), edge-replicated."""
    a, W, H, _ = _plane(img)
    src = np.ascontiguousarray(a)
    bw, bh = grid(W, H)
    out = np.empty((bw * bh, 64), np.float64)
    lib().or_exact_forward(src, W, H, W, out)
    return out


def exact_codec(img: np.ndarray, qs: int, want_q: bool = False):
    """Exact FP64 codec: DCT, quantize, dequantize, IDCT, level shift, round, clamp.
    Returns the reconstruction (H, W) uint8, and the quantized values if asked."""
    a, W, H, _ = _plane(img)
    src = np.ascontiguousarray(a)
    dst = np.empty((H, W), np.uint8)
    bw, bh = grid(W, H)
    q = np.empty((bw * bh, 64), np.float64) if want_q else None
    lib().or_exact_codec(src, W, H, W, qs, dst, W, None if q is None else _ptr(q))
    return (dst, q) if want_q else dst


# ---- O6: PSNR ----------------------------------------------------------------

def sse(a: np.ndarray, b: np.ndarray) -> int:
    """Exact sum of squared differences over the common W x H region (eq. (24))."""
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    if a.shape != b.shape:
        raise ValueError("shape mismatch")
    H, W = a.shape
    return int(lib().or_sse(_ptr(a), W, _ptr(b), W, W, H))


def max_pixel(a: np.ndarray) -> int:
    a = np.ascontiguousarray(a, dtype=np.uint8)
    H, W = a.shape
    return int(lib().or_max_pixel(_ptr(a), W, W, H))


def psnr_from_sse(sse_value: int, W: int, H: int, peak: float = 255.0) -> float:
    """PSNR = 20 log10(MAX / sqrt(MSE)) (eq. (23)); +inf when SSE is 0."""
    return float(lib().or_psnr_from_sse(int(sse_value), W, H, float(peak)))


def psnr(orig: np.ndarray, recon: np.ndarray, peak: float = 255.0) -> float:
    """PSNR of recon against orig; peak 0 means MAX = max(orig) (eq. (23))."""
    H, W = orig.shape
    if peak == 0:
        peak = float(max_pixel(orig))
    return psnr_from_sse(sse(orig, recon), W, H, peak)


# ---- O7: the integer Cordic-based Loeffler recipe -------------------------------

def recipe_info():
    n, f, p = C.c_int(), C.c_int(), C.c_int()
    lib().or_recipe_info(C.byref(n), C.byref(f), C.byref(p))
    return n.value, f.value, p.value


def recipe_tables():
    """(directions[3, n], gains[4]): CORDIC directions of the pi/16, 3pi/16 and
    6pi/16 rotation blocks, and M(pi/16), M(3pi/16), M(6pi/16) (with sqrt 2), M_sqrt2."""
    d = np.zeros(3 * N_ITER, np.intc)
    g = np.zeros(4, np.int64)
    lib().or_recipe_tables(d, g)
    return d.reshape(3, N_ITER).astype(np.int64), g


def cordic_forward(img: np.ndarray, return_peak: bool = False):
    """a1..a4: int32 coefficients [nblocks, 64] (coefficient = value / 2^15)."""
    a, W, H, _ = _plane(img)
    src = np.ascontiguousarray(a)
    bw, bh = grid(W, H)
    coef = np.empty((bw * bh, 64), np.int32)
    peak = lib().or_cordic_forward(_ptr(src), W, H, W, _ptr(coef))
    return (coef, int(peak)) if return_peak else coef


def cordic_quantize(coef: np.ndarray, qs: int) -> np.ndarray:
    """a5: int32 coefficients -> int16 quantized values."""
    coef = np.ascontiguousarray(coef, dtype=np.int32)
    nb = coef.size // 64
    q = np.empty((nb, 64), np.int16)
    lib().or_cordic_quantize(_ptr(coef), nb, qs, _ptr(q))
    return q


def cordic_inverse(qcoef: np.ndarray, qs: int, W: int, H: int, return_peak: bool = False):
    """a6..a8: int16 quantized values -> (H, W) uint8 reconstruction."""
    qcoef = np.ascontiguousarray(qcoef, dtype=np.int16)
    bw, bh = grid(W, H)
    if qcoef.size != bw * bh * 64:
        raise ValueError("qcoef size does not match the block grid")
    dst = np.empty((H, W), np.uint8)
    peak = lib().or_cordic_inverse(_ptr(qcoef), qs, W, H, _ptr(dst), W)
    return (dst, int(peak)) if return_peak else dst


def cordic_codec(img: np.ndarray, qs: int, want_q: bool = False):
    """a1..a9: returns (reconstruction, sse[, qcoef])."""
    a, W, H, _ = _plane(img)
    src = np.ascontiguousarray(a)
    dst = np.empty((H, W), np.uint8)
    bw, bh = grid(W, H)
    q = np.empty((bw * bh, 64), np.int16) if want_q else None
    s = lib().or_cordic_codec(_ptr(src), W, H, W, qs, _ptr(dst), W,
                              None if q is None else _ptr(q))
    if s == 2**64 - 1:
        raise MemoryError("oracle codec could not allocate")
    return (dst, int(s), q) if want_q else (dst, int(s))


def cordic_forward_block(x) -> tuple:
    """Forward recipe on one block of raw fixed-point samples; (c[8,8], peak)."""
    xi = np.ascontiguousarray(x, dtype=np.int64).reshape(64)
    c = np.empty(64, np.int64)
    peak = lib().or_cordic_forward_block(xi, c)
    return c.reshape(8, 8), int(peak)


def cordic_inverse_block(d) -> tuple:
    """Inverse recipe on one block of fixed-point coefficients; (x[8,8], peak)."""
    di = np.ascontiguousarray(d, dtype=np.int64).reshape(64)
    x = np.empty(64, np.int64)
    peak = lib().or_cordic_inverse_block(di, x)
    return x.reshape(8, 8), int(peak)


# ---- O7 family: recipe R(n, F, G) ------------------------------------------

def _recipe_ok(n: int, F: int, G: int):
    if not lib().or_recipe_valid(n, F, G):
        raise ValueError(f"recipe R({n}, {F}, {G}) outside 1<=n<=16, 1<=F<=16, 1<=G<=12")


def recipe_tables_n(n: int):
    """(directions[3, n], gains[4]) of the recipe with n micro-rotations."""
    _recipe_ok(n, 12, 12)
    d = np.zeros(3 * n, np.intc)
    g = np.zeros(4, np.int64)
    lib().or_recipe_tables_n(n, d, g)
    return d.reshape(3, n).astype(np.int64), g


def recipe_codec(n: int, F: int, G: int, img: np.ndarray, qs: int, want_q: bool = False):
    """a1..a9 under recipe R(n, F, G): (reconstruction, sse[, qcoef])."""
    _recipe_ok(n, F, G)
    a, W, H, _ = _plane(img)
    src = np.ascontiguousarray(a)
    dst = np.empty((H, W), np.uint8)
    bw, bh = grid(W, H)
    q = np.empty((bw * bh, 64), np.int16) if want_q else None
    s = lib().or_recipe_codec(n, F, G, _ptr(src), W, H, W, qs, _ptr(dst), W,
                              None if q is None else _ptr(q))
    if s == 2**64 - 1:
        raise MemoryError("oracle codec could not allocate")
    return (dst, int(s), q) if want_q else (dst, int(s))


def recipe_forward_block(n: int, F: int, G: int, x) -> tuple:
    """Forward recipe R(n, F, G) on one block of raw fixed-point samples; (c, peak)."""
    _recipe_ok(n, F, G)
    xi = np.ascontiguousarray(x, dtype=np.int64).reshape(64)
    c = np.empty(64, np.int64)
    peak = lib().or_recipe_forward_block(n, F, G, xi, c)
    return c.reshape(8, 8), int(peak)


def recipe_inverse_block(n: int, F: int, G: int, d) -> tuple:
    """Inverse recipe R(n, F, G) on one block of fixed-point coefficients; (x, peak)."""
    _recipe_ok(n, F, G)
    di = np.ascontiguousarray(d, dtype=np.int64).reshape(64)
    x = np.empty(64, np.int64)
    peak = lib().or_recipe_inverse_block(n, F, G, di, x)
    return x.reshape(8, 8), int(peak)


def recipe_peaks(n: int, F: int, G: int, img: np.ndarray, qs: int):
    """(forward peak, inverse peak): the largest |value| R(n, F, G) stores on img at qs."""
    _recipe_ok(n, F, G)
    a, W, H, _ = _plane(img)
    src = np.ascontiguousarray(a)
    fp, ip = C.c_int64(), C.c_int64()
    if lib().or_recipe_peaks(n, F, G, _ptr(src), W, H, W, qs, C.byref(fp), C.byref(ip)) != 0:
        raise MemoryError("oracle could not allocate")
    return int(fp.value), int(ip.value)


def cordic_rotate(a: int, b: int, rot: int, sense: int = 1):
    """One rotation block alone: n micro-rotations then gain compensation."""
    x, y = C.c_int64(a), C.c_int64(b)
    lib().or_cordic_rotate_pair(C.byref(x), C.byref(y), rot, sense)
    return x.value, y.value


def recipe_quantize(c: int, Q: int) -> int:
    return int(lib().or_recipe_quantize(int(c), int(Q)))


def recipe_dequantize(q: int, Q: int) -> int:
    return int(lib().or_recipe_dequantize(int(q), int(Q)))


def recipe_reconstruct(x: int) -> int:
    return int(lib().or_recipe_reconstruct(int(x)))


def loeffler_forward_f64(x) -> np.ndarray:
    xi = np.ascontiguousarray(x, dtype=np.float64).reshape(8)
    out = np.empty(8, np.float64)
    lib().or_loeffler_forward_f64(xi, out)
    return out


def loeffler_inverse_f64(Z) -> np.ndarray:
    Zi = np.ascontiguousarray(Z, dtype=np.float64).reshape(8)
    out = np.empty(8, np.float64)
    lib().or_loeffler_inverse_f64(Zi, out)
    return out


def rgb_to_ycbcr(rgb: np.ndarray):
    """Integer full-range YCbCr planes (Y, Cb, Cr) of an (H, W, 3) uint8 RGB image."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    H, W, ch = rgb.shape
    if ch != 3:
        raise ValueError("expected (H, W, 3)")
    y = np.empty((H, W), np.uint8)
    cb = np.empty((H, W), np.uint8)
    cr = np.empty((H, W), np.uint8)
    lib().or_rgb_to_ycbcr(_ptr(rgb), W, H, 3 * W, _ptr(y), _ptr(cb), _ptr(cr), W)
    return y, cb, cr


# ---- learned deblocking network (deblock.c) ---------------------------------

def db_nparam() -> int:
    """Number of parameters of the 1-32-32-32-1 network (19105)."""
    return lib().or_db_nparam()


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def conv3x3(x, w, b=None):
    """3x3 cross-correlation with zero padding: x (Ci, H, W), w (Co, Ci, 3, 3), b (Co,) -> (Co, H, W)."""
    x, w = _f64(x), _f64(w)
    ci, H, W = x.shape
    co = w.shape[0]
    y = np.empty((co, H, W), np.float64)
    bb = None if b is None else _f64(b)
    lib().or_conv3x3(x, ci, H, W, w, None if bb is None else bb.ctypes.data, co, y)
    return y


def conv3x3_bwd(x, w, gy):
    """(gx, gw, gb) of a conv layer given dL/dy."""
    x, w, gy = _f64(x), _f64(w), _f64(gy)
    ci, H, W = x.shape
    co = w.shape[0]
    gx = np.empty_like(x)
    gw = np.zeros_like(w)
    gb = np.zeros(co, np.float64)
    lib().or_conv3x3_bwd(x, ci, H, W, w, co, gy, gx.ctypes.data, gw.ctypes.data, gb.ctypes.data)
    return gx, gw, gb


def db_forward(params, x):
    """(y, acts) of the network on one image x (H, W) in [0, 1]; acts (3, 32, H, W)."""
    params, x = _f64(params), _f64(x)
    H, W = x.shape
    y = np.empty((H, W), np.float64)
    acts = np.empty((3, 32, H, W), np.float64)
    lib().or_db_forward(params, x, H, W, y, acts.ctypes.data)
    return y, acts


def db_loss_grad(params, x, t, want_grad: bool = True):
    """(loss, grad) of a batch x, t (B, H, W): mean squared error and its gradient."""
    params, x, t = _f64(params), _f64(x), _f64(t)
    B, H, W = x.shape
    grad = np.empty(db_nparam(), np.float64) if want_grad else None
    loss = lib().or_db_loss_grad(params, x, t, B, H, W, None if grad is None else grad.ctypes.data)
    return loss, grad


def adam_step(p, m, v, g, lr, b1=0.9, b2=0.999, eps=1e-8, step=1):
    """One Adam step, in place on the float64 arrays p, m, v."""
    for a in (p, m, v):
        if a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"]:
            raise TypeError("p, m, v must be contiguous float64 arrays")
    g = _f64(g)
    lib().or_adam_step(p, m, v, g, p.size, lr, b1, b2, eps, step)
