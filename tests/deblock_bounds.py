"""Error bounds of the deblocking network's GPU arithmetic against the FP64
oracle, entry by entry (test infrastructure).

The GPU kernels round the network's weights to FP16 (the oracle is given the
same rounded weights), store activations in FP16, accumulate in FP32, and may
round backward signals to FP16 (with an exact power-of-two scale) to feed the
matrix cores.  Every rounding is modelled as an independent error, uniform on
+-u |v| (variance (u v)^2 / 3) with u = 2^-24 for FP32 and 2^-11 for FP16, and
the variances are pushed through the network's linear maps with the squared
weights.  A ReLU passes its input's error where the exact pre-activation is
positive; where the pre-activation lies within its tolerance of 0 the GPU may
take the other branch, and the backward signal G there may be passed or
dropped: an error of +-G whose sign is unrelated to that of any other such
position, so it enters as variance G^2 and propagates like the rest.  The
tolerance of a value is SIGMAS standard deviations.

Errors are not independent where the computation repeats itself: two pixels
whose inputs within the reach of a quantity are equal (a flat block, the zero
fill past the edge of a plane) compute that quantity identically and carry the
same error, which then adds coherently in a sum.  So pixels are grouped by
their inputs within each quantity's reach, and every sum over taps or pixels
multiplies a term's variance by the number of terms in its group (by Cauchy-
Schwarz, (sum_k w_k e)^2 <= n sum_k w_k^2 e^2 for n terms sharing one error e).

The convolutions here are plain linear algebra over arrays shaped
(C, B, H, W): channels first, then images, rows, columns, with zero padding
outside each image.  They serve only to propagate error variances and to build
the bound; the values being checked come from oracle/deblock.c.
"""
import numpy as np

U32 = 2.0 ** -24
U16 = 2.0 ** -11
SIGMAS = 6.0
SIZES = [(32, 1), (32, 32), (32, 32), (1, 32)]   # (C_out, C_in) of the four layers


def layers(p):
    """[(W (Co, Ci, 3, 3), b (Co,))] of a flat parameter array."""
    o, out = 0, []
    for co, ci in SIZES:
        w = np.asarray(p[o:o + co * ci * 9], np.float64).reshape(co, ci, 3, 3)
        o += co * ci * 9
        out.append((w, np.asarray(p[o:o + co], np.float64)))
        o += co
    return out


def he_params(seed, nonzero_output=True):
    """Parameters for tests: He-normal hidden weights; with nonzero_output, small
    random biases and output layer too (the trained filter's shape), else zero
    ones (the untrained identity filter)."""
    rng = np.random.default_rng(seed)
    parts = []
    for co, ci in ((32, 1), (32, 32), (32, 32)):
        parts.append(rng.normal(0.0, (2.0 / (9 * ci)) ** 0.5, co * ci * 9))
        parts.append(rng.normal(0.0, 0.05, co) if nonzero_output else np.zeros(co))
    parts.append(rng.normal(0.0, 0.05, 32 * 9 + 1) if nonzero_output else np.zeros(32 * 9 + 1))
    return np.concatenate(parts).astype(np.float32)


def _pad(x):
    return np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))


def conv(x, w, b=None, mult=None):
    """y[co] = b[co] + sum_ci sum_{dy,dx} w[co, ci, dy, dx] x[ci][r + dy - 1, c + dx - 1]; with
    mult (3, 3, B, H, W), tap (dy, dx) of output pixel p is weighted by mult[dy, dx][p]."""
    ci, B, H, W = x.shape
    co = w.shape[0]
    xp = _pad(x)
    y = np.zeros((co, B * H * W), dtype=np.result_type(x, w))
    for dy in range(3):
        for dx in range(3):
            xs = np.ascontiguousarray(xp[:, :, dy:dy + H, dx:dx + W]).reshape(ci, -1)
            term = np.ascontiguousarray(w[:, :, dy, dx]) @ xs
            y += term if mult is None else term * mult[dy, dx].reshape(1, -1)
    y = y.reshape(co, B, H, W)
    if b is not None:
        y += np.asarray(b, y.dtype)[:, None, None, None]
    return y


def conv_bwd_data(g, w, mult=None):
    """The transpose of conv: gx[ci][r, c] = sum_co sum_{dy,dx} w[co, ci, dy, dx] g[co][r - dy + 1, c - dx + 1];
    with mult (3, 3, B, H, W), the term that reads neighbour (ny, nx) of pixel p is weighted by mult[ny, nx][p]."""
    co, B, H, W = g.shape
    ci = w.shape[1]
    gp = _pad(g)                       # gp[r + 1] = g[r]
    out = np.zeros((ci, B * H * W), dtype=np.result_type(g, w))
    for dy in range(3):
        for dx in range(3):
            gs = np.ascontiguousarray(gp[:, :, 2 - dy:2 - dy + H, 2 - dx:2 - dx + W]).reshape(co, -1)
            term = np.ascontiguousarray(w[:, :, dy, dx].T) @ gs
            out += term if mult is None else term * mult[2 - dy, 2 - dx].reshape(1, -1)
    return out.reshape(ci, B, H, W)


def conv_bwd_weight(g, x):
    """dW[co, ci, dy, dx] = sum over images and pixels of g[co][r, c] x[ci][r + dy - 1, c + dx - 1]."""
    co, B, H, W = g.shape
    ci = x.shape[0]
    xp = _pad(x)
    gf = g.reshape(co, -1)
    out = np.zeros((co, ci, 3, 3), dtype=np.result_type(g, x))
    for dy in range(3):
        for dx in range(3):
            xs = np.ascontiguousarray(xp[:, :, dy:dy + H, dx:dx + W]).reshape(ci, -1)
            out[:, :, dy, dx] = gf @ xs.T
    return out


def pixel_classes(x, t, rx, rt):
    """Class id (B, H, W) of every pixel: equal for pixels whose values of x within
    Chebyshev radius rx and of t within radius rt agree, positions outside the
    image counted as a value of their own.  Ids are 64-bit hashes of the
    neighbourhood; a collision can only merge two classes (a larger group, a
    larger bound)."""
    B, H, W = x.shape
    rng = np.random.default_rng(20240601)
    h = np.zeros((B, H, W), np.uint64)
    for img, r in ((x, rx), (t, rt)):
        if img is None or r < 0:
            continue
        code = np.pad(np.rint(np.asarray(img) * 255.0).astype(np.int64) + 2, ((0, 0), (r, r), (r, r)),
                      constant_values=1).astype(np.uint64)
        for dy in range(2 * r + 1):
            for dx in range(2 * r + 1):
                m = np.uint64(rng.integers(1, 2 ** 63, dtype=np.int64)) * np.uint64(2) + np.uint64(1)
                h = h * np.uint64(0x9E3779B97F4A7C15) + code[:, dy:dy + H, dx:dx + W] * m
    return h


def group_size(cls):
    """Number of pixels of the batch in each pixel's class (B, H, W)."""
    _, inv, cnt = np.unique(cls.ravel(), return_inverse=True, return_counts=True)
    return cnt[inv].reshape(cls.shape).astype(np.float64)


def neighbour_multiplicity(cls):
    """mult[ny, nx][p] (3, 3, B, H, W): how many of pixel p's nine 3 x 3 neighbours
    (positions outside the image excluded: they read exact zeros) share the class
    of neighbour (ny - 1, nx - 1)."""
    B, H, W = cls.shape
    pad = np.pad(cls.astype(np.int64), ((0, 0), (1, 1), (1, 1)), constant_values=-1)
    nb = [pad[:, dy:dy + H, dx:dx + W] for dy in range(3) for dx in range(3)]
    mult = np.zeros((3, 3, B, H, W))
    for i in range(9):
        mult[i // 3, i % 3] = sum((nb[i] == nb[j]) for j in range(9))
    return mult


class Exact:
    """The exact (FP64) quantities of one batch the bound is built from: x, the
    pre-activations z1..z4, the activations a1..a3, y, and the backward signals
    g4 = dL/dy and g_l = dL/dz_l (l = 3, 2, 1) of the mean squared error.
    x, t: (B, H, W) arrays in [0, 1]; p: the FP16-rounded parameters (float64).
    Without t only the forward quantities are formed."""

    def __init__(self, p, x, t=None):
        self.L = layers(p)
        self.x = np.asarray(x, np.float64)[None]
        self.N = self.x.size
        a = self.x
        self.z, self.a = [], [self.x]
        for l, (w, b) in enumerate(self.L):
            z = conv(a, w, b)
            self.z.append(z)
            if l < 3:
                a = np.maximum(z, 0.0)
                self.a.append(a)
        self.y = self.x + self.z[3]
        if t is None:
            return
        self.t = np.asarray(t, np.float64)[None]
        self.s = 2.0 / self.N
        self.g = [None] * 4                       # g[l] = dL/dz_{l+1}
        self.g[3] = self.s * (self.y - self.t)
        self.G = [None] * 3                       # G[l] = dL/da_{l+1} before the ReLU mask
        for l in (2, 1, 0):
            self.G[l] = conv_bwd_data(self.g[l + 1], self.L[l + 1][0])
            self.g[l] = np.where(self.z[l] > 0, self.G[l], 0.0)

    def grads(self):
        """The gradient as a flat array in parameter order (the FP64 definition)."""
        out = []
        for l in range(4):
            out.append(conv_bwd_weight(self.g[l], self.a[l]).ravel())
            out.append(self.g[l].sum(axis=(1, 2, 3)))
        return np.concatenate(out)


def forward_var(E):
    """Variances of the GPU's errors in z1..z4, a1..a3 and y (first order)."""
    var_x = 2.0 * (U32 * E.x) ** 2 / 3.0          # p * fl(1/255): two roundings
    var_in, vz, va = var_x, [], [var_x]
    for l, (w, b) in enumerate(E.L):
        K = 9 * w.shape[1] + 1
        S = conv(np.abs(E.a[l]), np.abs(w)) + np.abs(b)[:, None, None, None]
        # input a_l (a_0 = x) reaches l pixels of x: neighbours with equal inputs share their error
        mult = neighbour_multiplicity(pixel_classes(E.x[0], None, l, -1))
        v = conv(var_in, w * w, mult=mult) + K * (U32 * S) ** 2 / 3.0
        vz.append(v)
        if l < 3:
            var_in = np.where(E.z[l] > 0, v, 0.0) + (U16 * E.a[l + 1]) ** 2 / 3.0
            va.append(var_in)
    var_y = var_x + vz[3] + (U32 * E.y) ** 2 / 3.0
    return vz, va, var_y


def forward_tolerance(E):
    """Tolerance on |y_gpu - y| per pixel, shape (B, H, W)."""
    _, _, var_y = forward_var(E)
    return SIGMAS * np.sqrt(var_y[0]) + 1e-7


def gradient_tolerance(E, g16=True, depth=None):
    """Tolerance on every entry of the gradient (flat, parameter order).

    g16: the backward signals are rounded to FP16 (scaled by a power of two) before
    each product; depth: roundings a weight-gradient sum passes through (default
    the number of pixels, each at the sum's full magnitude)."""
    vz, va, var_y = forward_var(E)
    depth = E.N if depth is None else depth
    var_t = 2.0 * (U32 * E.t) ** 2 / 3.0
    vg = [None] * 4                       # variance of the GPU's dL/dz_l
    vg[3] = E.s ** 2 * (var_y + var_t) + 3.0 * (U32 * E.g[3]) ** 2 / 3.0
    # g[l] = dL/dz_{l+1} reaches 7 - l pixels of x and 3 - l of t
    gcls = [pixel_classes(E.x[0], E.t[0], 7 - l, 3 - l) for l in range(4)]
    for l in (2, 1, 0):
        w = E.L[l + 1][0]
        K = 9 * w.shape[0]
        v_op = vg[l + 1] + ((U16 * E.g[l + 1]) ** 2 / 3.0 if g16 else 0.0)
        SG = conv_bwd_data(np.abs(E.g[l + 1]), np.abs(w))
        vG = conv_bwd_data(v_op, w * w, mult=neighbour_multiplicity(gcls[l + 1])) + K * (U32 * SG) ** 2 / 3.0
        # ReLU decisions within reach of the pre-activation's rounding
        amb = np.abs(E.z[l]) <= SIGMAS * np.sqrt(vz[l]) + 2.0 ** -25
        vg[l] = np.where(E.z[l] > 0, vG, 0.0) + np.where(amb, E.G[l] ** 2 + vG, 0.0)
    out = []
    for l in range(4):
        a, va_l = E.a[l], va[l]
        # a term g[l](p) a_l(p + offset) repeats wherever p's class of g[l] (whose
        # reach covers a_l's at the neighbour) repeats
        n = group_size(gcls[l])[None]
        v_op = vg[l] + ((U16 * E.g[l]) ** 2 / 3.0 if g16 else 0.0)
        SW = conv_bwd_weight(np.abs(E.g[l]), np.abs(a))
        var_w = (conv_bwd_weight(n * v_op, a * a + va_l) + conv_bwd_weight(n * E.g[l] ** 2, va_l)
                 + depth * (U32 * SW) ** 2 / 3.0)
        Sb = np.abs(E.g[l]).sum(axis=(1, 2, 3))
        var_b = (n * v_op).sum(axis=(1, 2, 3)) + depth * (U32 * Sb) ** 2 / 3.0
        out.append(SIGMAS * np.sqrt(var_w).ravel())
        out.append(SIGMAS * np.sqrt(var_b))
    return np.concatenate(out) + 1e-30


def signal_scale(n):
    """The GPU's scale of the FP16 backward signals for a batch of n pixels:
    2^(floor(log2 n) + 8)."""
    return 2.0 ** (int(n).bit_length() - 1 + 8)


def emulate(p, x, t, g16=True, scale=None):
    """The network's forward and backward pass in the GPU's arithmetic: FP32
    products and sums (BLAS order; layer 1 on the pixel values 0..255, scaled by
    1/255 after the sum), activations stored as FP16, backward signals
    rounded to FP16 after multiplying by `scale` (default: the GPU's, from the
    batch's pixel count) when g16.  Returns (y, grad)."""
    f32, f16 = np.float32, np.float16
    L = [(w.astype(f32), b.astype(f32)) for w, b in layers(p)]
    inv = f32(1.0) / f32(255.0)
    P = (np.asarray(x, np.float64) * 255.0).round().astype(f32)[None]
    xp = P * inv
    tt = (np.asarray(t, np.float64) * 255.0).round().astype(f32)[None] * inv
    a = [xp]
    z = []
    for l, (w, b) in enumerate(L):
        if l == 0:     # the pixel values 0..255 (exact) against the weights, then 1/255 and the bias
            zz = (conv(P, w).astype(f32) * inv + b[:, None, None, None]).astype(f32)
        elif l == 3:   # the sums of the matrix cores, then the bias
            zz = (conv(a[-1], w).astype(f32) + b[:, None, None, None]).astype(f32)
        else:
            zz = conv(a[-1], w, b).astype(f32)
        z.append(zz)
        if l < 3:
            a.append(np.maximum(zz, f32(0)).astype(f16).astype(f32))
    y = (xp + z[3]).astype(f32)
    N = y.size
    if scale is None:
        scale = signal_scale(N)
    g = [None] * 4
    g[3] = (f32(2.0 / N) * (y - tt)).astype(f32)

    def op(v):
        return (v * f32(scale)).astype(f16).astype(f32) / f32(scale) if g16 else v

    for l in (2, 1, 0):
        G = conv_bwd_data(op(g[l + 1]), L[l + 1][0]).astype(f32)
        g[l] = np.where(a[l + 1] > 0, G, f32(0)).astype(f32)
    out = []
    for l in range(4):
        out.append(conv_bwd_weight(op(g[l]), a[l]).astype(np.float64).ravel())
        out.append(op(g[l]).astype(np.float64).sum(axis=(1, 2, 3)))
    return y[0].astype(np.float64), np.concatenate(out)
