"""Rounding bounds of the floating-point forms of the codec (test
infrastructure), and the block-by-block check of a form's reconstruction
against the FP64 codec.  See test_gpu_float_forms.py for the derivation.
"""
import numpy as np
import scipy.fft as sf

C8 = sf.dct(np.eye(8), type=2, norm="ortho", axis=0)
K = np.kron(C8, C8)   # K[j][k], j = 8u + v, k = 8i + jj


def bf16_round(x):
    """Round float64 values to the nearest bfloat16 (8 significant bits, ties to even)."""
    m, e = np.frexp(x)                 # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(m * 256.0) / 256.0, e)


K_HAT = {"f16": np.float16(K).astype(np.float64), "bf16": bf16_round(K)}
OPERAND = {"f16": lambda v: np.float16(v).astype(np.float64), "bf16": bf16_round}
U = 2.0 ** -24


def gamma(m):
    return m * U / (1.0 - m * U)


def loeffler_abs(inverse=False):
    """8 x 8 matrix of the Loeffler flow graph (forward, or its transpose for the
    inverse) with every constant replaced by its magnitude and every subtraction
    by an addition: the factor that bounds the graph's rounding errors."""
    c1, s1 = np.cos(np.pi / 16), np.sin(np.pi / 16)
    c3, s3 = np.cos(3 * np.pi / 16), np.sin(3 * np.pi / 16)
    c6, s6 = np.sqrt(2) * np.cos(6 * np.pi / 16), np.sqrt(2) * np.sin(6 * np.pi / 16)
    r2 = np.sqrt(2)

    def fwd(x):
        s = [x[i] + x[7 - i] for i in range(4)]
        d = s[:]
        e0, e1, e2, e3 = s[0] + s[3], s[1] + s[2], s[1] + s[2], s[0] + s[3]
        u4, u7 = c3 * d[3] + s3 * d[0], s3 * d[3] + c3 * d[0]
        u5, u6 = c1 * d[2] + s1 * d[1], s1 * d[2] + c1 * d[1]
        v4 = v6 = u4 + u6
        v7 = v5 = u7 + u5
        return [e0 + e1, v7 + v4, c6 * e2 + s6 * e3, r2 * v5, e0 + e1, r2 * v6, s6 * e2 + c6 * e3, v7 + v4]

    def inv(z):
        v7 = v4 = z[1] + z[7]
        v5, v6 = r2 * z[3], r2 * z[5]
        e0 = e1 = z[0] + z[4]
        e2, e3 = c6 * z[2] + s6 * z[6], s6 * z[2] + c6 * z[6]
        u4 = u6 = v4 + v6
        u7 = u5 = v7 + v5
        t4, t7 = c3 * u4 + s3 * u7, s3 * u4 + c3 * u7
        t5, t6 = c1 * u5 + s1 * u6, s1 * u5 + c1 * u6
        s0 = s3_ = e0 + e3
        s1_ = s2_ = e1 + e2
        return [s0 + t7, s1_ + t6, s2_ + t5, s3_ + t4, s3_ + t4, s2_ + t5, s1_ + t6, s0 + t7]

    f = inv if inverse else fwd
    return np.array([f(list(np.eye(8)[k])) for k in range(8)]).T     # [output][input]


A_FWD = np.kron(loeffler_abs(), loeffler_abs())                 # [coefficient][pixel], x 8
A_INV = np.kron(loeffler_abs(True), loeffler_abs(True))         # [pixel][coefficient], x 8


def coef_bound(form, X):
    """Per-coefficient bound [nblocks, 64] of a form's forward transform of X = p - 128."""
    Xa = np.abs(X)
    if form == "f32":
        return gamma(14) * (Xa @ A_FWD.T) / 8.0 + 1e-9
    Kh = K_HAT[form]
    return Xa @ np.abs(Kh - K).T + gamma(64) * (Xa @ np.abs(Kh).T) + 1e-9


def pixel_bound(form, d, x):
    """Per-pixel bound [nblocks, 64] of a form's x + 128.5 from dequantized values d."""
    da = np.abs(d)
    if form == "f32":
        return gamma(14) * (da @ A_INV.T) / 8.0 + U * (np.abs(x) + 128.5) + 1e-9
    Kh = K_HAT[form]
    dh = OPERAND[form](d)
    return da @ np.abs(Kh - K) + np.abs(dh - d) @ np.abs(Kh) + gamma(65) * (128.5 + np.abs(dh) @ np.abs(Kh)) + 1e-9


def blocks_of(img):
    """[nblocks, 64] of p - 128, edge-replicated to the block grid, block-major."""
    H, W = img.shape
    Hp, Wp = -(-H // 8) * 8, -(-W // 8) * 8
    p = np.pad(img, ((0, Hp - H), (0, Wp - W)), mode="edge").astype(np.float64) - 128
    return p.reshape(Hp // 8, 8, Wp // 8, 8).transpose(0, 2, 1, 3).reshape(-1, 64)


def check_codec_blocks(oracle_mod, img, rec, form, qs):
    """Check a form's reconstruction of img block by block against the FP64 codec
    (see the module docstring); returns (blocks, blocks with a quantizer decision
    within reach of rounding, pixels within reach of a reconstruction boundary)."""
    H, W = img.shape
    bw, bh = oracle_mod.grid(W, H)
    X = blocks_of(img)
    Fx = oracle_mod.exact_forward(img)                       # [nblocks, 64]
    eF = coef_bound(form, X)
    Q = oracle_mod.qtable(qs).reshape(64).astype(np.float64)
    r = np.abs(Fx) / Q
    amb = np.abs(r - np.floor(r) - 0.5) <= eF / Q + 3.0 * U * (r + 1.0)
    q0 = np.sign(Fx) * np.floor(r + 0.5)
    # the other side of an ambiguous decision: one step towards or away from zero
    q1 = np.sign(Fx) * np.where(r - np.floor(r) >= 0.5, np.floor(r), np.floor(r) + 1.0)
    n_amb_blocks, n_px_ties = 0, 0
    for b in range(bw * bh):
        by, bx = divmod(b, bw)
        h, w = min(8, H - by * 8), min(8, W - bx * 8)
        got = rec[by * 8:by * 8 + h, bx * 8:bx * 8 + w].astype(np.float64)
        ks = np.flatnonzero(amb[b])
        n_amb_blocks += ks.size > 0
        ok = False
        # up to 4 open decisions: each combination in turn; more: the base choice
        # with every open coefficient free to move by Q (each moves pixel k by at
        # most |K_jk| Q_j), an interval that holds every combination
        combos = range(1 << ks.size) if ks.size <= 4 else [None]
        for combo in combos:
            q = q0[b].copy()
            slack = np.zeros(64)
            if combo is None:
                slack = np.abs(K[ks]).T @ Q[ks]
                dq = np.where(np.isin(np.arange(64), ks), Q, 0.0)
            else:
                dq = np.zeros(64)
                for j, k in enumerate(ks):
                    if combo >> j & 1:
                        q[k] = q1[b, k]
            d = q * Q
            x = oracle_mod.idct8x8(d.reshape(8, 8)).reshape(64)
            e = pixel_bound(form, (np.abs(d) + dq)[None], x[None])[0] + slack
            lo = np.clip(np.floor(x + 128.5 - e), 0, 255).reshape(8, 8)[:h, :w]
            hi = np.clip(np.floor(x + 128.5 + e), 0, 255).reshape(8, 8)[:h, :w]
            if np.all((got >= lo) & (got <= hi)):
                ok = True
                n_px_ties += int((lo != hi).sum())
                break
        assert ok, (form, qs, W, H, b, ks)
    return bw * bh, n_amb_blocks, n_px_ties


