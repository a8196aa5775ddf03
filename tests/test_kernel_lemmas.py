"""The exact rewrites the fused kernel relies on, checked on the CPU.

Each rewrite must give the same bits as the recipe as written; the GPU parity
tests then check the kernels themselves.

* The level shift (p - 128) 2^F changes only the DC coefficient, by 2^(F+13).
* Adding a constant K to every output of the inverse equals adding K to the
  dequantized DC coefficient (so the reconstruction's rounding offset and +128
  fold into one add).
* The quantizer's division m / Q (m < 2^14) equals trunc(float32(m) * r) with
  r the smallest float32 >= 1/Q, for every table entry of every qs.
* For F > 12 the quantizer pre-shifts: floor((|c| + Q 2^(F+2)) / 2^(F+3)) =
  floor((floor(|c| / 2^s) + Q 2^(F+2-s)) / 2^(F+3-s)), s = F - 12, and the sum
  stays below 2^32.
* No coefficient of a uint8 block reaches the dequantization clamp.
* The gain compensation (v M + 2^14) >> 15 is the high word of
  (v 2^k)(M 2^(17-k)) + 2^31, and v 2^k fits int32 at every compensated value:
  bounded through the flow graph as affine forms of the block's inputs plus the
  truncation errors of every shift and compensation.

Each lemma is checked for every recipe R(n, F, G) the library is built with.
"""
import numpy as np
import pytest
import scipy.fft as sf

F = 12
RECIPES = [(n, F_, G_) for n in (4, 6, 8, 10, 12) for F_, G_ in ((8, 8), (12, 12), (16, 12))]


def test_level_shift_lands_on_dc_only(oracle_mod):
    rng = np.random.default_rng(31)
    for _ in range(200):
        p = rng.integers(0, 256, 64, dtype=np.int64)
        with_shift, _ = oracle_mod.cordic_forward_block((p - 128) << F)
        without, _ = oracle_mod.cordic_forward_block(p << F)
        diff = (without - with_shift).reshape(64)
        assert diff[0] == 64 * 128 * (1 << F) == 1 << 25
        assert not np.any(diff[1:])


@pytest.mark.parametrize("n,Fr,Gr", RECIPES)
def test_dc_folds_every_recipe(oracle_mod, n, Fr, Gr):
    rng = np.random.default_rng(33)
    K = (1 << (Gr + 2)) + (128 << (Gr + 3))
    for _ in range(40):
        p = rng.integers(0, 256, 64, dtype=np.int64)
        a, _ = oracle_mod.recipe_forward_block(n, Fr, Gr, (p - 128) << Fr)
        b, pk = oracle_mod.recipe_forward_block(n, Fr, Gr, p << Fr)
        diff = (b - a).reshape(64)
        assert diff[0] == 1 << (Fr + 13) and not np.any(diff[1:])
        assert pk < 2 ** 31   # the unshifted transform also fits int32
        d = rng.integers(-2048, 2048, 64, dtype=np.int64) << Gr
        x, _ = oracle_mod.recipe_inverse_block(n, Fr, Gr, d)
        d[0] += K
        x2, _ = oracle_mod.recipe_inverse_block(n, Fr, Gr, d)
        assert np.array_equal(x2 - x, np.full((8, 8), K))


def test_unshifted_transform_peak_bound():
    # the DC path of an all-255 block holds 64 * 255 * 2^F < 2^(F+14), below 2^31 for F <= 16;
    # every other path sees differences of pixels, as in the level-shifted transform
    assert 64 * 255 * (1 << 16) < 2 ** 31


def test_quantizer_preshift_identity():
    rng = np.random.default_rng(34)
    Qs = sorted({1 + (1 + s) * qs for qs in range(1, 1025) for s in range(15)})
    Fr = 16
    s = Fr - 12
    amax = (1026 << (Fr + 3))          # |c| / 2^(F+3) <= 1024 + recipe error (< 2)
    a = np.concatenate([rng.integers(0, amax, 4000, dtype=np.int64),
                        np.arange(0, 1 << 12, dtype=np.int64), np.array([amax])])
    for Q in Qs[::7] + [Qs[-1]]:
        direct = (a + (Q << (Fr + 2))) >> (Fr + 3)
        pre = ((a >> s) + (Q << (Fr + 2 - s))) >> (Fr + 3 - s)
        assert np.array_equal(direct, pre), Q
    # the 32-bit sums: pre-shifted for F = 16, direct for F <= 12
    Qmax = Qs[-1]
    assert (amax >> s) + (Qmax << (Fr + 2 - s)) < 2 ** 32
    assert (1026 << 15) + (Qmax << 14) < 2 ** 31


def test_output_offset_folds_into_dc(oracle_mod):
    rng = np.random.default_rng(32)
    K = (1 << (F + 2)) + (128 << (F + 3))
    for _ in range(200):
        d = (rng.integers(-2048, 2048, 64, dtype=np.int64)) << F
        x, _ = oracle_mod.cordic_inverse_block(d)
        d2 = d.copy()
        d2[0] += K
        x2, _ = oracle_mod.cordic_inverse_block(d2)
        assert np.array_equal(x2 - x, np.full((8, 8), K))


def test_float_reciprocal_division_exact():
    m = np.arange(1 << 14, dtype=np.int64)
    mf = m.astype(np.float32)
    Qs = sorted({1 + (1 + s) * qs for qs in range(1, 1025) for s in range(15)})
    for Q in Qs:
        r = np.float32(1.0 / Q)
        if float(r) < 1.0 / Q:
            r = np.nextafter(r, np.float32(np.inf))
        prod = (mf * r).astype(np.float32)          # IEEE binary32, round to nearest even
        q = np.trunc(prod).astype(np.int64)
        assert np.array_equal(q, m // Q), Q
        # the dequantized value q Q 2^G is exact in float32 for q Q <= 2047, G <= 12
        keep = (m // Q) * Q <= 2047
        for G in (8, 12):
            d = (np.trunc(prod) * np.float32(Q * (1 << G))).astype(np.float32)
            assert np.array_equal(d.astype(np.int64)[keep], ((m // Q) * Q * (1 << G))[keep]), Q


def test_quantizer_magnitude_stays_below_2_14(oracle_mod):
    # m = (|c| + Q 2^(F+2)) >> (F+3) < 2^14 for every coefficient of a uint8 block
    # and every Q the library accepts: |c| / 2^15 <= 1024 + the recipe's error (< 2)
    # and Q / 2 <= (1 + 15 * 1024) / 2
    Qmax = 1 + 15 * 1024
    assert ((1026 << 15) + (Qmax << 14)) >> 15 < (1 << 14)


def test_dequantization_clamp_never_binds(oracle_mod):
    # |F_uv| <= max over pixels in [-128, 127] of the basis response, plus the
    # recipe's coefficient error (< 1.75, pinned in the recipe tests); DC is exact
    # and lies in [-1024, 1016].  q = round(F / Q) then gives |q Q| <= 2047.
    C8 = sf.dct(np.eye(8), type=2, norm="ortho", axis=0)
    C64 = np.kron(C8, C8)
    P = np.where(C64 > 0, C64, 0).sum(axis=1)
    N = -np.where(C64 < 0, C64, 0).sum(axis=1)
    B = np.maximum(127 * P + 128 * N, 128 * P + 127 * N) + 1.75
    worst = 0.0
    for qs in range(1, 1025):
        for k in range(1, 64):
            u, v = divmod(k, 8)
            Q = 1 + (1 + u + v) * qs
            worst = max(worst, np.floor(B[k] / Q + 0.5) * Q)
        Q = 1 + qs
        assert np.floor(1016 / Q + 0.5) * Q <= 2047
        assert np.floor(1024 / Q + 0.5) * Q <= 2048
    assert worst <= 2047
    # every recipe of the family: bound each coefficient by its effective matrix row
    # (the recipe's linear part) plus the 80 LSB truncation allowance
    for n, Fr, Gr in RECIPES:
        M = np.zeros((64, 64))
        for k in range(64):
            e = np.zeros(64, np.int64)
            e[k] = 2 ** 36
            out, _ = oracle_mod.recipe_forward_block(n, Fr, Gr, e)
            M[:, k] = out.reshape(64) / 2 ** 36 / 8
        Pp = np.where(M > 0, M, 0).sum(axis=1)
        Nn = -np.where(M < 0, M, 0).sum(axis=1)
        Bk = np.maximum(127 * Pp + 128 * Nn, 128 * Pp + 127 * Nn) + 80 * 2.0 ** -Fr
        for qs in (1, 2, 3, 5, 7, 11, 64, 333, 1024):
            for k in range(1, 64):
                u, v = divmod(k, 8)
                Q = 1 + (1 + u + v) * qs
                assert np.floor(Bk[k] / Q + 0.5) * Q <= 2047, (n, Fr, Gr, qs, k)
    # the DC of the recipe is exact: constant blocks give 8 (c - 128) exactly
    img = np.zeros((8, 16), np.uint8)
    img[:, 8:] = 255
    c = oracle_mod.cordic_forward(img)
    assert c[0, 0] == -1024 << 15 and c[1, 0] == 1016 << 15


# ---------------------------------------------------------------------------
# The gain compensation as the high word of one 64-bit multiply-add
# ---------------------------------------------------------------------------

def _family_multipliers(oracle_mod):
    Ms = set()
    for n in (4, 6, 8, 10, 12):
        _, gains = oracle_mod.recipe_tables_n(n)
        Ms.update(int(g) for g in gains)
    return sorted(Ms)


def _high_word_form(v, M):
    k = 1 if M < 2 ** 15 else 2
    vs = v << k
    assert np.all((vs >= -2 ** 31) & (vs < 2 ** 31))   # int32
    return (vs * (M << (17 - k)) + 2 ** 31) >> 32


def test_compensation_high_word_identity(oracle_mod):
    # (v M + 2^14) >> 15 = ((v 2^k) (M 2^(17-k)) + 2^31) >> 32 for every multiplier of the
    # family, with both factors in int32
    rng = np.random.default_rng(35)
    for M in _family_multipliers(oracle_mod):
        k = 1 if M < 2 ** 15 else 2
        assert 0 < M < 2 ** 16 and M << (17 - k) < 2 ** 31
        lim = 2 ** (31 - k)
        v = np.concatenate([rng.integers(-lim, lim, 200000, dtype=np.int64),
                            np.arange(-70000, 70000, dtype=np.int64),
                            np.arange(lim - 70000, lim, dtype=np.int64),
                            np.arange(-lim, -lim + 70000, dtype=np.int64)])
        direct = (v * M + 2 ** 14) >> 15
        assert np.array_equal(_high_word_form(v, M), direct), M
    # the planted mistake of a missing rounding term is caught
    v = np.arange(-5000, 5000, dtype=np.int64)
    assert not np.array_equal((v * 19898) >> 15, (v * 19898 + 2 ** 14) >> 15)


class _Form:
    """An affine form over the 64 inputs of a block plus a truncation error:
    value = vec . inputs + const + e with |e| <= err."""

    def __init__(self, vec, const=0.0, err=0.0):
        self.vec, self.const, self.err = vec, const, err

    def __add__(self, o):
        return _Form(self.vec + o.vec, self.const + o.const, self.err + o.err)

    def __sub__(self, o):
        return _Form(self.vec - o.vec, self.const - o.const, self.err + o.err)

    def shr(self, i):   # floor(v / 2^i): v / 2^i minus less than 1
        return self if i == 0 else _Form(self.vec / 2 ** i, self.const / 2 ** i, self.err / 2 ** i + 1.0)

    def comp(self, M):  # (v M + 2^14) >> 15: v M / 2^15 within 1/2
        return _Form(self.vec * M / 2 ** 15, self.const * M / 2 ** 15, self.err * M / 2 ** 15 + 0.5)


def _compensation_peaks(oracle_mod, n, Fr, Gr):
    """Largest |v| 2^k over every compensated value of the forward transform of a
    uint8 block and of the inverse of any block of dequantized values in
    [-2048, 2048] 2^G plus the DC fold, for recipe R(n, F, G)."""
    dirs, gains = oracle_mod.recipe_tables_n(n)
    peaks = []

    def bound_fwd(f):   # inputs p in [0, 255]
        pos, neg = f.vec[f.vec > 0].sum(), f.vec[f.vec < 0].sum()
        return max(abs(f.const + 255 * pos), abs(f.const + 255 * neg)) + f.err

    def bound_inv(f):   # inputs d in [-2048, 2048]
        return abs(f.const) + 2048 * np.abs(f.vec).sum() + f.err

    def comp(f, M, bound):
        peaks.append((bound(f) * 2 ** (1 if M < 2 ** 15 else 2), bound is bound_fwd))
        return f.comp(M)

    def rotate(a, b, R, S):
        for i in range(n):
            sa, sb = a.shr(i), b.shr(i)
            a, b = (a + sb, b - sa) if S * dirs[R][i] > 0 else (a - sb, b + sa)
        return a, b

    def forward_line(v, bd):   # the four stages of Sec. 2.5.2
        s = [v[i] + v[7 - i] for i in range(4)]
        d = [v[i] - v[7 - i] for i in range(4)]
        e0, e1, e2, e3 = s[0] + s[3], s[1] + s[2], s[1] - s[2], s[0] - s[3]
        a3, b3 = rotate(d[3], d[0], 1, 1)
        a1, b1 = rotate(d[2], d[1], 0, 1)
        a6, b6 = rotate(e2, e3, 2, 1)
        a1, b1, a3, b3 = (comp(a1, gains[0], bd), comp(b1, gains[0], bd),
                          comp(a3, gains[1], bd), comp(b3, gains[1], bd))
        a6, b6 = comp(a6, gains[2], bd), comp(b6, gains[2], bd)
        v4, v7, v6, v5 = a3 + b1, b3 + a1, a3 - b1, b3 - a1
        return [e0 + e1, v7 + v4, a6, comp(v5, gains[3], bd), e0 - e1, comp(v6, gains[3], bd), b6, v7 - v4]

    def inverse_line(z, bd):   # the transposed graph
        v5, v6 = comp(z[3], gains[3], bd), comp(z[5], gains[3], bd)
        v7, v4 = z[1] + z[7], z[1] - z[7]
        e0, e1 = z[0] + z[4], z[0] - z[4]
        a3, b3 = rotate(v4 + v6, v7 + v5, 1, -1)
        a1, b1 = rotate(v7 - v5, v4 - v6, 0, -1)
        a6, b6 = rotate(z[2], z[6], 2, -1)
        a1, b1, a3, b3 = (comp(a1, gains[0], bd), comp(b1, gains[0], bd),
                          comp(a3, gains[1], bd), comp(b3, gains[1], bd))
        a6, b6 = comp(a6, gains[2], bd), comp(b6, gains[2], bd)
        s0, s3, s1, s2 = e0 + b6, e0 - b6, e1 + a6, e1 - a6
        return [s0 + b3, s1 + b1, s2 + a1, s3 + a3, s3 - a3, s2 - a1, s1 - b1, s0 - b3]

    def two_passes(x, line, bd, order):
        for rows in order:
            for L in range(8):
                idx = [L * 8 + k for k in range(8)] if rows else [k * 8 + L for k in range(8)]
                for i, o in zip(idx, line([x[i] for i in idx], bd)):
                    x[i] = o

    eye = np.eye(64)
    two_passes([_Form(eye[i] * 2 ** Fr) for i in range(64)], forward_line, bound_fwd, (True, False))
    x = [_Form(eye[i] * 2 ** Gr) for i in range(64)]
    x[0].const = 2 ** (Gr + 2) + 2 ** (Gr + 10)
    two_passes(x, inverse_line, bound_inv, (False, True))
    fwd = max(p for p, is_fwd in peaks if is_fwd)
    inv = max(p for p, is_fwd in peaks if not is_fwd)
    return fwd, inv, len(peaks)


@pytest.mark.parametrize("n,Fr,Gr", RECIPES)
def test_compensation_headroom_every_recipe(oracle_mod, n, Fr, Gr):
    fwd, inv, sites = _compensation_peaks(oracle_mod, n, Fr, Gr)
    assert sites == 256   # 2 passes x 8 lines x 8 compensations, forward and inverse
    assert fwd < 2 ** 30.5 and inv < 2 ** 29.6, (np.log2(fwd), np.log2(inv))


def test_compensation_headroom_margin_is_under_one_bit(oracle_mod):
    # for F = 16 the forward bound lies between 2^30 and 2^31: the pre-shift of one bit
    # fits, a second would not, so the shift is k = 1 below M = 2^15 and no more
    fwd, inv, _ = _compensation_peaks(oracle_mod, 10, 16, 12)
    assert 2 ** 30 < fwd < 2 ** 31
    fwd12, _, _ = _compensation_peaks(oracle_mod, 10, 12, 12)
    assert abs(np.log2(fwd) - np.log2(fwd12) - 4) < 1e-6   # linear in 2^F
