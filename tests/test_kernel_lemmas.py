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
