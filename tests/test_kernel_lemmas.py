"""The exact rewrites the fused kernel relies on, checked on the CPU.

Each rewrite must give the same bits as the recipe as written; the GPU parity
tests then check the kernels themselves.

* The level shift (p - 128) 2^F changes only the DC coefficient, by 2^25.
* Adding a constant K to every output of the inverse equals adding K to the
  dequantized DC coefficient (so the reconstruction's rounding offset and +128
  fold into one add).
* The quantizer's division m / Q (m < 2^14) equals trunc(float32(m) * r) with
  r the smallest float32 >= 1/Q, for every table entry of every qs.
* No coefficient of a uint8 block reaches the dequantization clamp.
"""
import numpy as np
import scipy.fft as sf

F = 12


def test_level_shift_lands_on_dc_only(oracle_mod):
    rng = np.random.default_rng(31)
    for _ in range(200):
        p = rng.integers(0, 256, 64, dtype=np.int64)
        with_shift, _ = oracle_mod.cordic_forward_block((p - 128) << F)
        without, _ = oracle_mod.cordic_forward_block(p << F)
        diff = (without - with_shift).reshape(64)
        assert diff[0] == 64 * 128 * (1 << F) == 1 << 25
        assert not np.any(diff[1:])


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
        # the dequantized value q Q 2^F is exact in float32
        d = (np.trunc(prod) * np.float32(Q * (1 << F))).astype(np.float32)
        assert np.array_equal(d.astype(np.int64), (m // Q) * Q * (1 << F)), Q


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
    # the DC of the recipe is exact: constant blocks give 8 (c - 128) exactly
    img = np.zeros((8, 16), np.uint8)
    img[:, 8:] = 255
    c = oracle_mod.cordic_forward(img)
    assert c[0, 0] == -1024 << 15 and c[1, 0] == 1016 << 15
