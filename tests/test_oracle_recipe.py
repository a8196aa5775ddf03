"""Pins of the integer Cordic-based Loeffler recipe R(n=10, F=12, P=15) (O7).

The paper's flow-graph figure is missing, so the recipe is a reading of
Sec. 2.5.2 (four Loeffler stages, rotations replaced by CORDIC shift-add
blocks).  What pins it here, without the oracle checking itself:

* the FP64 form of the same graph equals 2 sqrt(2) C (C = SciPy's orthonormal
  DCT-II matrix) and its transpose;
* the CORDIC directions and gains, read through complex arithmetic, rotate by
  the Loeffler angles within the CORDIC convergence bound;
* constant blocks are exact, DC-only inverses are exact;
* the recipe's effective matrix is within a derived bound of the exact DCT and
  every block's coefficients obey the error bound that follows from it;
* worst-case blocks keep every stored value inside int32;
* the quantizer, dequantizer and reconstruction obey their rounding rules,
  checked with exact rational arithmetic over their whole useful domain.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.fft as sf

N, F, P = 10, 12, 15
THETAS = (math.pi / 16, 3 * math.pi / 16, 6 * math.pi / 16)
C8 = sf.dct(np.eye(8), type=2, norm="ortho", axis=0)   # orthonormal DCT-II matrix
C64 = np.kron(C8, C8)


def test_recipe_parameters(oracle_mod):
    assert oracle_mod.recipe_info() == (N, F, P)


def test_loeffler_graph_fp64_is_scaled_dct(oracle_mod):
    # structure of the graph with exact rotations: Z = 2 sqrt(2) C x, x = (2 sqrt(2) C)^T Z
    A = np.stack([oracle_mod.loeffler_forward_f64(e) for e in np.eye(8)], axis=1)
    assert np.abs(A - 2 * math.sqrt(2) * C8).max() < 1e-12
    B = np.stack([oracle_mod.loeffler_inverse_f64(e) for e in np.eye(8)], axis=1)
    assert np.abs(B - 2 * math.sqrt(2) * C8.T).max() < 1e-12


def test_cordic_tables_rotate_by_the_loeffler_angles(oracle_mod):
    # A micro-rotation maps z = a + jb to (1 - j d_i 2^-i) z, so n of them multiply
    # by P = prod_i (1 - j d_i 2^-i); the rotation block R(a,b;theta) multiplies by
    # e^{-j theta}.  CORDIC's greedy directions leave an angle error below
    # atan(2^-(n-1)); the gain constant undoes |P| = K_n to within half an LSB of 2^P.
    dirs, gains = oracle_mod.recipe_tables()
    assert set(np.unique(dirs)) <= {-1, 1}
    k = (1.0, 1.0, math.sqrt(2.0))
    for r, theta in enumerate(THETAS):
        Pc = complex(1.0, 0.0)
        for i in range(N):
            Pc *= complex(1.0, -dirs[r, i] * 2.0 ** -i)
        assert abs(np.angle(Pc) + theta) <= math.atan(2.0 ** -(N - 1))
        assert abs(gains[r] * abs(Pc) / 2 ** P - k[r]) <= 0.5 * abs(Pc) / 2 ** P
    assert abs(gains[3] / 2 ** P - math.sqrt(2.0)) <= 0.5 / 2 ** P


def test_cordic_rotation_block_matches_rotation(oracle_mod):
    # one rotation block on large vectors: (a cos + b sin, -a sin + b cos), forward and inverse
    dirs, _ = oracle_mod.recipe_tables()
    rng = np.random.default_rng(3)
    for r, theta in enumerate(THETAS):
        resid = theta + np.angle(np.prod([complex(1, -dirs[r, i] * 2.0 ** -i) for i in range(N)]))
        scale = math.sqrt(2.0) if r == 2 else 1.0
        for _ in range(200):
            a, b = (int(v) for v in rng.integers(-(1 << 24), 1 << 24, 2))
            for sense in (1, -1):
                t = sense * theta
                ea = scale * (a * math.cos(t) + b * math.sin(t))
                eb = scale * (-a * math.sin(t) + b * math.cos(t))
                ga, gb = oracle_mod.cordic_rotate(a, b, r, sense)
                norm = math.hypot(a, b) * scale
                tol = norm * (abs(resid) + 1e-4) + 32
                assert abs(ga - ea) <= tol and abs(gb - eb) <= tol


def _effective_matrix(fn, scale=2 ** 36):
    # impulse responses at a scale where the floors are negligible
    M = np.zeros((64, 64))
    for k in range(64):
        x = np.zeros(64, np.int64)
        x[k] = scale
        out, _ = fn(x)
        M[:, k] = out.reshape(64) / scale
    return M


def test_effective_matrix_close_to_dct(oracle_mod):
    # Each 1-D pass is the Loeffler graph with angles off by the CORDIC residual
    # (< atan(2^-9) = 1.95e-3 rad) and gains off by < 2^-16 relative; every entry of
    # the orthonormal-scaled 2-D matrix moves by well under 2e-3.  A wrong
    # direction, gain, pairing or stage order moves entries by > 1e-2.
    A = _effective_matrix(oracle_mod.cordic_forward_block) / 8
    B = _effective_matrix(oracle_mod.cordic_inverse_block) / 8
    assert np.abs(A - C64).max() < 2e-3
    assert np.abs(B - C64.T).max() < 2e-3


def _forward_bound(oracle_mod):
    # |c/2^15 - F| <= max|x| * ||row_k(A/8 - C)||_1 + truncation; each of the < 200
    # floors on any path loses < 1 LSB (2^-12 pixel units), which after both passes
    # and the /8 is far below 0.02 coefficient units.
    A = _effective_matrix(oracle_mod.cordic_forward_block) / 8
    D = A - C64
    return 128 * np.abs(D).sum(axis=1) + 0.02, D


def test_forward_error_bound_random_and_adversarial(oracle_mod):
    bound, D = _forward_bound(oracle_mod)
    rng = np.random.default_rng(5)
    blocks = [rng.integers(0, 256, (8, 8), dtype=np.uint8) for _ in range(300)]
    # adversarial blocks: pixels 0 / 255 along the sign of each error row
    for k in range(64):
        blocks.append(np.where(D[k] > 0, 255, 0).astype(np.uint8).reshape(8, 8))
    # worst-case magnitude blocks: sign of each DCT basis function
    for k in range(64):
        blocks.append(np.where(C64[k] > 0, 255, 0).astype(np.uint8).reshape(8, 8))
    img = np.ascontiguousarray(np.concatenate(blocks, axis=1))
    c = oracle_mod.cordic_forward(img)
    Fx = oracle_mod.exact_forward(img)
    err = np.abs(c / 2 ** 15 - Fx)
    assert np.all(err <= bound[None, :])
    assert err.max() < 1.7


def test_forward_error_on_synthetic_image(oracle_mod):
    from paper_1306_1373_amd.synth import synth_image
    img = synth_image(512, 512, seed=0, sigma=5.0)
    bound, _ = _forward_bound(oracle_mod)
    err = np.abs(oracle_mod.cordic_forward(img) / 2 ** 15 - oracle_mod.exact_forward(img))
    assert np.all(err <= bound[None, :])
    assert err.max() < 0.5


def test_constant_blocks_are_exact(oracle_mod):
    # constant c: every row pass gives [8(c-128) 2^F, 0, ...], the column pass
    # 64 (c-128) 2^F at DC, exactly (no rotation sees a nonzero input)
    img = np.repeat(np.arange(256, dtype=np.uint8), 64).reshape(256, 8, 8)
    img = np.ascontiguousarray(img.transpose(1, 0, 2).reshape(8, 256 * 8))
    c = oracle_mod.cordic_forward(img)
    dc = (np.arange(256, dtype=np.int64) - 128) * 8 * 2 ** 15
    assert np.array_equal(c[:, 0], dc)
    assert not np.any(c[:, 1:])


def test_dc_only_inverse_is_exact(oracle_mod):
    # a DC-only block D 2^F reconstructs to the constant D 2^F after both inverse passes
    for D in range(-2048, 2048, 7):
        d = np.zeros(64, np.int64)
        d[0] = D * 2 ** F
        x, _ = oracle_mod.cordic_inverse_block(d)
        assert np.all(x == D * 2 ** F)


def test_constant_image_codec_closed_form(oracle_mod):
    # constant c, table entry Q00 = 1 + qs: q = nearest(8(c-128)/Q00) (ties away from 0),
    # reconstruction = clamp(floor(q Q00 / 8 + 1/2) + 128, 0, 255)
    for qs in (0, 1, 2, 3, 4, 8, 16, 32):
        Q00 = 1 + qs
        for c in range(256):
            img = np.full((8, 8), c, np.uint8)
            rec, s = oracle_mod.cordic_codec(img, qs)
            r = Fraction(8 * (c - 128), Q00)
            mag = math.floor(abs(r) + Fraction(1, 2))
            q = mag if r >= 0 else -mag
            dq = max(-2048, min(2047, q * Q00))
            p = math.floor(Fraction(dq, 8) + Fraction(1, 2)) + 128
            p = min(255, max(0, p))
            assert np.all(rec == p), (qs, c)
            assert s == 64 * (p - c) ** 2


def test_round_trip_with_unit_table(oracle_mod):
    # qs = 0 (Q = 1): the codec is the recipe's forward and inverse with only
    # coefficient rounding between them; compare with the exact FP64 codec.
    from paper_1306_1373_amd.synth import synth_image
    img = synth_image(256, 256, seed=2, sigma=5.0)
    rec, s = oracle_mod.cordic_codec(img, 0)
    assert oracle_mod.psnr_from_sse(s, 256, 256) > 48.0
    assert np.abs(rec.astype(int) - img.astype(int)).max() <= 3


@pytest.mark.parametrize("qs", [2, 4, 8, 16])
def test_psnr_close_to_exact_codec(oracle_mod, qs):
    # the recipe's codec sits within 0.01 dB of the exact FP64 codec on the synthetic images
    from paper_1306_1373_amd.synth import synth_image
    img = synth_image(512, 512, seed=1, sigma=5.0)
    _, s = oracle_mod.cordic_codec(img, qs)
    p_rec = oracle_mod.psnr_from_sse(s, 512, 512)
    p_ex = oracle_mod.psnr(img, oracle_mod.exact_codec(img, qs))
    assert abs(p_rec - p_ex) < 0.01


def test_no_int32_overflow_on_worst_case_blocks(oracle_mod):
    # forward: pixels 0/255 along the sign of every basis function
    blocks = [np.where(C64[k] > 0, 255, 0).astype(np.uint8).reshape(8, 8) for k in range(64)]
    blocks += [np.where(C64[k] > 0, 0, 255).astype(np.uint8).reshape(8, 8) for k in range(64)]
    img = np.ascontiguousarray(np.concatenate(blocks, axis=1))
    _, peak = oracle_mod.cordic_forward(img, return_peak=True)
    assert peak < 2 ** 31
    assert peak < 2 ** 25.3          # L1 bound 128 * 72 * 2^F
    # inverse: clamped dequantized values +-2048 along the sign of every inverse basis row
    worst = 0
    for k in range(64):
        for sgn in (1, -1):
            d = (np.where(sgn * C64.T[k] > 0, 2047, -2048) * 2 ** F).astype(np.int64)
            _, pk = oracle_mod.cordic_inverse_block(d)
            worst = max(worst, pk)
    assert worst < 2 ** 31
    # and through the image-level inverse with the most extreme int16 inputs
    q = np.full((1, 64), 32767, np.int16)
    q[0, ::2] = -32768
    _, pk = oracle_mod.cordic_inverse(q, 1024, 8, 8, return_peak=True)
    assert pk < 2 ** 31


def test_quantizer_rounding_exact(oracle_mod):
    # q = c / (Q 2^(F+3)) rounded to nearest, ties away from zero: checked with
    # Fractions on every tie point and its neighbours for every Q of several tables
    D_shift = F + 3
    for qs in (0, 1, 4, 16, 1024):
        for Q in sorted({1 + (1 + s) * qs for s in range(15)}):
            D = Q << D_shift
            for m in range(0, 40):
                for base in (m * D + D // 2, m * D):
                    for delta in (-2, -1, 0, 1, 2):
                        for sgn in (1, -1):
                            c = sgn * (base + delta)
                            r = Fraction(c, D)
                            mag = math.floor(abs(r) + Fraction(1, 2))
                            exp = mag if r >= 0 else -mag
                            assert oracle_mod.recipe_quantize(c, Q) == exp, (c, Q)


def test_quantizer_division_domain(oracle_mod):
    # over the whole range a valid coefficient can take (|c| < 2^(F+3) * 1100),
    # q equals the nearest integer for every Q of the tables used (strided sweep)
    rng = np.random.default_rng(6)
    for qs in (1, 2, 4, 8, 16, 32, 1024):
        for s in range(15):
            Q = 1 + (1 + s) * qs
            D = Q << (F + 3)
            for c in rng.integers(-(1100 << (F + 3)), 1100 << (F + 3), 400):
                r = Fraction(int(c), D)
                mag = math.floor(abs(r) + Fraction(1, 2))
                assert oracle_mod.recipe_quantize(int(c), Q) == (mag if r >= 0 else -mag)


def test_dequantizer_clamps(oracle_mod):
    assert oracle_mod.recipe_dequantize(3, 5) == 15 * 2 ** F
    assert oracle_mod.recipe_dequantize(-3, 5) == -15 * 2 ** F
    assert oracle_mod.recipe_dequantize(1000, 5) == 2047 * 2 ** F
    assert oracle_mod.recipe_dequantize(-1000, 5) == -2048 * 2 ** F
    assert oracle_mod.recipe_dequantize(32767, 15361) == 2047 * 2 ** F


def test_reconstruct_rounding(oracle_mod):
    # p = clamp(floor(x / 2^(F+3) + 1/2) + 128, 0, 255)
    S = 2 ** (F + 3)
    for k in range(-140, 140):
        for delta in (-1, 0, 1, S // 2 - 1, S // 2, S // 2 + 1):
            x = k * S + delta
            p = math.floor(Fraction(x, S) + Fraction(1, 2)) + 128
            assert oracle_mod.recipe_reconstruct(x) == min(255, max(0, p))


def test_quantize_saturates_to_int16(oracle_mod):
    # arbitrary int32 coefficients: the int16 container saturates at its limits.
    # qs = 1: Q[0][0] = 2, so c = 2^31 - 1 rounds to 32768 -> 32767 and c = -2^31
    # gives exactly -32768; Q[0][1] = 3 gives 21845 with no saturation.
    coef = np.zeros((2, 64), np.int32)
    coef[0, 0] = 2 ** 31 - 1
    coef[1, 0] = -(2 ** 31)
    coef[0, 1] = 2 ** 31 - 1
    q = oracle_mod.cordic_quantize(coef, 1)
    assert q[0, 0] == 32767 and q[1, 0] == -32768 and q[0, 1] == 21845
    assert not np.any(q[0, 2:]) and not np.any(q[1, 1:])
