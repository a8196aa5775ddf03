"""Pins of the recipe family R(n, F, G) of the oracle (O7 with its parameters free).

n CORDIC micro-rotations per rotation block, F fractional bits in the forward
transform, G in the inverse, P = 15 bits in the gain constants.  The sweep is
n in {4, 6, 8, 10, 12} with (F, G) in {(8, 8), (12, 12), (16, 12)}; G stops at 12
because the inverse's worst case needs 2^(G + 16.9) < 2^31.  The pins hold for
every member without the oracle checking itself:

* the directions and gains, read as complex products, rotate by the Loeffler
  angles within the greedy CORDIC residual, and the gains undo K_n;
* the effective 2-D matrix moves from the exact DCT by no more than the
  residual angles and gain errors allow;
* every coefficient obeys the L1 error bound of its matrix row plus the
  truncation of the floors (80 LSB of 2^-F);
* constant blocks, DC-only inverses and constant-image codecs are exact (closed
  forms that do not depend on the recipe);
* worst-case blocks keep every stored value inside int32;
* R(10, 12, 12) is the default recipe, bit for bit.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.fft as sf

THETAS = (math.pi / 16, 3 * math.pi / 16, 6 * math.pi / 16)
C8 = sf.dct(np.eye(8), type=2, norm="ortho", axis=0)
C64 = np.kron(C8, C8)
NS = (4, 6, 8, 10, 12)
FG = ((8, 8), (12, 12), (16, 12))
RECIPES = [(n, F, G) for n in NS for F, G in FG]
P = 15


def _residuals(oracle_mod, n):
    d, g = oracle_mod.recipe_tables_n(n)
    prods = [np.prod([complex(1.0, -d[r, i] * 2.0 ** -i) for i in range(n)]) for r in range(3)]
    return d, g, prods


@pytest.mark.parametrize("n", NS)
def test_tables_rotate_by_loeffler_angles(oracle_mod, n):
    d, g, prods = _residuals(oracle_mod, n)
    assert set(np.unique(d)) <= {-1, 1}
    k = (1.0, 1.0, math.sqrt(2.0))
    for r, theta in enumerate(THETAS):
        assert abs(np.angle(prods[r]) + theta) <= math.atan(2.0 ** -(n - 1))
        assert abs(g[r] * abs(prods[r]) / 2 ** P - k[r]) <= 0.5 * abs(prods[r]) / 2 ** P
    assert g[3] == round(math.sqrt(2.0) * 2 ** P)


def _matrix(oracle_mod, fn, n, F, G, scale=2 ** 36):
    M = np.zeros((64, 64))
    for k in range(64):
        x = np.zeros(64, np.int64)
        x[k] = scale
        out, _ = fn(n, F, G, x)
        M[:, k] = out.reshape(64) / scale
    return M / 8


@pytest.mark.parametrize("n", NS)
def test_effective_matrix_within_residual(oracle_mod, n):
    # A rotation by theta + delta with gain (1 + eps) moves each output by at most
    # (|delta| + |eps|) |(a, b)|; through both passes of the orthonormal-scaled
    # graph this moves each matrix entry by at most 2 (delta + eps).
    _, g, prods = _residuals(oracle_mod, n)
    k = (1.0, 1.0, math.sqrt(2.0))
    delta = max(abs(np.angle(prods[r]) + THETAS[r]) for r in range(3))
    eps = max(abs(g[r] * abs(prods[r]) / 2 ** P / k[r] - 1) for r in range(3)) + 2.0 ** -P
    A = _matrix(oracle_mod, oracle_mod.recipe_forward_block, n, 12, 12)
    B = _matrix(oracle_mod, oracle_mod.recipe_inverse_block, n, 12, 12)
    assert np.abs(A - C64).max() <= 2 * (delta + eps)
    assert np.abs(B - C64.T).max() <= 2 * (delta + eps)


@pytest.mark.parametrize("n,F,G", RECIPES)
def test_forward_error_bound(oracle_mod, n, F, G):
    A = _matrix(oracle_mod, oracle_mod.recipe_forward_block, n, F, G)
    bound = 128 * np.abs(A - C64).sum(axis=1) + 80 * 2.0 ** -F
    rng = np.random.default_rng(6)
    blocks = [rng.integers(0, 256, (8, 8), dtype=np.uint8) for _ in range(120)]
    blocks += [np.where(C64[k] > 0, 255, 0).astype(np.uint8).reshape(8, 8) for k in range(64)]
    blocks += [np.where(A[k] - C64[k] > 0, 255, 0).astype(np.uint8).reshape(8, 8) for k in range(64)]
    img = np.ascontiguousarray(np.concatenate(blocks, axis=1))
    exact = oracle_mod.exact_forward(img)
    for b, blk in enumerate(blocks):
        c, _ = oracle_mod.recipe_forward_block(n, F, G, (blk.astype(np.int64) - 128) * 2 ** F)
        assert np.all(np.abs(c.reshape(64) / 2 ** (F + 3) - exact[b]) <= bound)


@pytest.mark.parametrize("n,F,G", RECIPES)
def test_constant_blocks_and_dc_inverse_exact(oracle_mod, n, F, G):
    for c in (0, 1, 37, 128, 200, 255):
        x = np.full(64, (c - 128) * 2 ** F, np.int64)
        out, _ = oracle_mod.recipe_forward_block(n, F, G, x)
        out = out.reshape(64)
        # every row pass gives 8 (c - 128) 2^F at index 0; the column pass 64 (c - 128) 2^F
        assert out[0] == 64 * (c - 128) * 2 ** F
        assert not np.any(out[1:])
    for D in range(-2048, 2048, 61):
        d = np.zeros(64, np.int64)
        d[0] = D * 2 ** G
        x, _ = oracle_mod.recipe_inverse_block(n, F, G, d)
        assert np.all(x == D * 2 ** G)


@pytest.mark.parametrize("n,F,G", RECIPES)
def test_constant_image_codec_closed_form(oracle_mod, n, F, G):
    for qs in (1, 4, 16):
        Q00 = 1 + qs
        for c in range(0, 256, 3):
            rec, s = oracle_mod.recipe_codec(n, F, G, np.full((8, 8), c, np.uint8), qs)
            r = Fraction(8 * (c - 128), Q00)
            mag = math.floor(abs(r) + Fraction(1, 2))
            q = mag if r >= 0 else -mag
            p = math.floor(Fraction(max(-2048, min(2047, q * Q00)), 8) + Fraction(1, 2)) + 128
            p = min(255, max(0, p))
            assert np.all(rec == p) and s == 64 * (p - c) ** 2


@pytest.mark.parametrize("n,F,G", RECIPES)
def test_int32_headroom(oracle_mod, n, F, G):
    fwd = [np.where(s * C64[k] > 0, 255, 0).astype(np.int64).reshape(64) for k in range(64) for s in (1, -1)]
    worst_f = max(oracle_mod.recipe_forward_block(n, F, G, (b - 128) * 2 ** F)[1] for b in fwd)
    assert worst_f < 2 ** 31
    worst_i = 0
    for k in range(64):
        for s in (1, -1):
            d = (np.where(s * C64.T[k] > 0, 2047, -2048) * 2 ** G).astype(np.int64)
            worst_i = max(worst_i, oracle_mod.recipe_inverse_block(n, F, G, d)[1])
    assert worst_i < 2 ** 31


def test_default_recipe_is_r10_12_12(oracle_mod):
    from paper_1306_1373_amd.synth import synth_image
    img = synth_image(200, 136, seed=9, sigma=6.0)
    rec_d, s_d, q_d = oracle_mod.cordic_codec(img, 4, want_q=True)
    rec_r, s_r, q_r = oracle_mod.recipe_codec(10, 12, 12, img, 4, want_q=True)
    assert s_d == s_r and np.array_equal(rec_d, rec_r) and np.array_equal(q_d, q_r)


def test_psnr_against_exact_codec(oracle_mod):
    # n >= 8 stays within 0.01 dB of the exact FP64 codec at every F; fewer
    # micro-rotations cost PSNR, and n = 4 costs more than n = 6
    from paper_1306_1373_amd.synth import synth_image
    img = synth_image(256, 256, seed=1, sigma=5.0)
    p_ex = oracle_mod.psnr(img, oracle_mod.exact_codec(img, 4))
    loss = {}
    for n, F, G in RECIPES:
        _, s = oracle_mod.recipe_codec(n, F, G, img, 4)
        loss[(n, F, G)] = p_ex - oracle_mod.psnr_from_sse(s, 256, 256)
    for (n, F, G), v in loss.items():
        if n >= 8:
            assert abs(v) < 0.01, (n, F, G, v)
    for F, G in FG:
        assert loss[(4, F, G)] > loss[(6, F, G)] > 0.01


def test_invalid_recipes_rejected(oracle_mod):
    for bad in ((0, 12, 12), (17, 12, 12), (10, 0, 12), (10, 17, 12), (10, 12, 13)):
        with pytest.raises(ValueError):
            oracle_mod.recipe_codec(*bad, np.zeros((8, 8), np.uint8), 4)
