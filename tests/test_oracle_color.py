"""Pins of the integer RGB -> YCbCr conversion used for three-channel inputs.

The weights are the full-range JFIF / BT.601 ones; the checks compare with the
real-valued definition and with closed forms, not with the integer formula.
"""
import numpy as np


def jfif(rgb):
    R, G, B = (rgb[..., k].astype(np.float64) for k in range(3))
    y = 0.299 * R + 0.587 * G + 0.114 * B
    cb = -0.168736 * R - 0.331264 * G + 0.5 * B + 128
    cr = 0.5 * R - 0.418688 * G - 0.081312 * B + 128
    return y, cb, cr


def test_grays_are_exact(oracle_mod):
    v = np.arange(256, dtype=np.uint8)
    rgb = np.stack([v, v, v], axis=-1)[None, :, :]
    y, cb, cr = oracle_mod.rgb_to_ycbcr(rgb)
    assert np.array_equal(y[0], v)
    assert np.all(cb == 128) and np.all(cr == 128)


def test_matches_real_valued_definition(oracle_mod):
    rng = np.random.default_rng(41)
    rgb = rng.integers(0, 256, (300, 700, 3), dtype=np.uint8)
    y, cb, cr = oracle_mod.rgb_to_ycbcr(rgb)
    for got, ref in zip((y, cb, cr), jfif(rgb)):
        ref = np.clip(ref, 0, 255)
        # round half up of the real value, up to the 2^-16 rounding of the weights
        assert np.all(np.abs(got.astype(np.float64) - ref) <= 0.5 + 3 * 255 * 0.5 / 65536 + 1e-9)


def test_primaries(oracle_mod):
    rgb = np.array([[[255, 0, 0], [0, 255, 0], [0, 0, 255], [255, 255, 255], [0, 0, 0]]], np.uint8)
    y, cb, cr = oracle_mod.rgb_to_ycbcr(rgb)
    ry, rcb, rcr = jfif(rgb)
    assert np.array_equal(y[0], np.floor(ry[0] + 0.5).astype(int))
    assert np.array_equal(cb[0], np.clip(np.floor(rcb[0] + 0.5), 0, 255).astype(int))
    assert np.array_equal(cr[0], np.clip(np.floor(rcr[0] + 0.5), 0, 255).astype(int))
