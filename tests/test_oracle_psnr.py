"""Pins of the PSNR oracle (O6), Sec. 4.1 eq. (23)-(24), against hand-worked values."""
import json
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "psnr_worked_example.json")


def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


def test_hand_worked_examples(oracle_mod):
    c = _cases()
    O = np.array(c[0]["O"], np.uint8)
    Cm = np.array(c[0]["C"], np.uint8)
    assert oracle_mod.sse(O, Cm) == c[0]["sse"]
    assert oracle_mod.psnr(O, Cm) == c[0]["psnr_peak255"]  # same double, no tolerance needed
    O3 = np.array(c[2]["O"], np.uint8)
    C3 = np.array(c[2]["C"], np.uint8)
    assert oracle_mod.sse(O3, C3) == c[2]["sse"]
    assert abs(oracle_mod.psnr(O3, C3, peak=0) - c[2]["psnr_peak_max_of_O"]) < 1e-12


def test_off_by_one_everywhere(oracle_mod):
    rng = np.random.default_rng(0)
    O = rng.integers(0, 255, (37, 53), dtype=np.uint8)
    Cm = (O + 1).astype(np.uint8)
    assert abs(oracle_mod.psnr(O, Cm) - _cases()[1]["psnr_peak255"]) < 1e-12


def test_identical_is_infinite(oracle_mod):
    O = np.arange(64, dtype=np.uint8).reshape(8, 8)
    assert oracle_mod.sse(O, O) == 0
    assert math.isinf(oracle_mod.psnr(O, O))


def test_sse_exact_beyond_32_bits(oracle_mod):
    # 4096 x 4096 pixels off by 255: SSE = 255^2 * 2^24 > 2^32
    O = np.zeros((4096, 4096), np.uint8)
    Cm = np.full((4096, 4096), 255, np.uint8)
    assert oracle_mod.sse(O, Cm) == 255 * 255 * 4096 * 4096
    assert abs(oracle_mod.psnr(O, Cm) - 0.0) < 1e-12


def test_sse_matches_numpy(oracle_mod):
    rng = np.random.default_rng(1)
    O = rng.integers(0, 256, (123, 77), dtype=np.uint8)
    Cm = rng.integers(0, 256, (123, 77), dtype=np.uint8)
    d = O.astype(np.int64) - Cm.astype(np.int64)
    assert oracle_mod.sse(O, Cm) == int(np.sum(d * d))
