"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of oracle.c (on the CPU, in a temporary
directory), runs the pin modules in a child process with the mutant loaded in
place of the real oracle, and checks that at least one pin fails.  A control
case runs the same harness on an unmodified copy, which must pass.
"""
import os
import subprocess
import sys

import pytest

from oracle import build as obuild

MUTANTS = {
    # a CORDIC direction read with the wrong sense
    "direction_sign": ("const int d = z >= 0.0 ? 1 : -1;", "const int d = z >= 0.0 ? -1 : 1;"),
    # gain compensation without the sqrt(2) of the even rotation
    "gain_k": ("const double k[3] = {1.0, 1.0, sqrt(2.0)};", "const double k[3] = {1.0, 1.0, 1.0};"),
    # odd rotation pairs swapped
    "odd_pairing": ("int64_t u4 = d3, u7 = d0, u5 = d2, u6 = d1;",
                    "int64_t u4 = d2, u7 = d1, u5 = d3, u6 = d0;"),
    # a dropped sqrt(2) on an odd output
    "dropped_sqrt2": ("Z3 = compensate(v5, R->sqrt2), Z5", "Z3 = v5, Z5"),
    # a sign flip in a butterfly of the inverse
    "inverse_butterfly": ("const int64_t v7 = Z[1] + Z[7], v4 = Z[1] - Z[7];",
                          "const int64_t v7 = Z[1] - Z[7], v4 = Z[1] + Z[7];"),
    # transposed coefficient layout
    "transposed_layout": ("for (int i = 0; i < 8; ++i) c[i * 8 + j] = t[i];",
                          "for (int i = 0; i < 8; ++i) c[j * 8 + i] = t[i];"),
    # quantizer rounding toward zero instead of to nearest
    "quantizer_truncates": ("const int64_t m = (i64_abs(c) + (Q << (F + 2))) / D;",
                            "const int64_t m = i64_abs(c) / D;"),
    # reconstruction without the rounding half
    "reconstruct_floor": ("floor_div_pow2(x + ((int64_t)1 << (G + 2)), G + 3) + 128",
                          "floor_div_pow2(x, G + 3) + 128"),
    # exact DCT with alpha indexed by position instead of frequency
    "alpha_index": ("alpha(u) * alpha(v) * s;", "alpha(0) * alpha(0) * s;"),
    # PSNR with MSE not divided by the pixel count
    "psnr_mse": ("const double mse = (double)sse / ((double)W * (double)H);",
                 "const double mse = (double)sse;"),
    # luma weights of green and blue swapped
    "ycbcr_weights": ("19595 * R + 38470 * G + 7471 * B", "19595 * R + 7471 * G + 38470 * B"),
    # the forward transform scaled by the inverse's fractional bits
    "forward_uses_G": ("((int64_t)1 << R->F);", "((int64_t)1 << R->G);"),
    # truncating shift where the recipe floors
    "truncating_shift": ("if (v % d != 0 && v < 0) q -= 1;", "(void)0;"),
}

# planted in deblock.c
DEBLOCK_MUTANTS = {
    # ReLU gradient mask dropped after the last hidden layer
    "relu_mask": ("    for (long k = 0; k < DB_C * n; ++k) g2[k] = a3[k] > 0.0 ? g2[k] : 0.0;\n", ""),
    # convolution (flipped kernel) instead of cross-correlation
    "flipped_kernel": ("s += w[((long)co * ci_n + ci) * 9 + dy * 3 + dx]",
                       "s += w[((long)co * ci_n + ci) * 9 + (2 - dy) * 3 + (2 - dx)]"),
    # the residual connection missing
    "no_residual": ("  for (long k = 0; k < n; ++k) y[k] += x[k];\n", ""),
    # Adam without bias correction
    "adam_no_bias_correction": ("const double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);",
                                "const double c1 = 1.0, c2 = 1.0;"),
    # loss gradient without the factor 2
    "loss_grad_scale": ("const double scale = 2.0 / ((double)B * n);", "const double scale = 1.0 / ((double)B * n);"),
}

PIN_MODULES = ["tests/test_oracle_exact.py", "tests/test_oracle_recipe.py", "tests/test_oracle_recipe_family.py",
               "tests/test_oracle_psnr.py", "tests/test_oracle_color.py", "tests/test_oracle_deblock.py"]


def _run_pins_with(src_text, tmp_path, deblock_text=None):
    mutated = tmp_path / "oracle_mut.c"
    mutated.write_text(src_text)
    mutated_db = tmp_path / "deblock_mut.c"
    mutated_db.write_text(deblock_text if deblock_text is not None else open(obuild.SRC_DEBLOCK).read())
    lib = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-std=c11", "-O1", "-fPIC", "-shared", str(mutated), str(mutated_db), "-o", str(lib),
                    "-lm", "-lpthread"], check=True)
    # run the pin modules in a child process with the mutant loaded in place of the oracle
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PIN_MODULES], cwd=root, env=env, capture_output=True, text=True,
                       timeout=600)
    return r


def test_harness_control_passes(tmp_path):
    r = _run_pins_with(open(obuild.SRC).read(), tmp_path)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(obuild.SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found once"
    r = _run_pins_with(src.replace(old, new), tmp_path)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name", sorted(DEBLOCK_MUTANTS))
def test_pins_catch_deblock_mutant(name, tmp_path):
    old, new = DEBLOCK_MUTANTS[name]
    src = open(obuild.SRC_DEBLOCK).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found once"
    r = _run_pins_with(open(obuild.SRC).read(), tmp_path, deblock_text=src.replace(old, new))
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
