"""The oracle's pins must catch plausible mistakes.

Each case plants one slip into a copy of the oracle's C source (on the CPU, in
a temporary directory), builds it, and runs the pin suite of test_oracle.py
against the planted copy: the suite must fail.  The committed oracle is never
modified.
"""

from __future__ import annotations

import os
import subprocess
import sys

import pytest

from oracle import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "no_clamp": ("return (v > 0.0f) ? (double)v : 0.0;", "return (double)v;"),
    "C2_for_C1": ("A += sum_abs / (dif_abs + C1);", "A += sum_abs / (dif_abs + C2);"),
    "C_for_C2": ("lisi[t] = D * A / (fmax(Sx, Sy) + C2);", "lisi[t] = D * A / (fmax(Sx, Sy) + C);"),
    "C1_for_C": ("auglisi[t] = 1.0 - P / (Sx + Sy + C);", "auglisi[t] = 1.0 - P / (Sx + Sy + C1);"),
    "min_for_max": ("lisi[t] = D * A / (fmax(Sx, Sy) + C2);", "lisi[t] = D * A / (fmin(Sx, Sy) + C2);"),
    "no_abs_diff": ("const double dif_abs = fabs(xi - yi);", "const double dif_abs = (xi - yi);"),
    "no_D": ("lisi[t] = D * A /", "lisi[t] = A /"),
    "sum_for_product": ("P += sum_abs * dif_abs;", "P += sum_abs + dif_abs;"),
    "Sx_from_y": ("Sx += xi;", "Sx += yi;"),
    "transposed_pixel": ("(ty * NT + r) * N + tx * NT + c", "(tx * NT + r) * N + ty * NT + c"),
    "tile_row_stride": ("(ty * NT + r) * N + tx * NT + c", "(ty * NT + r) * NT + tx * NT + c"),
    "transposed_output": ("const int64_t t = ty * ns + tx;", "const int64_t t = tx * ns + ty;"),
    "skip_first_column": ("for (int64_t c = 0; c < NT; ++c)", "for (int64_t c = 1; c < NT; ++c)"),
    "merge_no_n_minus_1": ("(num_a - (n - 1.0) * C)", "(num_a)"),
    "merge_n_for_n_minus_1": ("(num_a - (n - 1.0) * C)", "(num_a - n * C)"),
    "merge_C_for_C2": ("num_l += lisi_c[t] * (fmax(sx, sy) + C2);", "num_l += lisi_c[t] * (fmax(sx, sy) + C);"),
    "clamp_only_x": ("const double yi = clamp_negative(y[i]);", "const double yi = (double)y[i];"),
    "diff_for_sum": ("const double sum_abs = fabs(xi + yi);", "const double sum_abs = fabs(xi - yi);"),
    "Sy_from_x": ("Sy += yi;", "Sy += xi;"),
    "aug_sign": ("auglisi[t] = 1.0 - P / (Sx + Sy + C);", "auglisi[t] = 1.0 + P / (Sx + Sy + C);"),
    "merge_min_for_max": ("num_l += lisi_c[t] * (fmax(sx, sy) + C2);", "num_l += lisi_c[t] * (fmin(sx, sy) + C2);"),
    "merge_weight_without_C": ("num_a += aug_c[t] * (sx + sy + C);", "num_a += aug_c[t] * (sx + sy);"),
    "merge_A_from_P": ("A += sums_c[4 * t + 0];", "A += sums_c[4 * t + 1];"),
    "merge_parent_sum_for_max": ("lisi_p[p] = num_l / (fmax(Sx, Sy) + C2);", "lisi_p[p] = num_l / (Sx + Sy + C2);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", *[f for f in oracle.CFLAGS if f != "-Werror"], str(mut), "-o",
                    str(lib), "-lm"], check=True, capture_output=True)
    env = dict(os.environ, IQA_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle.py"),
                          "-k", "not thread_count"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert res.returncode != 0, f"mutant {name} survived the pin suite:\n{res.stdout[-2000:]}"
