"""Mutation check of the oracle's pins.

Each case plants one plausible mistake in a private copy of ``bm_oracle.c``
(on the CPU, in a temporary directory), builds it, and requires that at least
one of the quick pins of ``test_oracle_pins`` fails against the broken copy.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import importlib
oracle_build = importlib.import_module("oracle.buildlib")

import test_oracle_pins as pins

MUTANTS = {
    "non_strict_ball": ("if (sx < e2) s->local[t][c++]", "if (sx <= e2) s->local[t][c++]"),
    "dropped_first_coordinate": ("    for (int32_t k = 0; k < d; ++k) {\n        double t = a[k] - b[k];",
                                 "    for (int32_t k = 1; k < d; ++k) {\n        double t = a[k] - b[k];"),
    "wrong_sign": ("double t = a[k] - b[k];", "double t = a[k] + b[k];"),
    "ignores_covered": ("if (covered[p]) continue;", "if (0 && covered[p]) continue;"),
    "rows_only_new_points": ("if (sx < e2) s->local[t][c++] = (int32_t)x;",
                             "if (sx < e2 && !(covered && covered[x])) s->local[t][c++] = (int32_t)x;"),
    "edges_both_directions": ("if (j > i && mark[j] != (int32_t)i)", "if (j != i && mark[j] != (int32_t)i)"),
    "early_exit_returns_zero": ("if (acc >= stop) return acc;", "if (acc >= stop) return 0.0;"),
    "ignores_order": ("int64_t p = order ? order[r] : r;", "int64_t p = r;"),
    "knn_skips_self": ("kdist[i] = sqrt(row[k - 1]);", "kdist[i] = sqrt(row[k]);"),
    "float_threshold": ("const double e2 = eps * eps;   /* RN(eps^2), computed once */",
                        "const double e2 = (float)(eps * eps);"),
    "fused_multiply_add": None,   # source unchanged, built with contraction on
    "first_member_takes_last": ("for (int64_t i = 0; i < L && f < 0; ++i)", "for (int64_t i = 0; i < L; ++i)"),
    "covering_takes_min": ("if (best > worst) worst = best;", "if (best < worst) worst = best;"),
    "separation_skips_neighbours": ("for (int64_t j = i + 1; j < L; ++j) {\n            double s2 = sqdist_w(w + (int64_t)landmarks[i] * d",
                                    "for (int64_t j = i + 2; j < L; ++j) {\n            double s2 = sqdist_w(w + (int64_t)landmarks[i] * d"),
}


def quick_pins():
    yield "line", lambda: [pins.test_hand_computed_line(dt) for dt in (np.float64, np.float32)]
    yield "bitwise", lambda: pins.test_sqdist_bitwise_equals_plain_float64(np.float64)
    yield "ties", pins.test_exact_ties_are_excluded
    yield "path", pins.test_unit_spaced_line_is_a_path
    yield "certificate", lambda: pins.test_certificate_random(1)
    yield "knn", pins.test_knn_eps_closed_form
    yield "threshold", pins.test_threshold_is_rounded_in_double
    yield "net", pins.test_net_measures_hand_computed
    yield "first", pins.test_first_member_hand_computed


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(oracle_build.SRC).read()
    flags = list(oracle_build.CFLAGS)
    mut = MUTANTS[name]
    if mut is None:
        flags = [f for f in flags if f not in ("-ffp-contract=off",)] + ["-ffp-contract=fast", "-mfma"]
    else:
        assert src.count(mut[0]) >= 1, f"mutation anchor for {name} not found"
        src = src.replace(mut[0], mut[1])
    shutil.copy(os.path.join(os.path.dirname(oracle_build.SRC), "bm_oracle.h"), tmp_path)
    (tmp_path / "m.c").write_text(src)
    so = str(tmp_path / "libm.so")
    subprocess.run(["gcc", *flags, str(tmp_path / "m.c"), "-o", so, "-lm"], check=True)
    good = oracle._load()
    oracle._lib = oracle.configure(ctypes.CDLL(so))
    failed = []
    try:
        for pin, fn in quick_pins():
            try:
                fn()
            except (AssertionError, ValueError):
                failed.append(pin)
    finally:
        oracle._lib = good
    assert failed, f"mutant {name} passed every quick pin"
