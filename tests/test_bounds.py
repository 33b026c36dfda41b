"""The deterministic error bounds of the low-precision paths, checked on the CPU.

The MFMA paths compute G = -RN32(|a|^2)/2 + sum_k P_k Q_k with 16-bit operands
and FP32 accumulation; the library claims |G - h| <= alpha |a|^2 + beta |x|^2 +
abs with h = -|a|^2/2 + a.x exactly (bm_error_bound).  Here the operand
rounding is emulated bit for bit and the FP32 accumulation in several orders;
h is evaluated in exact rational arithmetic.  The adversarial cases put every
coordinate at the worst bf16 rounding error with the same sign, where the bound
is nearly tight, so an under-estimated constant fails.
"""
from fractions import Fraction

import numpy as np
import pytest

import paper_2601_01405_amd as bm


def bf16_rne(x32):
    """float32 array -> float32 values rounded to bf16 (nearest, ties to even)."""
    u = np.asarray(x32, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def f16_scale(x64, stored_f16):
    """Power of two s with max |s x| <= 2^15 (1 for float16 storage)."""
    m = float(np.abs(x64).max())
    if stored_f16 or m == 0.0:
        return 1.0
    return 2.0 ** (15 - np.frexp(m)[1])


def operands(x64, path, scale=1.0):
    """Per point: (P, Q) operand vectors as float64 holding the exact 16-bit values
    (for f16, of the data scaled by `scale`: float32 rounding, then float16)."""
    x32 = x64.astype(np.float32)
    if path == "f16":
        v = (x64 * scale).astype(np.float32).astype(np.float16).astype(np.float64)
        return v, v
    hi = bf16_rne(x32).astype(np.float64)
    if path == "bf16":
        return hi, hi
    lo = bf16_rne((x64 - hi).astype(np.float32)).astype(np.float64)
    return np.concatenate([hi, hi, lo], axis=-1), np.concatenate([hi, lo, hi], axis=-1)


def fp32_sum(terms, order):
    acc = np.float32(0.0)
    for i in order:
        acc = np.float32(acc + np.float32(terms[i]))   # products are exact in float32
    return acc


def check_pairs(points, pairs, path, eps=1.0, rng=None, stored_f16=None):
    """G is formed in working units (data times s, s a power of two, for the
    scaled f16 path) and compared in data units against the reported bound."""
    rng = rng or np.random.default_rng(0)
    x = np.asarray(points, np.float64)
    d = x.shape[1]
    nu = np.einsum("ij,ij->i", x, x)
    if stored_f16 is None:
        stored_f16 = path == "f16"
    dtype = np.float16 if stored_f16 else np.float32
    b = bm.error_bound(path, dtype, d, eps, nu.max(), np.abs(x).max())
    s = f16_scale(x, stored_f16) if path == "f16" else 1.0
    P, Q = operands(x, path, s)
    worst = 0.0
    for a, p in pairs:
        init = np.float32(-np.float32(nu[a] * s * s) / np.float32(2.0))
        terms = [float(init)] + list(Q[a] * P[p])
        h = -Fraction(nu[a]) / 2 + sum((Fraction(u) * Fraction(v) for u, v in zip(x[a], x[p])), Fraction(0))
        # exact norms for the bound's right-hand side
        nua = sum((Fraction(u) ** 2 for u in x[a]), Fraction(0))
        nux = sum((Fraction(u) ** 2 for u in x[p]), Fraction(0))
        bound = Fraction(b["alpha"]) * nua + Fraction(b["beta"]) * nux + Fraction(b["abs_err"])
        n = len(terms)
        for order in (range(n), range(n - 1, -1, -1), rng.permutation(n)):
            g = fp32_sum(terms, order)
            err = abs(Fraction(float(g)) / Fraction(s * s) - h)
            assert err <= bound, f"{path}: |G-h| = {float(err)} > bound {float(bound)} (pair {a},{p})"
            if bound > 0:
                worst = max(worst, float(err / bound))
    return worst


@pytest.mark.parametrize("path", ["bf16", "bf16x3"])
def test_bound_random_pairs(path):
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal((40, 12)) * 3, rng.uniform(-20, 20, (40, 12))])
    pairs = [(int(i), int(j)) for i, j in rng.integers(0, 80, (120, 2))] + [(i, i) for i in range(10)]
    w = check_pairs(x, pairs, path, rng=rng)
    assert w <= 1.0


def test_bound_f16_storage():
    rng = np.random.default_rng(2)
    x = (rng.standard_normal((60, 20)) * 0.7).astype(np.float16).astype(np.float64)
    x[:5, :3] = 3e-6                       # float16 subnormals
    pairs = [(int(i), int(j)) for i, j in rng.integers(0, 60, (150, 2))]
    check_pairs(x, pairs, "f16", eps=0.3, rng=rng)


@pytest.mark.parametrize("scale", [1e-3, 1.0, 37.0, 3e4])
def test_bound_f16_scaled(scale):
    """float32 data of any magnitude on the f16 path: scaled by a power of two
    into float16 range, rounded, and the bound reported back in data units."""
    rng = np.random.default_rng(5)
    x = (rng.standard_normal((60, 24)) * scale).astype(np.float32).astype(np.float64)
    x[:4, :5] *= 1e-6                      # values that land among float16 subnormals
    pairs = [(int(i), int(j)) for i, j in rng.integers(0, 60, (150, 2))] + [(i, i) for i in range(6)]
    w = check_pairs(x, pairs, "f16", eps=scale, rng=rng, stored_f16=False)
    assert w <= 1.0


def test_bound_f16_scaled_worst_case():
    """Every coordinate just under half a float16 spacing above 1 (after the
    scale): all round down, all with the same sign."""
    v = (1.0 + 2.0 ** -11 - 2.0 ** -20) * 2.0 ** -16      # scaled by 2^30 to just above 2^14
    x = np.full((2, 7), v).astype(np.float32).astype(np.float64)
    w = check_pairs(x, [(0, 1), (0, 0)], "f16", stored_f16=False)
    assert 0.5 < w <= 1.0, w


def test_bound_is_nearly_tight_for_bf16_worst_case():
    """Every coordinate 1 + 2^-8 - 2^-20 rounds down to 1 in bf16 (error just
    under 2^-8 relative); a point against itself then has G - h close to
    -2^-7 |x|^2, which the bound must cover (and does with little room)."""
    d = 3
    v = 1.0 + 2.0 ** -8 - 2.0 ** -20
    x = np.full((2, d), v)
    w = check_pairs(x, [(0, 1), (1, 0), (0, 0)], "bf16")
    assert 0.5 < w <= 1.0, w


def test_bound_three_product_worst_case():
    """hi and lo both near their worst rounding error, all of one sign."""
    v = np.float64(np.float32(1.0 + 2.0 ** -8 - 2.0 ** -20 + 2.0 ** -17 * 0.999))
    x = np.full((2, 9), v)
    w = check_pairs(x, [(0, 1), (0, 0)], "bf16x3")
    assert w <= 1.0


def test_fp32_relative_bound():
    """The plain path's squared distance in FP32 (fused multiply-add per term)
    stays within rel_err of the exact squared distance."""
    rng = np.random.default_rng(4)
    x = (rng.standard_normal((50, 17)) * rng.uniform(0.01, 100, (50, 1))).astype(np.float32)
    b = bm.error_bound("fp32", np.float32, 17, 1.0, 1.0, 1.0)
    for a, p in rng.integers(0, 50, (200, 2)):
        acc = np.float32(0.0)
        for k in range(17):
            t = np.float32(x[a, k] - x[p, k])
            acc = np.float32(np.float64(t) * np.float64(t) + np.float64(acc))   # one rounding per fma
        D = sum((Fraction(float(x[a, k])) - Fraction(float(x[p, k]))) ** 2 for k in range(17))
        assert abs(Fraction(float(acc)) - D) <= Fraction(b["rel_err"]) * D + Fraction(b["abs_err"])


def test_delta_matches_definition():
    """delta is the additive radius error of Sec. 5.1 implied by the D-space bound."""
    b = bm.error_bound("bf16", np.float32, 32, 2.0, 50.0, 3.0)
    w = 2 * ((b["alpha"] + b["beta"]) * 50.0 + b["abs_err"]) + 2.0 ** -23 * (50.0 + 4.0)
    assert b["delta"] == pytest.approx(max(2.0 - np.sqrt(4.0 - w), np.sqrt(4.0 + w) - 2.0), rel=1e-12)
    assert b["exact_range"] == 1
    assert bm.error_bound("bf16", np.float32, 32, 1e-60, 50.0, 3.0)["exact_range"] == 0
