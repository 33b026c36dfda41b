// bounds.h — host-side error bounds that turn a low-precision distance filter
// into an exact decision (the verified range set of Sec. 5.3).
//
// Notation.  x̄ is a stored point widened exactly to FP64, D(a,x) = |ā - x̄|^2
// the exact real squared distance, s(a,x) the FP64 predicate value (sequential
// sum, round to nearest, no FMA) and e2 = RN(eps^2).  Standard summation
// analysis gives |s - D| <= g64 * D with g64 = gamma_{d+2}(2^-53), so
//     D >= T_out := e2 / (1 - g64)   implies  s >= e2   (not a member)
//     D <  T_in  := e2 / (1 + g64)   implies  s <  e2   (member).
// A filter f with a proven bound |f - D| <= Delta then decides "out" when
// f - Delta >= T_out and "in" when f + Delta < T_in; every other pair is
// recomputed with s.  This is the additive delta-accurate model of Sec. 5.1
// (delta on squared distances) with an exact verification of the band.
#pragma once
#include <cfloat>
#include <cmath>

#include "bm_internal.h"

namespace bm {

inline double gamma_u(double m, double u) { return m * u / (1.0 - m * u); }

// Smallest float >= v / largest float <= v (v finite double).
inline float f32_up(double v)
{
    if (!(v <= (double)FLT_MAX)) return INFINITY;
    float f = (float)v;
    if ((double)f < v) f = std::nextafter(f, INFINITY);
    return f;
}
inline float f32_down(double v)
{
    if (!(v >= -(double)FLT_MAX)) return -INFINITY;
    float f = (float)v;
    if ((double)f > v) f = std::nextafter(f, -INFINITY);
    return f;
}

constexpr double kRel = 1e-12;     // slack for the FP64 evaluation of the bounds themselves

inline void exact_window(double e2, int d, double *t_in, double *t_out)
{
    const double g64 = gamma_u(d + 2.0, std::ldexp(1.0, -53));
    *t_out = e2 / (1.0 - g64) * (1.0 + kRel);
    *t_in = e2 / (1.0 + g64) * (1.0 - kRel);
}

// Plain FP32 path.  The kernel rounds the points to FP32 (exact for f32/f16
// storage; |x̂ - x̄| <= 2^-24 |x̄| componentwise for f64 storage) and forms
// s32 = sum_k fma(t_k, t_k, acc) with t_k = RN32(â_k - x̂_k).  With
// Ŝ = |â - x̂|^2:  |s32 - Ŝ| <= g32 Ŝ, g32 = gamma_{d+2}(2^-24) (the relative
// error model of Sec. 5.2), plus at most d * 2^-126 from values below the
// normal range; and |sqrt(Ŝ) - sqrt(D)| <= E := 2^-24 (|ā| + |x̄|) <= 2^-23 R
// with R the largest point norm, plus sqrt(d) 2^-148 for coordinates below the
// FP32 normal range (E = 0 for f32/f16 storage).
//   out for sure:  s32 >= hi := (1 + g32) (sqrt(T_out) + E)^2 + d 2^-125
//   in  for sure:  s32 <  lo := (1 - g32) (sqrt(T_in) - E)^2 - d 2^-125
// A NaN `hi` disables "out" and -inf `lo` disables "in" (every pair is then
// rechecked), used when the data or eps leave the range where these bounds hold.
inline Fp32Thresholds fp32_thresholds(double e2, int d, int dtype, double max_norm, double max_abs)
{
    Fp32Thresholds t;
    t.unrefined = (float)e2;
    double t_in, t_out;
    exact_window(e2, d, &t_in, &t_out);
    const double g32 = gamma_u(d + 2.0, std::ldexp(1.0, -24));
    const double E = (dtype == 0) ? (std::ldexp(max_norm, -23) + std::sqrt((double)d) * std::ldexp(1.0, -148)) * (1.0 + kRel)
                                  : 0.0;
    const double tiny = d * std::ldexp(1.0, -125);
    const bool sane = e2 >= std::ldexp(1.0, -100) && e2 <= std::ldexp(1.0, 100) &&
                      max_abs <= std::ldexp(1.0, 60);
    if (!sane) {
        t.lo = -INFINITY;
        t.hi = NAN;
        return t;
    }
    const double so = std::sqrt(t_out) * (1.0 + kRel) + E;
    t.hi = f32_up((1.0 + g32) * so * so * (1.0 + kRel) + tiny);
    if (std::isinf(t.hi)) t.hi = NAN;
    const double si = std::sqrt(t_in) * (1.0 - kRel) - E;
    if (si <= 0.0) {
        t.lo = -INFINITY;
    } else {
        const double lo = (1.0 - g32) * si * si * (1.0 - kRel) - tiny;
        t.lo = lo > 0.0 ? f32_down(lo) : -INFINITY;
    }
    return t;
}

// MFMA paths.  Per coordinate the operands carry a relative error rho
// (|x̂ - x̄| <= rho |x̄| + tau), so a product term is off by at most
// rho_p |ā_k x̄_k| + m tau (1 + rho)(|ā_k| + |x̄_k|) + m tau^2 (m products per
// coordinate); summed, sum_k |ā_k x̄_k| <= |ā||x̄| <= (nu_a + nu_x)/2 and
// sum_k (|ā_k| + |x̄_k|) <= sqrt(d)(|ā| + |x̄|) <= 2 sqrt(d) R.  The matrix core
// accumulates K products and the initial value in FP32 in an unspecified
// order; we charge gamma_{K+1}(2^-23) on the sum of magnitudes (this also
// covers truncating instead of rounding) and 2^-126 per step for values below
// the normal range.  The initial value -RN32(nu_a)/2 is off by
// (2^-24 + gamma_d(2^-53)) nu_a / 2.
//   rho_p:  BF16  (2 rho + rho^2), rho = (2^-8 + 2^-24)(1 + 2^-20): bf16 keeps 8
//                 significant bits, so round-to-nearest is off by up to 2^-8
//                 relative, after at most 2^-24 from a float64 -> float32 step
//           BF16X3  3 * 2^-16 (1 + 2^-6)   (hi off by 2^-8, lo by 2^-8 of the
//                 remainder: the dropped lo.lo and residual terms)
//           F16   0 for float16 storage (exact); otherwise the data are scaled by
//                 a power of two into float16 range and rounded: 2 rho + rho^2 with
//                 rho = (2^-11 + 2^-24)(1 + 2^-20), in the scaled units
//   tau:    2^-126 for bf16 (values flushed below the normal range), for f16
//           0 (stored) or 2^-25 (rounded) when the device honours f16 subnormals
//           in MFMA, else 2^-14.
// Power-of-two scale that brings float32/float64 data into float16 range for
// the F16 path: max |s x| <= 2^15 < 65504.  float16 storage is used as is (s = 1).
inline double f16_scale(int dtype, double max_abs)
{
    if (dtype == 2 || !(max_abs > 0.0)) return 1.0;
    int e;
    std::frexp(max_abs, &e);                 // max_abs < 2^e
    return std::ldexp(1.0, 15 - e);
}

// All inputs in the path's working units (for a scaled F16 path: e2, max_norm
// and max_abs already multiplied by s^2, s, s).  `stored_f16` tells whether the
// operands are the stored float16 values (exact) or roundings of wider data.
inline MfmaBound mfma_bound(int kind, int d, int K, double e2, double max_norm, double max_abs, bool f16_subnormals_ok,
                            bool stored_f16 = true)
{
    MfmaBound b{};
    const double u24 = std::ldexp(1.0, -24);
    const double g64d = gamma_u((double)d, std::ldexp(1.0, -53));
    const double gK = gamma_u(K + 1.0, std::ldexp(1.0, -23));
    double rho, rho_p, tau;
    int m = 1;
    if (kind == MFMA_BF16) {
        rho = (std::ldexp(1.0, -8) + u24) * (1.0 + std::ldexp(1.0, -20));
        rho_p = 2.0 * rho + rho * rho;
        tau = std::ldexp(1.0, -126);
    } else if (kind == MFMA_BF16X3) {
        rho = (std::ldexp(1.0, -8) + u24) * (1.0 + std::ldexp(1.0, -20));
        rho_p = 3.0 * std::ldexp(1.0, -16) * (1.0 + std::ldexp(1.0, -6));
        tau = std::ldexp(1.0, -126);
        m = 3;
    } else if (stored_f16) {
        rho = 0.0;
        rho_p = 0.0;
        tau = f16_subnormals_ok ? 0.0 : std::ldexp(1.0, -14);
    } else {
        // round to nearest float16 (11 significant bits) after at most one float32 rounding;
        // below the normal range the error is absolute: half the subnormal spacing 2^-24,
        // or the whole value if subnormals were flushed
        rho = (std::ldexp(1.0, -11) + u24) * (1.0 + std::ldexp(1.0, -20));
        rho_p = 2.0 * rho + rho * rho;
        tau = f16_subnormals_ok ? std::ldexp(1.0, -25) : std::ldexp(1.0, -14);
    }
    const double mag = (1.0 + rho) * (1.0 + rho) * (1.0 + std::ldexp(1.0, -6));   // sum|P Q| <= mag (nu_a+nu_x)/2
    const double op_abs = 2.0 * m * tau * (1.0 + rho) * std::sqrt((double)d) * max_norm + m * (double)d * tau * tau;
    const double slack = 1.0 + std::ldexp(1.0, -20);
    b.alpha = slack * ((u24 + g64d) / 2.0 + rho_p / 2.0 + gK * ((1.0 + u24) / 2.0 + mag / 2.0)) ;
    b.beta = slack * (rho_p / 2.0 + gK * mag / 2.0 + g64d);
    b.abs_err = 2.0 * ((1.0 + gK) * op_abs + (K + 2.0) * std::ldexp(1.0, -126));
    exact_window(e2, d, &b.t_in, &b.t_out);
    b.sane = e2 >= std::ldexp(1.0, -100) && e2 <= std::ldexp(1.0, 100) && max_abs <= std::ldexp(1.0, 60) &&
             max_norm * max_norm <= std::ldexp(1.0, 100);
    return b;
}

} // namespace bm
