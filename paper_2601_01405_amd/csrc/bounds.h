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

} // namespace bm
