// bm_internal.h — types shared by the host driver and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bm {

// Stored point cloud on the device.  All per-point device arrays of the
// driver are indexed by RANK (position in the visiting order); `perm` maps a
// rank to the original row of `X` (nullptr = identity).
struct PointsView {
    const void *X;
    int64_t n;
    int32_t d;
    int32_t dtype;          // 0 f64, 1 f32, 2 f16
    const int32_t *perm;
};

// Per-block state of the greedy, written by the kernels, read back by the host.
struct GreedyState {
    int64_t cursor;                 // every rank < cursor is a landmark or covered
    int32_t nc;                     // candidates gathered in this block
    int32_t na;                     // candidates accepted in this block
    unsigned long long nkeys;       // membership keys appended so far
    unsigned long long band;        // pairs the filter sent to the FP64 recheck
    unsigned long long rounds;      // acceptance rounds (diagnostic)
};

// Decision thresholds of the plain FP32 filter (direct difference):
// s32 <  lo  => member for sure;  s32 >= hi => non-member for sure; else band.
struct Fp32Thresholds {
    float lo, hi;
    float unrefined;                // threshold used when refine == 0
};

// MFMA operand layout: points are stored as K-padded rows of 16-bit values
// (bf16 or f16), K = kpad, grouped in tiles of 32 points.  For the three-product
// split the row holds [hi | hi | lo] against the landmark side [hi | lo | hi].
enum MfmaKind { MFMA_BF16 = 2, MFMA_BF16X3 = 3, MFMA_F16 = 4 };

struct MfmaParams {
    int32_t kind;
    int32_t kpad;                   // padded K (multiple of 16)
    float   w_scale;                // not used on device; kept for stats
};

} // namespace bm
