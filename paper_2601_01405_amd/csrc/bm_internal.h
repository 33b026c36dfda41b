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

// State of the greedy, kept on the device so blocks can be queued back to
// back; the host reads it once per batch of blocks.
struct GreedyState {
    int64_t cursor;                 // every rank < cursor is a landmark or covered
    int64_t L0;                     // ordinal of this block's first landmark      } read by the
    int64_t na;                     // candidates accepted in this block            } range pass
    int64_t rlo;                    // ranks >= rlo (a multiple of 32) are scanned  } as blk[0..3]
    int64_t m;                      // settled non-landmarks (ranks < rlo) listed   }
    int64_t L;                      // landmarks so far
    int32_t nc;                     // candidates gathered in this block
    int32_t done;                   // 1 once a gather found no uncovered rank
    int32_t error;                  // 1 if the acceptance rounds did not converge
    int32_t pad_;
    unsigned long long nkeys;       // membership keys appended so far
    unsigned long long band;        // pairs the filter sent to the FP64 recheck
    unsigned long long rounds;      // acceptance rounds (diagnostic)
    unsigned long long blocks;      // blocks with at least one candidate
    unsigned long long candidates;  // candidates over all blocks
    unsigned long long resolve_pairs;
    unsigned long long range_pairs; // landmark-point pairs the range passes computed
};

// Per-block record for recomputing a block's memberships after the key
// buffer overflowed: its first ordinal, accepted count and key count before it.
struct BlockLog {
    int64_t L0, na, rlo, m;         // the range pass's blk[0..3]
    unsigned long long nkeys_before;
};

// Settled non-landmarks.  In refined mode a landmark is never in another
// landmark's ball (the net is separated and the exact predicate is symmetric),
// so a block's range pass need not look at earlier landmarks: it scans every
// rank >= rlo (rlo = the block's first candidate rounded down to a tile) and,
// below rlo, only this compacted list of covered non-landmarks, in rank order.
// Entries >= m carry +inf thresholds and zero operands.
struct SettledSet {
    uint16_t *Pop;                  // point-side operands, swizzled like MfmaArgs::Pop
    float *T3;                      // thresholds, tiled like MfmaArgs::T3
    int32_t *idx;                   // original row index of entry j
};
constexpr int kBlockLogSize = 256;

// Decision thresholds of the plain FP32 filter (direct difference):
// s32 <  lo  => member for sure;  s32 >= hi => non-member for sure; else band.
struct Fp32Thresholds {
    float lo, hi;
    float unrefined;                // threshold used when refine == 0
};

// MFMA paths.  Operands are 16-bit words (bf16 or f16) in K-padded rows
// (K a multiple of 16), swizzled so that one 32x32x16 step of a 32-point tile
// is 1 KB of contiguous memory: element e of lane l of step s of tile t sits
// at ((t * S + s) * 64 + l) * 8 + e and holds coordinate k = 16 s + 8 (l / 32) + e
// of point 32 t + l % 32.  With the three-product split the point side holds
// [hi | hi | lo] and the landmark side [hi | lo | hi], so their dot product is
// hi.hi + hi.lo + lo.hi.
enum MfmaKind { MFMA_BF16 = 2, MFMA_BF16X3 = 3, MFMA_F16 = 4 };
constexpr int kMaxMfmaSteps = 30;           // K <= 480: d <= 480 (one product) or 160 (three)

// 16-bit words of a swizzled operand array for `points` points and S steps:
// ceil(points / 32) tiles x S steps x 64 lanes x 8 values.
inline size_t mfma_operand_words(int64_t points, int S)
{
    return (size_t)((points + 31) / 32) * (size_t)S * 64 * 8;
}

// Execution window of a kernel on the device clock: every workgroup lowers
// `start` at entry; the last one to finish adds (now - start) to `ticks` and
// resets `start` and `done` for the next launch.
struct KernelClock {
    unsigned long long start, done, ticks;
};

enum { T3_U = 0, T3_V = 1, T3_Z = 2 };
__host__ __device__ inline int64_t t3_index(int64_t r, int which) { return (r >> 5) * 96 + which * 32 + (r & 31); }
// floats of a tiled threshold array for `points` points
inline size_t t3_floats(int64_t points) { return (size_t)((points + 31) / 32) * 96; }

// Constants of the MFMA error bound (host computed, see bounds.h).  The kernel
// output for landmark a and point x is  G = -RN32(nu_a)/2 + sum_k P_k Q_k, an
// estimate of (nu_x - D)/2, and |G - (nu_x - D)/2| <= alpha nu_a + beta nu_x + abs.
struct MfmaBound {
    double alpha, beta, abs_err;
    double t_in, t_out;             // exact-decision window on D
    bool sane;                      // false: every pair goes to the FP64 recheck
};

struct MfmaArgs {
    const uint16_t *Pop;            // point-side operands, swizzled
    const uint16_t *Qop;            // landmark-side operands, swizzled
    const float *cinit;             // per rank: -RN32(nu)/2
    const float *nuup;              // per rank: nu rounded up
    // Decision thresholds, tiled per 32 ranks: tile t holds U[32], V[32], Z[32]
    // (t3_index); padding ranks hold +inf.
    //   G <= U - alpha*nu_a  =>  not a member;   G > V + alpha*nu_a  =>  member;
    //   unrefined: member iff G > Z.
    const float *T3;
    float alpha;                    // rounded up
    int32_t S;                      // K / 16
    int32_t kind;
    int32_t refine;
};

} // namespace bm
