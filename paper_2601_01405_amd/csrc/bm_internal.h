// bm_internal.h — types shared by the host driver and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bm {

// Stored point cloud on the device.  All per-point device arrays of the
// driver are indexed by RANK (position in the visiting order); `perm` maps a
// rank to the original row of `X` (nullptr = identity).
// Largest candidate block B (the serial steps hold a block's bitmaps in LDS).
constexpr int kMaxBlock = 16384;

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
    unsigned long long accepted;    // blocks accepted (their block log entries are written)
    unsigned int ticket;            // workgroups of the running launch that have finished
    unsigned int pad2_;
    int64_t settle_from;            // settled entries [settle_from, m) listed by the last
                                    // opening (ranks in idx), copied by the next resolve
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
    int32_t *idx;                   // original row index of entry j (its rank until copied)
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
// resets `start` and `done` for the next launch.  `tail` sums the time of the
// serial step a task's last workgroup runs after the window (accept or open).
struct KernelClock {
    unsigned long long start, done, ticks, tail;
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

// Where a range pass puts its members: key (ordinal << bn | original index) | tag
// at position atomicAdd(nkeys, 1) when it is below cap (the count goes on past
// cap, so an overflow is seen and the block recomputed into a bigger buffer).
struct RangeOut {
    uint64_t *covered;              // rank-order bitmap, may be null (fixed-landmark mode)
    uint64_t *keys;
    unsigned long long cap;
    unsigned long long *nkeys;      // key counter (one per build, or shared by a batch)
    GreedyState *st;                // band counter
    uint64_t tag;                   // or-ed into every key: the chain number in a batch, else 0
    int32_t bn;                     // bits of the original index in a key
};

// One greedy chain (one point cloud at one radius), as the block-opening and
// acceptance kernels see it; a launch of those kernels runs one workgroup per chain.
struct ChainTask {
    const uint64_t *covered;        // rank-order covered bitmap
    int64_t n;
    GreedyState *st;
    int32_t B;                      // candidate block size
    int32_t settle;                 // 1: keep the settled non-landmark list (refined matrix-core path)
    int32_t *cand;                  // [B] candidate ranks
    int32_t *rowflag;               // [B]
    uint64_t *islm;                 // rank-order landmark bitmap (settle)
    MfmaArgs a;                     // the chain's operands and scalars
    SettledSet sd;
    const int32_t *perm;            // rank -> original index (null: identity)
    uint64_t *C;                    // conflict words, ceil(B/64) per candidate (zero between blocks)
    int32_t *A;                     // accepted ranks of the block
    int32_t *landmarks;             // original indices, selection order
    int32_t *lm_rank;               // ranks, selection order
    BlockLog *blog;
    const unsigned long long *nkeys;   // the key counter its range passes append to
    unsigned long long *ndone;      // chains finished (batch), or null
};

// One matrix-core range pass (or candidate-block resolve) of a launch.  A launch
// serves one or more tasks of the same operand kind and K: workgroup b works for
// task task_of[b] (task 0 without a map) as its local workgroup b - wg0.
struct RangeTask {
    MfmaArgs a;
    PointsView P;                   // resolve: the candidates (perm = their original indices)
    const int32_t *n_dev;           // device-side point count (resolve: candidate count), or null
    double e2;
    const int32_t *A;               // landmark ranks; null: 0, 1, 2, ... (resolve)
    const int64_t *blk;             // blk[0..3]: first ordinal, count, rlo, settled count (see SettledSet)
    RangeOut o;
    SettledSet sd;
    uint32_t *C32;                  // resolve output: conflict words, row flags
    int32_t c32_stride;
    int32_t *rowflag;
    int32_t NGW, chunks;            // this task's grid: NGW landmark groups x chunks point chunks
    int32_t wg0;                    // its first workgroup in the launch (a multiple of 8)
    const ChainTask *chain;         // if set, the task's last workgroup to finish runs the chain's
                                    // next serial step: accept after a resolve, open the next
                                    // block after a range pass
};

} // namespace bm
