// kernels.h — host-side launchers of the gfx950 kernels (all asynchronous on `s`).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "bm_internal.h"

namespace bm {

// ---- preparation (prep.hip) ------------------------------------------------------------
// Sets *bad = 1 if any coordinate is NaN or infinite.
hipError_t launch_check_finite(const void *X, int32_t dtype, int64_t count, int *bad, hipStream_t s);

// Per point (by rank): nu[r] = |x_r|^2 in FP64; maxima of |x|^2 and of |x_k| go to
// stats[0], stats[1] as the bit patterns of non-negative doubles.
hipError_t launch_point_stats(const PointsView &P, double *nu, unsigned long long *stats, hipStream_t s);

// FP32 copy of the points in rank order (round to nearest).
hipError_t launch_to_f32(const PointsView &P, float *xf, hipStream_t s);

// MFMA operands in the swizzled tile layout (range_mfma.hip).  Qop may equal Pop.
// `scale` multiplies the coordinates before rounding (F16 path on wider storage; 1 otherwise).
hipError_t launch_mfma_operands(const PointsView &P, int kind, int S, double scale, uint16_t *Pop, uint16_t *Qop,
                                hipStream_t s);
// Per-point accumulator start, rounded-up norm and decision thresholds for one eps,
// in working units: nu_scale = scale^2, b and e2 already in those units.
hipError_t launch_mfma_scalars(int64_t n, const double *nu, double nu_scale, const MfmaBound &b, double e2, int d,
                               float *cinit, float *nuup, float *T3, hipStream_t s);

// ---- greedy (greedy.hip) ----------------------------------------------------------------
// Lists up to B uncovered ranks after the cursor and clears rowflag[0..B).
hipError_t launch_gather(const uint64_t *covered, int64_t n, GreedyState *st, int B, int32_t *cand,
                         int *rowflag, hipStream_t s);
// Conflict words of the candidate block with the FP64 predicate on every pair.
hipError_t launch_resolve_exact(const PointsView &P, double e2, const int32_t *cand, const GreedyState *st,
                                int B, uint64_t *C, int *rowflag, hipStream_t s);
// Accepts in rank order; appends to landmarks (original indices) and lm_rank
// at ordinal st->L, and records the block in blog[st->blocks % kBlockLogSize].
hipError_t launch_accept(const uint64_t *C, const int *rowflag, const int32_t *cand, GreedyState *st, int B,
                         int32_t *A, int32_t *landmarks, int32_t *lm_rank, BlockLog *blog, const int32_t *perm,
                         uint64_t *islm, int64_t n, hipStream_t s);
// After a gather: append the settled non-landmarks below the block's first candidate.
hipError_t launch_settle(const uint64_t *islm, GreedyState *st, const int32_t *cand, const MfmaArgs &a,
                         const SettledSet &out, const int32_t *perm, hipStream_t s);

// ---- range passes -----------------------------------------------------------------------
// Range pass of landmarks A[0..blk[1]) (ranks) with ordinals blk[0] + i;
// blk points to device memory (the greedy state's L0/na, or a fixed table).
// Members are appended as keys (ordinal << bn | original index) and their
// covered bits set.
struct RangeOut {
    uint64_t *covered;              // rank-order bitmap, may be null (fixed-landmark mode)
    uint64_t *keys;
    unsigned long long cap;
    GreedyState *st;                // nkeys / band counters
    int32_t bn;                     // bits of the original index in a key
};

// Range-pass launchers take an optional event pair (null: none) that records
// the dispatch's own start and end (no separate marker packets on the stream).
struct LaunchEvents {
    hipEvent_t start, stop;
    KernelClock *clock;             // device-clock execution window (may be null)
};

hipError_t launch_range_fp32(const float *xf, const PointsView &P, double e2, Fp32Thresholds thr,
                             int refine, const int32_t *A, const int64_t *blk, int na_max,
                             const RangeOut &o, hipStream_t s, LaunchEvents ev = {});

// One-wave check of the matrix-core layout and subnormal handling (flags, see range_mfma.hip).
hipError_t run_selfcheck(int *flags_dev, hipStream_t s);
// blk[0..3] = first ordinal, landmark count, rlo, settled count (see SettledSet);
// rlo = 0 and a zero count scan every rank.
hipError_t launch_range_mfma(const MfmaArgs &a, const PointsView &P, double e2, const int32_t *A,
                             const int64_t *blk, int na_max, const RangeOut &o, const SettledSet &sd, hipStream_t s,
                             LaunchEvents ev = {});
// Candidate-block resolve on the matrix cores: `packed` holds the candidates'
// operands and scalars in candidate order, Pc.perm their original indices;
// writes the conflict words (as 32-bit halves) and row flags.
hipError_t launch_resolve_mfma(const MfmaArgs &packed, const PointsView &Pc, const int32_t *nc_dev, double e2, int B,
                               uint32_t *C32, int *rowflag, GreedyState *st, hipStream_t s);
hipError_t launch_pack_candidates(const MfmaArgs &a, const int32_t *cand, const GreedyState *st, const int32_t *perm,
                                  int B, const MfmaArgs &out, int32_t *cand_orig, hipStream_t s);

// ---- membership CSR (csr.hip) -------------------------------------------------------------
hipError_t sort_keys(void *tmp, size_t *tmp_bytes, const uint64_t *in, uint64_t *out, size_t count,
                     int end_bit, hipStream_t s);
hipError_t launch_csr_from_sorted(const uint64_t *keys, int64_t M, int64_t L, int32_t bn,
                                  int64_t *row_ptr, int32_t *member_idx, hipStream_t s);

// ---- edges (edges.hip) ----------------------------------------------------------------------
hipError_t scan_excl_i64(void *tmp, size_t *tmp_bytes, const int64_t *in, int64_t *out, size_t count,
                         hipStream_t s);
hipError_t launch_point_degree(const int32_t *member_idx, int64_t M, int64_t *cnt, hipStream_t s);
// S(x): the landmarks whose ball holds x, from the sorted membership keys.
hipError_t launch_fill_slists(const uint64_t *keys, int64_t M, int32_t bn, const int64_t *sptr,
                              int64_t *sfill, int32_t *slist, hipStream_t s);
// mode 0: deg[i] = number of neighbours j > i;  mode 1: write them at eptr[i].
hipError_t launch_edge_pass(int mode, int64_t L, const int64_t *row_ptr, const int32_t *member_idx,
                            const int64_t *sptr, const int32_t *slist, int64_t *deg,
                            const int64_t *eptr, int32_t *edges, hipStream_t s);

} // namespace bm
