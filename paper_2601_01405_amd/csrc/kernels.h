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
// Opens a block of every chain (one workgroup each): lists up to B uncovered
// ranks after the cursor and clears rowflag[0..B); with `settle` appends the
// settled non-landmarks below the first candidate to the chain's settled set;
// with `pack` packs the candidates' operands and scalars for the matrix-core
// resolve.  A chain whose gather finds nothing is done (counted in *ndone).
hipError_t launch_block_begin(const ChainTask *chains, int nchains, hipStream_t s);
// Conflict words of the candidate block with the FP64 predicate on every pair.
hipError_t launch_resolve_exact(const PointsView &P, double e2, const int32_t *cand, const GreedyState *st,
                                int B, uint64_t *C, int *rowflag, hipStream_t s);
// Accepts in rank order (one workgroup per chain); appends to landmarks
// (original indices) and lm_rank at ordinal st->L, and records the block in
// blog[(st->blocks - 1) % kBlockLogSize].
hipError_t launch_accept(const ChainTask *chains, int nchains, int maxB, hipStream_t s);

// ---- range passes -----------------------------------------------------------------------
// Range-pass launchers take an optional event pair (null: none) that records
// the dispatch's own start and end (no separate marker packets on the stream).
struct LaunchEvents {
    hipEvent_t start, stop;
    KernelClock *clock;             // device-clock execution window (may be null)
};

// Plain FP32 range pass of landmarks A[0..blk[1]) (ranks), ordinals blk[0] + i.
hipError_t launch_range_fp32(const float *xf, const PointsView &P, double e2, Fp32Thresholds thr,
                             int refine, const int32_t *A, const int64_t *blk, int na_max,
                             const RangeOut &o, hipStream_t s, LaunchEvents ev = {});

// One-wave check of the matrix-core layout and subnormal handling (flags, see range_mfma.hip).
hipError_t run_selfcheck(int *flags_dev, hipStream_t s);
// Grid of one matrix-core range task: landmark groups and point chunks (a
// multiple of 8) for up to na_max landmarks against up to n_max points, about
// target_wg workgroups.
void range_grid(int na_max, int64_t n_max, int64_t target_wg, int32_t *NGW, int32_t *chunks);
// Matrix-core range passes (conflict = false) or candidate resolves (true) of
// tasks that share operand kind and K = 16 S, in one launch of total_wgs
// workgroups (task_of maps workgroups to tasks; null: one task).
hipError_t launch_range_tasks(const RangeTask *tasks, const int32_t *task_of, int64_t total_wgs, int kind, int S,
                              bool conflict, hipStream_t s, LaunchEvents ev = {});

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
// Work list of the edge pass: rows i with a member x in some other ball
// (|S(x)| > 1), from the sorted keys; flag[L] and *count must start at zero.
hipError_t launch_edge_rows(const uint64_t *keys, int64_t M, int32_t bn, const int64_t *sptr, int64_t L, int *flag,
                            int32_t *list, unsigned long long *count, hipStream_t s);
// Over the rows rows[0..nrows) (null: 0..nrows-1) of L rows.  mode 0: deg[i] =
// number of neighbours j > i;  mode 1: write them at eptr[i].  seg[0..nseg]
// (device, may be null) splits the rows into segments that share no column
// (the chains of a batch), which bounds the neighbours of a row.
// Row bitmaps the counting pass keeps for the emitting pass: `cap` slots of
// `words` words (one bit per landmark past the row), claimed with *count (zero
// at the start); slots[b] is the slot of the pass's workgroup b, or -1.  All
// null: every row is walked twice.
struct EdgeStore {
    uint64_t *bits;
    int64_t words, cap;
    unsigned long long *count;
    int32_t *slots;
};
hipError_t launch_edge_pass(int mode, int64_t nrows, const int32_t *rows, int64_t L, const int64_t *seg, int nseg,
                            const int64_t *row_ptr, const int32_t *member_idx, const int64_t *sptr,
                            const int32_t *slist, int64_t *deg, const int64_t *eptr, int32_t *edges,
                            const EdgeStore &store, hipStream_t s);

// ---- batches (batch.hip) ---------------------------------------------------------------------
// Sorted chain-tagged keys (chain << (bl + bn) | ordinal << bn | index) into the
// disjoint union: (lm_off[chain] + ordinal) << bnu | (pt_off[chain] + index).
hipError_t launch_union_keys(uint64_t *keys, int64_t M, int32_t bn, int32_t bl, const int64_t *lm_off,
                             const int64_t *pt_off, int32_t bnu, hipStream_t s);
// Per chain: union landmarks, rebased row pointers (L_c + 1 at lm_off[c] + c),
// columns and edges in the chain's own numbering, and ranges[4c..4c+3] = its
// member range and edge range in the union arrays.
hipError_t launch_rebase_chains(int nchains, const int32_t *const *lm, const int64_t *lm_off, const int64_t *pt_off,
                                const int64_t *row_ptr, int32_t *midx, const int64_t *eptr, int32_t *edges,
                                int32_t *lm_union, int64_t *mp_union, int64_t *ranges, hipStream_t s);

} // namespace bm
