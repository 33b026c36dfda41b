// batch.hip — finishing many greedy chains at once.
//
// The chains of a batch append their memberships to one key buffer as
// (chain << (bl + bn)) | (ordinal << bn) | index.  After one sort the keys are
// renumbered into the disjoint union of all chains: row lm_off[c] + ordinal,
// column pt_off[c] + index.  Renumbering keeps the order (offsets grow with
// the chain), so the union's CSR and its edges come from the single-build
// kernels, and no edge joins two chains (their columns are disjoint).  Each
// chain's result is then a slice of the union, rebased to its own numbering.
#include "dev_common.h"
#include "kernels.h"

namespace bm {

__global__ void k_union_keys(uint64_t *keys, int64_t M, int32_t bn, int32_t bl, const int64_t *lm_off,
                             const int64_t *pt_off, int32_t bnu)
{
    const uint64_t mn = (1ull << bn) - 1, ml = (1ull << bl) - 1;
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < M; m += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[m];
        const int64_t c = (int64_t)(k >> (bn + bl));
        const uint64_t row = (uint64_t)lm_off[c] + ((k >> bn) & ml);
        const uint64_t col = (uint64_t)pt_off[c] + (k & mn);
        keys[m] = (row << bnu) | col;
    }
}

hipError_t launch_union_keys(uint64_t *keys, int64_t M, int32_t bn, int32_t bl, const int64_t *lm_off,
                             const int64_t *pt_off, int32_t bnu, hipStream_t s)
{
    if (M <= 0) return hipSuccess;
    int64_t blocks = (M + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_union_keys<<<(int)blocks, 256, 0, s>>>(keys, M, bn, bl, lm_off, pt_off, bnu);
    return hipGetLastError();
}

// One workgroup per chain c: its landmarks into the union list; its row
// pointers rebased to start at 0 (L_c + 1 entries at lm_off[c] + c); its
// columns back to its own point indices; its edges back to its own ordinals;
// and its member and edge ranges in the union.
__global__ void k_rebase_chains(int nchains, const int32_t *const *lm, const int64_t *lm_off, const int64_t *pt_off,
                                const int64_t *row_ptr, int32_t *midx, const int64_t *eptr, int32_t *edges,
                                int32_t *lm_union, int64_t *mp_union, int64_t *ranges)
{
    const int c = (int)blockIdx.x;
    if (c >= nchains) return;
    const int64_t l0 = lm_off[c], L = lm_off[c + 1] - l0;
    const int64_t p0 = pt_off[c];
    const int64_t m0 = row_ptr[l0], m1 = row_ptr[l0 + L];
    const int64_t e0 = eptr[l0], e1 = eptr[l0 + L];
    for (int64_t i = threadIdx.x; i < L; i += blockDim.x) lm_union[l0 + i] = lm[c][i];
    for (int64_t i = threadIdx.x; i <= L; i += blockDim.x) mp_union[l0 + c + i] = row_ptr[l0 + i] - m0;
    for (int64_t m = m0 + threadIdx.x; m < m1; m += blockDim.x) midx[m] = (int32_t)(midx[m] - p0);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        edges[2 * e] = (int32_t)(edges[2 * e] - l0);
        edges[2 * e + 1] = (int32_t)(edges[2 * e + 1] - l0);
    }
    if (threadIdx.x == 0) {
        ranges[4 * c] = m0;
        ranges[4 * c + 1] = m1;
        ranges[4 * c + 2] = e0;
        ranges[4 * c + 3] = e1;
    }
}

hipError_t launch_rebase_chains(int nchains, const int32_t *const *lm, const int64_t *lm_off, const int64_t *pt_off,
                                const int64_t *row_ptr, int32_t *midx, const int64_t *eptr, int32_t *edges,
                                int32_t *lm_union, int64_t *mp_union, int64_t *ranges, hipStream_t s)
{
    if (nchains <= 0) return hipSuccess;
    k_rebase_chains<<<nchains, 256, 0, s>>>(nchains, lm, lm_off, pt_off, row_ptr, midx, eptr, edges, lm_union,
                                            mp_union, ranges);
    return hipGetLastError();
}

} // namespace bm
