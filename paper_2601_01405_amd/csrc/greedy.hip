// greedy.hip — the serial steps of the blocked greedy (greedy_dev.h) as
// kernels of their own, one workgroup per chain, and the exact FP64 resolve of
// the plain FP32 path.
#include "dev_common.h"
#include "greedy_dev.h"
#include "kernels.h"

namespace bm {

constexpr int STEP_THREADS = 1024;

__global__ __launch_bounds__(STEP_THREADS) void k_block_begin(const ChainTask *__restrict__ chains)
{
    extern __shared__ __align__(16) unsigned char lds[];
    block_open<STEP_THREADS>(chains[blockIdx.x], lds);
}

hipError_t launch_block_begin(const ChainTask *chains, int nchains, hipStream_t s)
{
    if (nchains <= 0) return hipSuccess;
    k_block_begin<<<nchains, STEP_THREADS, (uint32_t)open_lds_bytes<STEP_THREADS>(), s>>>(chains);
    return hipGetLastError();
}

// Conflict words: C[j * nw + w] bit i' = 1 iff candidate i = 64 w + i' < j and
// cand[i] has cand[j] in its ball.  One wave per (row j, word w) with 64 w < j.
__global__ __launch_bounds__(256) void k_resolve_exact(PointsView P, double e2, const int32_t *cand,
                                                       const GreedyState *st, int nw, uint64_t *C, int *rowflag)
{
    const int nc = st->nc;
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int w = blockIdx.x;
    if (j >= nc || (w << 6) >= j) return;      // wave-uniform
    const int i = (w << 6) + lane_id();
    bool hit = false;
    if (i < j) hit = exact_member(P, orig_index(P, cand[i]), orig_index(P, cand[j]), e2);
    uint64_t m = __ballot(hit);
    if (lane_id() == 0) {
        C[(int64_t)j * nw + w] = m;
        if (m) rowflag[j] = 1;
    }
}

hipError_t launch_resolve_exact(const PointsView &P, double e2, const int32_t *cand, const GreedyState *st,
                                int B, uint64_t *C, int *rowflag, hipStream_t s)
{
    const int nw = (B + 63) / 64;
    dim3 grid(nw, (B + 3) / 4);
    k_resolve_exact<<<grid, 256, 0, s>>>(P, e2, cand, st, nw, C, rowflag);
    return hipGetLastError();
}

__global__ __launch_bounds__(STEP_THREADS) void k_accept(const ChainTask *__restrict__ chains)
{
    extern __shared__ __align__(16) unsigned char lds[];
    block_accept<STEP_THREADS>(chains[blockIdx.x], lds);
}

hipError_t launch_accept(const ChainTask *chains, int nchains, int maxB, hipStream_t s)
{
    if (maxB > MAX_B) return hipErrorInvalidValue;
    if (nchains <= 0) return hipSuccess;
    k_accept<<<nchains, STEP_THREADS, (uint32_t)accept_lds_bytes<STEP_THREADS>(), s>>>(chains);
    return hipGetLastError();
}

} // namespace bm
