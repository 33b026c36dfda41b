// range_fp32.hip — the plain FP32 range pass (baseline path).
//
// Every accepted landmark is compared with every point (the direct range
// query of Sec. 1/Sec. 3), the squared distance summed in FP32 as a direct
// difference.  Its error is multiplicative (the relative-error model of
// Sec. 5.2); the host turns that bound into two thresholds so that pairs
// outside [lo, hi) are decided for sure and the band in between is recomputed
// with the FP64 predicate.
#include <hip/hip_ext.h>

#include "dev_common.h"
#include "kernels.h"

namespace bm {

constexpr int RF_THREADS = 256;
constexpr int RF_LT = 32;      // landmarks per LDS tile
constexpr int RF_KC = 32;      // coordinates per chunk

__global__ __launch_bounds__(RF_THREADS) void k_range_fp32(const float *__restrict__ xf, PointsView P, double e2,
                                                           Fp32Thresholds thr, int refine,
                                                           const int32_t *__restrict__ A,
                                                           const int64_t *blk, RangeOut o, KernelClock *clk)
{
    clock_enter(clk);
    __shared__ float lt[RF_LT][RF_KC];
    __shared__ int32_t lrank[RF_LT];
    const int64_t ord0 = blk[0];
    const int na = (int)blk[1];
    const int d = P.d;
    const int64_t r = blockIdx.x * (int64_t)RF_THREADS + threadIdx.x;
    const bool valid = r < P.n;
    const int64_t xo = valid ? orig_index(P, r) : 0;
    const float *xr = xf + (valid ? r : 0) * (int64_t)d;
    bool cov = false;
    unsigned long long band = 0;

    float p[RF_KC];
    const bool one_chunk = d <= RF_KC;
    if (one_chunk) {
#pragma unroll
        for (int kk = 0; kk < RF_KC; ++kk) p[kk] = (valid && kk < d) ? xr[kk] : 0.f;
    }

    for (int a0 = 0; a0 < na; a0 += RF_LT) {
        const int nl = min(RF_LT, na - a0);
        __syncthreads();
        if (threadIdx.x < RF_LT) lrank[threadIdx.x] = (int)threadIdx.x < nl ? A[a0 + threadIdx.x] : 0;
        float acc[RF_LT];
#pragma unroll
        for (int l = 0; l < RF_LT; ++l) acc[l] = 0.f;
        for (int k0 = 0; k0 < d; k0 += RF_KC) {
            __syncthreads();
            for (int t = threadIdx.x; t < RF_LT * RF_KC; t += RF_THREADS) {
                const int l = t / RF_KC, kk = t % RF_KC, k = k0 + kk;
                lt[l][kk] = (l < nl && k < d) ? xf[(int64_t)lrank[l] * d + k] : 0.f;
            }
            __syncthreads();
            if (!one_chunk) {
#pragma unroll
                for (int kk = 0; kk < RF_KC; ++kk) p[kk] = (valid && k0 + kk < d) ? xr[k0 + kk] : 0.f;
            }
#pragma unroll 4
            for (int l = 0; l < RF_LT; ++l) {
                float a = acc[l];
#pragma unroll
                for (int kk = 0; kk < RF_KC; ++kk) {
                    const float t = p[kk] - lt[l][kk];
                    a = __builtin_fmaf(t, t, a);
                }
                acc[l] = a;
            }
        }
        for (int l = 0; l < nl; ++l) {
            const float sv = acc[l];
            bool mem = false;
            if (valid) {
                if (!refine) {
                    mem = sv < thr.unrefined;
                } else if (sv < thr.lo) {
                    mem = true;
                } else if (!(sv >= thr.hi)) {     // NaN hi: nothing is out for sure
                    ++band;
                    mem = exact_member(P, orig_index(P, lrank[l]), xo, e2);
                }
            }
            const unsigned long long pos = wave_append(o.nkeys, mem);
            if (mem) {
                cov = true;
                if (pos < o.cap) o.keys[pos] = ((uint64_t)(ord0 + a0 + l) << o.bn) | (uint64_t)xo | o.tag;
            }
        }
    }
    if (o.covered) {
        const uint64_t m = __ballot(cov);
        if (m && lane_id() == 0) atomicOr((unsigned long long *)&o.covered[r >> 6], (unsigned long long)m);
    }
    band = wave_sum(band);
    if (band && lane_id() == 0) atomicAdd(&o.st->band, band);
    if (clk) {
        __syncthreads();
        clock_leave(clk);
    }
}

hipError_t launch_range_fp32(const float *xf, const PointsView &P, double e2, Fp32Thresholds thr, int refine,
                             const int32_t *A, const int64_t *blk, int na_max, const RangeOut &o, hipStream_t s,
                             LaunchEvents ev)
{
    (void)na_max;
    if (P.n <= 0) return hipSuccess;
    const int blocks = (int)((P.n + RF_THREADS - 1) / RF_THREADS);
    if (ev.start || ev.stop)          // events attached to the dispatch (not capturable in a graph)
        hipExtLaunchKernelGGL(k_range_fp32, dim3(blocks), dim3(RF_THREADS), 0, s, ev.start, ev.stop, 0, xf, P, e2,
                              thr, refine, A, blk, o, ev.clock);
    else
        k_range_fp32<<<dim3(blocks), dim3(RF_THREADS), 0, s>>>(xf, P, e2, thr, refine, A, blk, o, ev.clock);
    return hipGetLastError();
}

} // namespace bm
