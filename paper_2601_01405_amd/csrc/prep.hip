// prep.hip — one streaming pass over the stored points: finiteness check,
// FP64 squared norms (Sec. 3.2 precomputes d^2(x,0) once per point), range
// statistics for the error bounds, and the FP32 copy used by the plain path.
#include "dev_common.h"
#include "kernels.h"

namespace bm {

template <int DT>
__global__ void k_check_finite(const void *X, int64_t count, int *bad)
{
    int found = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        double v = load_coord<DT>(X, i);
        found |= !__builtin_isfinite(v);
    }
    if (__ballot(found) && lane_id() == 0) atomicOr(bad, 1);
}

hipError_t launch_check_finite(const void *X, int32_t dtype, int64_t count, int *bad, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (dtype == 0) k_check_finite<0><<<(int)blocks, 256, 0, s>>>(X, count, bad);
    else if (dtype == 1) k_check_finite<1><<<(int)blocks, 256, 0, s>>>(X, count, bad);
    else k_check_finite<2><<<(int)blocks, 256, 0, s>>>(X, count, bad);
    return hipGetLastError();
}

// Non-negative doubles order like their bit patterns, so a 64-bit atomicMax keeps the maximum.
// The slot only grows, so a value not above what it already holds cannot change it: the
// atomic (serialised with every other one on the address) is skipped then.
__device__ __forceinline__ void atomic_max_nonneg(unsigned long long *slot, double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (b > __hip_atomic_load(gbl(slot), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(slot, b);
}

// Grid-stride over the points; the maxima are reduced per workgroup first, so
// that only two atomics per workgroup reach the two counters (atomics on one
// address are serialised).
constexpr int PS_THREADS = 256;
template <int DT>
__global__ __launch_bounds__(PS_THREADS) void k_point_stats(PointsView P, double *nu, unsigned long long *stats)
{
    __shared__ double sh[2][PS_THREADS / 64];
    double smax = 0.0, mabs = 0.0;
    // float32 rows of a multiple of 4 coordinates on a 16-byte aligned array are
    // read 4 at a time (a quarter of the load instructions; the same products
    // added in the same order)
    const bool vec4 = DT == 1 && (P.d & 3) == 0 && ((uintptr_t)P.X & 15u) == 0;   // uniform
    for (int64_t r = blockIdx.x * (int64_t)PS_THREADS + threadIdx.x; r < P.n; r += (int64_t)gridDim.x * PS_THREADS) {
        const int64_t o = orig_index(P, r) * (int64_t)P.d;
        double s = 0.0;
        if (vec4) {
            const BM_GLOBAL u32x4 *row = (const BM_GLOBAL u32x4 *)((const BM_GLOBAL float *)P.X + o);
            for (int32_t k4 = 0; k4 < (P.d >> 2); ++k4) {
                const u32x4 q = row[k4];
                const double v[4] = {(double)__uint_as_float(q[0]), (double)__uint_as_float(q[1]),
                                     (double)__uint_as_float(q[2]), (double)__uint_as_float(q[3])};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    s = __fma_rn(v[e], v[e], s);
                    mabs = fmax(mabs, fabs(v[e]));
                }
            }
        } else {
            for (int32_t k = 0; k < P.d; ++k) {
                double v = load_coord<DT>(P.X, o + k);
                s = __fma_rn(v, v, s);
                mabs = fmax(mabs, fabs(v));
            }
        }
        gbl(nu)[r] = s;
        smax = fmax(smax, s);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        smax = fmax(smax, __shfl_xor(smax, off, 64));
        mabs = fmax(mabs, __shfl_xor(mabs, off, 64));
    }
    const int wid = (int)(threadIdx.x >> 6);
    if (lane_id() == 0) {
        sh[0][wid] = smax;
        sh[1][wid] = mabs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < PS_THREADS / 64; ++w) {
            smax = fmax(smax, sh[0][w]);
            mabs = fmax(mabs, sh[1][w]);
        }
        atomic_max_nonneg(&stats[0], smax);
        atomic_max_nonneg(&stats[1], mabs);
    }
}

hipError_t launch_point_stats(const PointsView &P, double *nu, unsigned long long *stats, hipStream_t s)
{
    if (P.n <= 0) return hipSuccess;
    int64_t blocks = (P.n + PS_THREADS - 1) / PS_THREADS;
    if (blocks > 1024) blocks = 1024;
    if (P.dtype == 0) k_point_stats<0><<<(int)blocks, PS_THREADS, 0, s>>>(P, nu, stats);
    else if (P.dtype == 1) k_point_stats<1><<<(int)blocks, PS_THREADS, 0, s>>>(P, nu, stats);
    else k_point_stats<2><<<(int)blocks, PS_THREADS, 0, s>>>(P, nu, stats);
    return hipGetLastError();
}

template <int DT>
__global__ void k_to_f32(PointsView P, float *xf)
{
    const int64_t total = P.n * (int64_t)P.d;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i / P.d, k = i - r * P.d;
        xf[i] = (float)load_coord<DT>(P.X, orig_index(P, r) * (int64_t)P.d + k);
    }
}

hipError_t launch_to_f32(const PointsView &P, float *xf, hipStream_t s)
{
    const int64_t total = P.n * (int64_t)P.d;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (P.dtype == 0) k_to_f32<0><<<(int)blocks, 256, 0, s>>>(P, xf);
    else if (P.dtype == 1) k_to_f32<1><<<(int)blocks, 256, 0, s>>>(P, xf);
    else k_to_f32<2><<<(int)blocks, 256, 0, s>>>(P, xf);
    return hipGetLastError();
}

} // namespace bm
