// dev_common.h — device helpers for the gfx950 kernels (wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bm_internal.h"

namespace bm {

typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

// ---- global-memory access ------------------------------------------------------------
// A pointer read from a task table (rather than passed as a kernel argument)
// reaches the compiler as a generic pointer, accessed with FLAT instructions.
// Those count in the same wait counter as LDS operations, so every wait for an
// LDS read or a lane shuffle would also wait for all global loads in flight
// (the prefetched stages of a pass).  Every array this library hands to a
// kernel is global memory; gbl() says so, and the accesses become global ones.
#define BM_GLOBAL __attribute__((address_space(1)))
template <class T> __device__ __forceinline__ BM_GLOBAL T *gbl(T *p) { return (BM_GLOBAL T *)p; }
template <class T> __device__ __forceinline__ T gatomic_add(T *p, T v)
{
    return __hip_atomic_fetch_add(gbl(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T> __device__ __forceinline__ T gatomic_or(T *p, T v)
{
    return __hip_atomic_fetch_or(gbl(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- exact widening of a stored coordinate -------------------------------------------
template <int DT>
__device__ __forceinline__ double load_coord(const void *X, int64_t off)
{
    if constexpr (DT == 0) return ((const BM_GLOBAL double *)X)[off];
    else if constexpr (DT == 1) return (double)((const BM_GLOBAL float *)X)[off];
    else return (double)(float)((const BM_GLOBAL _Float16 *)X)[off];   // binary16 -> f32 -> f64, exact
}

__device__ __forceinline__ int64_t orig_index(const PointsView &P, int64_t rank)
{
    return P.perm ? (int64_t)gbl(P.perm)[rank] : rank;
}

// ---- the FP64 predicate --------------------------------------------------------------
// s(a,b) = sum over k of RN(RN(a_k - b_k)^2), added left to right with round to
// nearest and no fused multiply-add; member iff s < e2 = RN(eps^2).  The two
// rows are read in chunks of 8 coordinates (independent loads in flight) and
// the terms are then added strictly in order k = 0, 1, ..., d-1.  (No early
// exit: pairs reach this recheck only near the threshold, and the decision
// does not depend on it.)
template <int DT>
__device__ __forceinline__ void load8(const void *X, int64_t off, int valid, double *v)
{
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = e < valid ? load_coord<DT>(X, off + e) : 0.0;
}

template <int DT>
__device__ __forceinline__ bool exact_member_t(const void *X, int32_t d, int64_t a, int64_t b,
                                                         double e2)
{
#pragma clang fp contract(off)
    const int64_t oa = a * (int64_t)d, ob = b * (int64_t)d;
    double acc = 0.0;
    for (int32_t k0 = 0; k0 < d; k0 += 8) {
        const int valid = min(8, d - k0);
        double va[8], vb[8];
        load8<DT>(X, oa + k0, valid, va);
        load8<DT>(X, ob + k0, valid, vb);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if (e < valid) {
                const double t = va[e] - vb[e];
                const double sq = t * t;
                acc = acc + sq;
            }
        }
    }
    return acc < e2;
}

// a, b: ORIGINAL row indices.
__device__ __forceinline__ bool exact_member(const PointsView &P, int64_t a, int64_t b, double e2)
{
    if (P.dtype == 0) return exact_member_t<0>(P.X, P.d, a, b, e2);
    if (P.dtype == 1) return exact_member_t<1>(P.X, P.d, a, b, e2);
    return exact_member_t<2>(P.X, P.d, a, b, e2);
}

// ---- kernel execution window (see KernelClock) ------------------------------------------
__device__ __forceinline__ void clock_enter(KernelClock *clk)
{
    if (clk && threadIdx.x == 0) atomicMin(&clk->start, (unsigned long long)wall_clock64());
}
// Called by every workgroup once all its threads are done (after a barrier).
// Only atomics touch the clock, so no fence is needed.
__device__ __forceinline__ void clock_leave(KernelClock *clk)
{
    if (!clk || threadIdx.x != 0) return;
    const unsigned long long prev = atomicAdd(&clk->done, 1ull);
    if (prev == (unsigned long long)gridDim.x * gridDim.y * gridDim.z - 1ull) {
        const unsigned long long st = atomicAdd(&clk->start, 0ull);
        const unsigned long long now = (unsigned long long)wall_clock64();
        atomicAdd(&clk->ticks, now - st);
        atomicExch(&clk->start, ~0ull);
        atomicExch(&clk->done, 0ull);
    }
}

// ---- wave64 helpers ------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ int mbcnt(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Wave-aggregated append: every lane with `want` gets a distinct slot; one atomic per wave.
__device__ __forceinline__ unsigned long long wave_append(unsigned long long *counter, bool want,
                                                          uint64_t *ballot_out = nullptr)
{
    uint64_t m = __ballot(want);
    if (ballot_out) *ballot_out = m;
    if (!m) return 0;
    int leader = __ffsll((unsigned long long)m) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (unsigned long long)__popcll(m));
    base = __shfl(base, leader, 64);
    return base + (unsigned long long)mbcnt(m);
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Exclusive scan over a whole workgroup of BLOCK threads. `sh` holds BLOCK/64 values.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *total, T *sh)
{
    constexpr int NW = BLOCK / 64;
    const int lane = lane_id(), wid = (int)(threadIdx.x >> 6);
    T x = wave_incl_scan(v);
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    if (wid == 0) {
        T s = lane < NW ? sh[lane] : T(0);
        s = wave_incl_scan(s);
        if (lane < NW) sh[lane] = s;
    }
    __syncthreads();
    T off = wid ? sh[wid - 1] : T(0);
    *total = sh[NW - 1];
    __syncthreads();
    return off + x - v;
}

} // namespace bm
