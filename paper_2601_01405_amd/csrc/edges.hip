// edges.hip — edges of the Ball Mapper graph, the 1-skeleton of the nerve
// (Sec. 2.1): (i, j) with i < j whenever the balls of landmarks i and j share a
// data point.
//
// Built through the transpose of the membership CSR: S(x) lists the landmarks
// whose ball holds x, and the neighbours j > i of landmark i are the union of
// S(x) over x in its ball.  Only rows with a member in some other ball are
// visited (a work list built first); the others have no edge.  One workgroup per landmark deduplicates that union
// either by sorting it in LDS (small unions) or with an LDS bitmap over the
// range of j (large unions).  Rows come out in landmark order and each row in
// increasing j, so the list is lexicographic without a global sort.
#include <climits>
#include <cstring>
#include <rocprim/device/device_scan.hpp>

#include "dev_common.h"
#include "kernels.h"

namespace bm {

__global__ void k_zero_i64(int64_t *p, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// out[0] = 0, out[1 + i] = in[0] + ... + in[i]  (count + 1 outputs)
hipError_t scan_excl_i64(void *tmp, size_t *tmp_bytes, const int64_t *in, int64_t *out, size_t count, hipStream_t s)
{
    size_t bytes = *tmp_bytes;
    hipError_t e;
    if (count == 0) {
        e = hipSuccess;
        bytes = bytes ? bytes : 16;
    } else {
        e = rocprim::inclusive_scan(tmp, bytes, in, out + 1, count, rocprim::plus<int64_t>(), s);
    }
    if (tmp != nullptr && e == hipSuccess) {
        k_zero_i64<<<1, 64, 0, s>>>(out, 1);
        e = hipGetLastError();
    }
    *tmp_bytes = bytes;
    return e;
}

__global__ void k_point_degree(const int32_t *member_idx, int64_t M, int64_t *cnt)
{
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < M; m += (int64_t)gridDim.x * blockDim.x)
        atomicAdd((unsigned long long *)&cnt[member_idx[m]], 1ull);
}

hipError_t launch_point_degree(const int32_t *member_idx, int64_t M, int64_t *cnt, hipStream_t s)
{
    if (M <= 0) return hipSuccess;
    int64_t blocks = (M + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_point_degree<<<(int)blocks, 256, 0, s>>>(member_idx, M, cnt);
    return hipGetLastError();
}

__global__ void k_fill_slists(const uint64_t *keys, int64_t M, int32_t bn, const int64_t *sptr, int64_t *sfill,
                              int32_t *slist)
{
    const uint64_t mask = (1ull << bn) - 1;
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < M; m += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[m];
        const int64_t x = (int64_t)(k & mask);
        const int32_t i = (int32_t)(k >> bn);
        const int64_t pos = sptr[x] + (int64_t)atomicAdd((unsigned long long *)&sfill[x], 1ull);
        slist[pos] = i;
    }
}

hipError_t launch_fill_slists(const uint64_t *keys, int64_t M, int32_t bn, const int64_t *sptr, int64_t *sfill,
                              int32_t *slist, hipStream_t s)
{
    if (M <= 0) return hipSuccess;
    int64_t blocks = (M + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_fill_slists<<<(int)blocks, 256, 0, s>>>(keys, M, bn, sptr, sfill, slist);
    return hipGetLastError();
}

constexpr int EP_THREADS = 256;
constexpr int EP_CAP = 2048;                    // union sizes sorted in LDS
constexpr int EP_WORDS = 4096;                  // bitmap words per chunk (262144 landmarks, 32 KB)

// Rows that can have an edge: some member x of row i lies in another ball
// (|S(x)| > 1).  flag[] must start at zero.
__global__ void k_flag_rows(const uint64_t *keys, int64_t M, int32_t bn, const int64_t *sptr, int *flag)
{
    const uint64_t mask = (1ull << bn) - 1;
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < M; m += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[m];
        const int64_t x = (int64_t)(k & mask);
        if (sptr[x + 1] - sptr[x] > 1) flag[k >> bn] = 1;
    }
}

// The flagged rows, in no particular order: list[0 .. *count).
__global__ void k_list_rows(const int *flag, int64_t L, int32_t *list, unsigned long long *count)
{
    for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x; i0 < L; i0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = i0 + threadIdx.x;
        const bool want = i < L && flag[i] != 0;
        const unsigned long long pos = wave_append(count, want);
        if (want) list[pos] = (int32_t)i;
    }
}

hipError_t launch_edge_rows(const uint64_t *keys, int64_t M, int32_t bn, const int64_t *sptr, int64_t L, int *flag,
                            int32_t *list, unsigned long long *count, hipStream_t s)
{
    if (L <= 0) return hipSuccess;
    int64_t blocks = (M + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (M > 0) k_flag_rows<<<(int)blocks, 256, 0, s>>>(keys, M, bn, sptr, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    blocks = (L + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_list_rows<<<(int)blocks, 256, 0, s>>>(flag, L, list, count);
    return hipGetLastError();
}

// The union of S(x) over the members x of row i is walked as one flattened
// sequence: members are taken EP_THREADS at a time, their list lengths scanned
// into LDS offsets, and thread e of the workgroup reads entry e, e + EP_THREADS,
// ... of the concatenated lists (a binary search in the offsets finds its
// member), so the loads of consecutive threads are consecutive in slist and
// many are in flight.  visit(j) is called for every entry j > i.
template <class F>
__device__ __forceinline__ void walk_union(int32_t i, int64_t m0, int64_t m1, const int32_t *member_idx,
                                           const int64_t *sptr, const int32_t *slist, int64_t *sh_off,
                                           int64_t *sh_s0, int64_t *sh_scan, F &&visit)
{
    const int tid = (int)threadIdx.x;
    for (int64_t mc = m0; mc < m1; mc += EP_THREADS) {
        const int64_t m = mc + tid;
        int64_t s0 = 0, len = 0;
        if (m < m1) {
            const int32_t x = member_idx[m];
            s0 = sptr[x];
            len = sptr[x + 1] - s0;
        }
        int64_t tot;
        const int64_t off = block_excl_scan<EP_THREADS>(len, &tot, sh_scan);
        sh_off[tid] = off;
        sh_s0[tid] = s0;
        __syncthreads();
        const int nm = (int)min<int64_t>(EP_THREADS, m1 - mc);
        // entry e's member: the last one with offset <= e; e grows by
        // EP_THREADS per step, so each thread advances its own cursor (a few
        // members per step) instead of searching the offsets again
        // (eight entries per step: their loads are all in flight before the
        // first visit; the last step reads in-bounds repeats it ignores)
        int lo = 0;
        int64_t next_off = nm > 1 ? sh_off[1] : INT64_MAX;
        constexpr int U = 8;
        for (int64_t e = tid; e < tot; e += U * EP_THREADS) {
            int32_t jv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t eu = min(e + (int64_t)u * EP_THREADS, tot - 1);
                while (next_off <= eu) {
                    ++lo;
                    next_off = lo + 1 < nm ? sh_off[lo + 1] : INT64_MAX;
                }
                jv[u] = slist[sh_s0[lo] + (eu - sh_off[lo])];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (e + (int64_t)u * EP_THREADS < tot && jv[u] > i) visit(jv[u]);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(EP_THREADS) void k_edge_pass(int mode, const int32_t *rows, int64_t L,
                                                          const int64_t *seg, int nseg, const int64_t *row_ptr,
                                                          const int32_t *member_idx, const int64_t *sptr,
                                                          const int32_t *slist, int64_t *deg, const int64_t *eptr,
                                                          int32_t *edges, EdgeStore store)
{
    __shared__ int32_t buf[EP_CAP];
    __shared__ unsigned long long bits[EP_WORDS];
    __shared__ int sh_cnt;
    __shared__ int64_t sh_slot;
    __shared__ int64_t sh_scan[EP_THREADS / 64];
    __shared__ int64_t sh_off[EP_THREADS], sh_s0[EP_THREADS];
    const int32_t i = rows ? rows[blockIdx.x] : (int32_t)blockIdx.x;
    const int64_t m0 = row_ptr[i], m1 = row_ptr[i + 1];
    const int tid = (int)threadIdx.x;
    // neighbours of row i lie in its segment [seg[c], seg[c + 1]) (a batch's
    // chain), or anywhere below L
    int64_t jend = L;
    if (nseg > 0) {
        int lo = 0, hi = nseg - 1;                                  // last c with seg[c] <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (seg[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        jend = seg[lo + 1];
    }
    // upper bound of the union (with repeats and entries <= i) from the list lengths
    int64_t ub = 0;
    for (int64_t m = m0 + tid; m < m1; m += EP_THREADS) {
        const int32_t x = member_idx[m];
        ub += sptr[x + 1] - sptr[x];
    }
    int64_t bound;
    (void)block_excl_scan<EP_THREADS>(ub, &bound, sh_scan);
    const int64_t out0 = (mode == 1) ? eptr[i] : 0;
    if (bound <= EP_CAP) {
        // gather, bitonic sort, keep the first of each run
        if (tid == 0) sh_cnt = 0;
        __syncthreads();
        walk_union(i, m0, m1, member_idx, sptr, slist, sh_off, sh_s0, sh_scan,
                   [&](int32_t j) { buf[atomicAdd(&sh_cnt, 1)] = j; });
        const int total = sh_cnt;
        if (total == 0) {
            if (mode == 0 && tid == 0) deg[i] = 0;
            return;
        }
        int P2 = 2;
        while (P2 < total) P2 <<= 1;
        for (int t = total + tid; t < P2; t += EP_THREADS) buf[t] = INT_MAX;
        __syncthreads();
        for (int k = 2; k <= P2; k <<= 1) {
            for (int jj = k >> 1; jj > 0; jj >>= 1) {
                for (int t = tid; t < P2; t += EP_THREADS) {
                    const int u = t ^ jj;
                    if (u > t) {
                        const int32_t a = buf[t], b = buf[u];
                        const bool up = (t & k) == 0;
                        if ((a > b) == up) {
                            buf[t] = b;
                            buf[u] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        // each thread owns a contiguous slice so positions follow the sorted order
        const int per = (total + EP_THREADS - 1) / EP_THREADS;
        const int t0 = tid * per;
        int64_t mine = 0;
        for (int t = t0; t < t0 + per && t < total; ++t) mine += (t == 0 || buf[t] != buf[t - 1]);
        int64_t uniq;
        int64_t pos = block_excl_scan<EP_THREADS>(mine, &uniq, sh_scan);
        if (mode == 0) {
            if (tid == 0) deg[i] = uniq;
        } else {
            for (int t = t0; t < t0 + per && t < total; ++t) {
                if (t == 0 || buf[t] != buf[t - 1]) {
                    edges[2 * (out0 + pos)] = i;
                    edges[2 * (out0 + pos) + 1] = buf[t];
                    ++pos;
                }
            }
        }
        return;
    }
    // bitmap over j in (i, jend) in chunks of EP_WORDS * 64 landmarks.  The
    // counting pass keeps the row's bitmap in a slot of `store` while slots
    // last (slots[b] records which); the emitting pass reads a kept bitmap
    // back instead of walking the union again.
    const int b = (int)blockIdx.x;
    if (tid == 0) {
        int64_t slot = -1;
        if (mode == 0) {
            if (store.bits) {
                const unsigned long long t = atomicAdd(store.count, 1ull);
                if ((int64_t)t < store.cap) slot = (int64_t)t;
            }
            if (store.slots) store.slots[b] = (int32_t)slot;
        } else if (store.slots) {
            slot = store.slots[b];
        }
        sh_slot = slot;
    }
    __syncthreads();
    uint64_t *kept = sh_slot >= 0 ? store.bits + sh_slot * store.words : nullptr;
    int64_t written = 0;
    for (int64_t base = (int64_t)i + 1; base < jend; base += (int64_t)EP_WORDS * 64) {
        const int64_t span = min((int64_t)EP_WORDS * 64, jend - base);
        const int nwords = (int)((span + 63) >> 6);
        const int64_t wofs = (base - (int64_t)i - 1) >> 6;
        if (mode == 1 && kept) {
            for (int t = tid; t < nwords; t += EP_THREADS) bits[t] = kept[wofs + t];
            __syncthreads();
        } else {
            for (int t = tid; t < nwords; t += EP_THREADS) bits[t] = 0ull;
            __syncthreads();
            walk_union(i, m0, m1, member_idx, sptr, slist, sh_off, sh_s0, sh_scan, [&](int32_t j) {
                const int64_t r = (int64_t)j - base;
                if (r >= 0 && r < span) atomicOr(&bits[r >> 6], 1ull << (r & 63));
            });
            if (mode == 0 && kept)
                for (int t = tid; t < nwords; t += EP_THREADS) kept[wofs + t] = bits[t];
        }
        const int per = (nwords + EP_THREADS - 1) / EP_THREADS;
        const int w0 = tid * per;
        int64_t mine = 0;
        for (int w = w0; w < w0 + per && w < nwords; ++w) mine += __popcll(bits[w]);
        int64_t chunk_total;
        int64_t pos = block_excl_scan<EP_THREADS>(mine, &chunk_total, sh_scan);
        if (mode == 1) {
            for (int w = w0; w < w0 + per && w < nwords; ++w) {
                unsigned long long bb = bits[w];
                while (bb) {
                    const int bit = __ffsll(bb) - 1;
                    bb &= bb - 1;
                    edges[2 * (out0 + written + pos)] = i;
                    edges[2 * (out0 + written + pos) + 1] = (int32_t)(base + (w << 6) + bit);
                    ++pos;
                }
            }
        }
        written += chunk_total;
        __syncthreads();
    }
    if (mode == 0 && tid == 0) deg[i] = written;
}

hipError_t launch_edge_pass(int mode, int64_t nrows, const int32_t *rows, int64_t L, const int64_t *seg, int nseg,
                            const int64_t *row_ptr, const int32_t *member_idx, const int64_t *sptr,
                            const int32_t *slist, int64_t *deg, const int64_t *eptr, int32_t *edges,
                            const EdgeStore &store, hipStream_t s)
{
    if (nrows <= 0) return hipSuccess;
    k_edge_pass<<<(unsigned)nrows, EP_THREADS, 0, s>>>(mode, rows, L, seg, nseg, row_ptr, member_idx, sptr, slist,
                                                       deg, eptr, edges, store);
    return hipGetLastError();
}

} // namespace bm
