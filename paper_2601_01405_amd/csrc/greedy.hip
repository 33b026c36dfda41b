// greedy.hip — the blocked form of the greedy eps-net of Sec. 2.2.
//
// The sequential greedy visits ranks 0..n-1 and makes every still-uncovered
// rank a landmark.  Blocked, one step takes the next B uncovered ranks after
// the cursor (gather), decides among them with the exact predicate which ones
// the sequential greedy would accept (resolve + accept: candidate j is a
// landmark iff no earlier accepted candidate has j in its ball; all of them
// are uncovered by the landmarks of earlier blocks, whose range passes are
// complete), and then runs one range pass for the accepted ones.  Rejected
// candidates are members of an accepted one, so that pass covers them.
#include "dev_common.h"
#include "kernels.h"

namespace bm {

constexpr int GATHER_THREADS = 1024;

// One workgroup: scans the covered bitmap from the cursor, 64 ranks per thread
// per sweep, and lists up to B uncovered ranks in increasing order.
__global__ __launch_bounds__(GATHER_THREADS) void k_gather(const uint64_t *covered, int64_t n,
                                                           GreedyState *st, int B, int32_t *cand, int *rowflag)
{
    for (int j = threadIdx.x; j < B; j += GATHER_THREADS) rowflag[j] = 0;
    __shared__ int sh_scan[GATHER_THREADS / 64];
    __shared__ int64_t sh_cursor;
    const int64_t nwords = (n + 63) >> 6;
    int64_t cur = st->cursor;
    int count = 0;
    if (threadIdx.x == 0) sh_cursor = n;
    __syncthreads();
    while (cur < n && count < B) {
        const int64_t w0 = cur >> 6;
        const int64_t w = w0 + threadIdx.x;
        uint64_t m = 0;
        if (w < nwords) {
            m = ~covered[w];
            if (w == w0) m &= (~0ull) << (cur & 63);
            if (w == nwords - 1 && (n & 63)) m &= (1ull << (n & 63)) - 1;
        }
        int total;
        int pre = block_excl_scan<GATHER_THREADS>((int)__popcll(m), &total, sh_scan);
        const int room = B - count;
        int k = pre;
        while (m && k < room) {
            int b = __ffsll((unsigned long long)m) - 1;
            int64_t r = (w << 6) + b;
            cand[count + k] = (int32_t)r;
            if (count + k == B - 1) sh_cursor = r + 1;
            m &= m - 1;
            ++k;
        }
        if (total >= room) {
            count = B;
        } else {
            count += total;
            cur = (w0 + GATHER_THREADS) << 6;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->nc = count;
        st->na = 0;
        st->cursor = (count == B) ? sh_cursor : n;
        if (count == 0) st->done = 1;
        else {
            st->blocks += 1;
            st->candidates += (unsigned long long)count;
            st->resolve_pairs += (unsigned long long)count * (unsigned long long)(count - 1) / 2;
        }
    }
}

hipError_t launch_gather(const uint64_t *covered, int64_t n, GreedyState *st, int B, int32_t *cand,
                         int *rowflag, hipStream_t s)
{
    k_gather<<<1, GATHER_THREADS, 0, s>>>(covered, n, st, B, cand, rowflag);
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

// Acceptance in rank order, by rounds: a candidate without any earlier
// conflict (rowflag 0) is accepted at once; otherwise it is rejected as soon
// as one of its earlier conflicts is accepted, and accepted once all of them
// are rejected.  Decisions never change, so a stale view only delays one; the
// earliest undecided candidate always has all its conflicts decided, so every
// round decides at least one.  The result equals the sequential scan.
constexpr int ACCEPT_THREADS = 1024;
constexpr int MAX_B = 4096;

__global__ __launch_bounds__(ACCEPT_THREADS) void k_accept(const uint64_t *C, const int *rowflag, int nw,
                                                           const int32_t *cand, GreedyState *st, int32_t *A,
                                                           int32_t *landmarks, int32_t *lm_rank, BlockLog *blog,
                                                           const int32_t *perm, uint64_t *islm, int64_t n)
{
    const int64_t L0 = st->L;
    __shared__ unsigned long long acc[MAX_B / 64], rej[MAX_B / 64];
    __shared__ int sh_undecided, sh_scan[ACCEPT_THREADS / 64];
    const int nc = st->nc;
    for (int t = threadIdx.x; t < MAX_B / 64; t += blockDim.x) acc[t] = rej[t] = 0ull;
    __syncthreads();
    unsigned long long rounds = 0;
    for (;;) {
        if (threadIdx.x == 0) sh_undecided = 0;
        __syncthreads();
        for (int j = threadIdx.x; j < nc; j += blockDim.x) {
            const int wj = j >> 6;
            const unsigned long long bit = 1ull << (j & 63);
            if ((acc[wj] | rej[wj]) & bit) continue;
            if (!rowflag[j]) {
                atomicOr(&acc[wj], bit);
                continue;
            }
            bool any_acc = false, any_open = false;
            const int nwj = (j + 63) >> 6;       // words holding candidates < j
            for (int w = 0; w < nwj && !any_acc; ++w) {
                unsigned long long c = C[(int64_t)j * nw + w];
                if (w == wj) c &= bit - 1ull;     // only candidates i < j (the rest of the word is not written)
                unsigned long long a = __atomic_load_n(&acc[w], __ATOMIC_RELAXED);
                unsigned long long r = __atomic_load_n(&rej[w], __ATOMIC_RELAXED);
                if (c & a) any_acc = true;
                else if (c & ~(a | r)) any_open = true;
            }
            if (any_acc) atomicOr(&rej[wj], bit);
            else if (!any_open) atomicOr(&acc[wj], bit);
            else sh_undecided = 1;
        }
        __syncthreads();
        ++rounds;
        const int und = sh_undecided;
        __syncthreads();
        if (!und) break;
        if (rounds > (unsigned long long)nc) {   // every round decides one candidate: cannot happen
            if (threadIdx.x == 0) st->error = 1;
            break;
        }
    }
    // compaction of the accepted candidates, in rank order
    int total = 0;
    int mine = 0;
    const int per = (nc + ACCEPT_THREADS - 1) / ACCEPT_THREADS;   // candidates per thread, contiguous
    const int j0 = threadIdx.x * per;
    for (int j = j0; j < j0 + per && j < nc; ++j) mine += (int)((acc[j >> 6] >> (j & 63)) & 1ull);
    int pos = block_excl_scan<ACCEPT_THREADS>(mine, &total, sh_scan);
    for (int j = j0; j < j0 + per && j < nc; ++j) {
        if ((acc[j >> 6] >> (j & 63)) & 1ull) {
            const int32_t r = cand[j];
            A[pos] = r;
            landmarks[L0 + pos] = perm ? perm[r] : r;
            lm_rank[L0 + pos] = r;
            if (islm) atomicOr((unsigned long long *)&islm[r >> 6], 1ull << (r & 63));
            ++pos;
        }
    }
    if (threadIdx.x == 0) {
        st->L0 = L0;
        st->na = total;
        st->L = L0 + total;
        st->rounds += rounds;
        st->range_pairs += (unsigned long long)total * (unsigned long long)(st->m + n - st->rlo);
        if (nc > 0) {
            BlockLog &b = blog[(st->blocks - 1) % kBlockLogSize];
            b.L0 = L0;
            b.na = total;
            b.rlo = st->rlo;
            b.m = st->m;
            b.nkeys_before = st->nkeys;
        }
    }
}

hipError_t launch_accept(const uint64_t *C, const int *rowflag, const int32_t *cand, GreedyState *st, int B,
                         int32_t *A, int32_t *landmarks, int32_t *lm_rank, BlockLog *blog, const int32_t *perm,
                         uint64_t *islm, int64_t n, hipStream_t s)
{
    if (B > MAX_B) return hipErrorInvalidValue;
    k_accept<<<1, ACCEPT_THREADS, 0, s>>>(C, rowflag, (B + 63) / 64, cand, st, A, landmarks, lm_rank, blog, perm,
                                          islm, n);
    return hipGetLastError();
}

// Settling, run after a gather: every rank below the new block's first
// candidate is final (a landmark, or covered and never a landmark).  The
// non-landmarks among ranks [rlo, R), R = that candidate rounded down to a
// tile, are appended in rank order to the settled list (their point-side
// operands, thresholds and original index), and rlo becomes R.
constexpr int SETTLE_THREADS = 1024;

__global__ __launch_bounds__(SETTLE_THREADS) void k_settle(const uint64_t *islm, GreedyState *st, const int32_t *cand,
                                                           MfmaArgs a, SettledSet out, const int32_t *perm)
{
    __shared__ int sh_scan[SETTLE_THREADS / 64];
    __shared__ int32_t sel[SETTLE_THREADS];
    const int nc = st->nc;
    if (nc == 0) return;                                   // workgroup-uniform
    const int64_t R0 = st->rlo;
    const int64_t R1 = ((int64_t)cand[0] >> 5) << 5;
    int64_t m = st->m;
    const int S = a.S, nvec = 2 * S;
    for (int64_t r0 = R0; r0 < R1; r0 += SETTLE_THREADS) {
        const int64_t r = r0 + threadIdx.x;
        const bool take = r < R1 && !((islm[r >> 6] >> (r & 63)) & 1ull);
        int total;
        const int pre = block_excl_scan<SETTLE_THREADS>((int)take, &total, sh_scan);
        if (take) {
            const int64_t j = m + pre;
            sel[pre] = (int32_t)r;
#pragma unroll
            for (int w = 0; w < 3; ++w) out.T3[t3_index(j, w)] = a.T3[t3_index(r, w)];
            out.idx[j] = perm ? perm[r] : (int32_t)r;
        }
        __syncthreads();
        for (int v = threadIdx.x; v < total * nvec; v += SETTLE_THREADS) {
            const int q = v / nvec, rem = v - q * nvec, ss = rem >> 1, half = rem & 1;
            const int64_t src = sel[q], dst = m + q;
            const int64_t so = ((((src >> 5) * S + ss) * 64) + (src & 31) + 32 * half) * 8;
            const int64_t dof = ((((dst >> 5) * S + ss) * 64) + (dst & 31) + 32 * half) * 8;
            *(u32x4 *)(out.Pop + dof) = *(const u32x4 *)(a.Pop + so);
        }
        m += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->rlo = R1;
        st->m = m;
    }
}

hipError_t launch_settle(const uint64_t *islm, GreedyState *st, const int32_t *cand, const MfmaArgs &a,
                         const SettledSet &out, const int32_t *perm, hipStream_t s)
{
    k_settle<<<1, SETTLE_THREADS, 0, s>>>(islm, st, cand, a, out, perm);
    return hipGetLastError();
}

} // namespace bm
