// greedy_dev.h — the two serial steps of one block of the blocked greedy
// (Sec. 2.2), each run by one workgroup of NT threads: as kernels of their own
// (greedy.hip) or by the last workgroup of a matrix-core launch of the same
// chain (range_mfma.hip), which saves a kernel boundary per step.
//
// The sequential greedy visits ranks 0..n-1 and makes every still-uncovered
// rank a landmark.  Blocked, one step takes the next B uncovered ranks after
// the cursor (open), decides among them with the exact predicate which ones
// the sequential greedy would accept (resolve + accept: candidate j is a
// landmark iff no earlier accepted candidate has j in its ball; all of them
// are uncovered by the landmarks of earlier blocks, whose range passes are
// complete), and then runs one range pass for the accepted ones.  Rejected
// candidates are members of an accepted one, so that pass covers them.
#pragma once
#include "dev_common.h"

namespace bm {

constexpr int MAX_B = kMaxBlock;

// LDS bytes the steps use (from a caller-provided, 16-byte aligned buffer).
template <int NT> constexpr size_t open_lds_bytes()
{
    return 16 + (size_t)NT / 64 * 4 + (size_t)MAX_B * 4;
}
template <int NT> constexpr size_t accept_lds_bytes()
{
    return (size_t)MAX_B / 64 * 16 + 16 + ((size_t)MAX_B / 64 + 4) * 4 + (size_t)MAX_B * 2;
}

// Exclusive prefix of per-wave counts in (k, wave) order, for a workgroup whose
// thread t holds items k * NT + t (k < RUN).  Before the call, lane 0 of each
// wave has written its count of item row k to tab[k * NT / 64 + wave] (after a
// barrier that ended tab's previous use).  On return tab holds the bases,
// tab[RUN * NT / 64] the total, which is returned.
template <int NT, int RUN>
__device__ int slot_scan(int *tab)
{
    constexpr int NW = NT / 64, E = RUN * NW, PER = (E + 63) / 64;
    static_assert(E <= MAX_B / 64, "at most one entry per bitmap word");
    const int lane = lane_id(), wid = (int)(threadIdx.x >> 6);
    __syncthreads();
    if (wid == 0) {
        int v[PER], sum = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = lane * PER + i;
            v[i] = e < E ? tab[e] : 0;
            sum += v[i];
        }
        const int incl = wave_incl_scan(sum);
        int run = incl - sum;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = lane * PER + i;
            if (e < E) tab[e] = run;
            run += v[i];
        }
        if (lane == 63) tab[E] = incl;
    }
    __syncthreads();
    return tab[E];
}

// Open a block of chain T:
//  1. Gather: scan the covered bitmap from the cursor, 64 ranks per thread per
//     sweep, and list up to B uncovered ranks in increasing order (in LDS,
//     then copied out coalesced); clear rowflag[0..B).
//  2. (settle) Every rank below the first candidate is final (a landmark, or
//     covered and never a landmark).  The non-landmarks among ranks [rlo, R),
//     R = that candidate rounded down to a tile, are appended in rank order to
//     the settled list (point-side operands, thresholds, original index), and
//     rlo becomes R.
// A chain whose gather finds nothing is done (counted once in *ndone); a done
// chain opens empty blocks (nc = na = 0) that every later step skips.
template <int NT>
__device__ void block_open(const ChainTask &T, unsigned char *lds)
{
    int64_t *sh_cursor = (int64_t *)lds;
    int32_t *sh_first = (int32_t *)(lds + 8);
    int *sh_scan = (int *)(lds + 16);
    int32_t *clist = (int32_t *)(lds + 16 + NT / 64 * 4);       // [MAX_B] the gathered ranks
    const int tid = (int)threadIdx.x;
    BM_GLOBAL GreedyState *st = gbl(T.st);
    const int64_t n = T.n;
    const int B = T.B;
    if (st->done) {                                              // workgroup-uniform
        if (tid == 0) {
            st->nc = 0;
            st->na = 0;
        }
        return;
    }
    for (int j = tid; j < B; j += NT) gbl(T.rowflag)[j] = 0;
    const int64_t nwords = (n + 63) >> 6;
    int64_t cur = st->cursor;
    const int64_t R0 = st->rlo;
    int64_t m = st->m;
    int count = 0;
    if (tid == 0) {
        *sh_cursor = n;
        *sh_first = 0;
    }
    __syncthreads();
    while (cur < n && count < B) {                               // uniform: count, cur from scan totals
        const int64_t w0 = cur >> 6;
        const int64_t w = w0 + tid;
        uint64_t msk = 0;
        if (w < nwords) {
            msk = ~gbl(T.covered)[w];
            if (w == w0) msk &= (~0ull) << (cur & 63);
            if (w == nwords - 1 && (n & 63)) msk &= (1ull << (n & 63)) - 1;
        }
        int total;
        const int pre = block_excl_scan<NT>((int)__popcll(msk), &total, sh_scan);
        const int room = B - count;
        int k = pre;
        while (msk && k < room) {                                // into LDS: a thread's ranks are adjacent
            const int b = __ffsll((unsigned long long)msk) - 1;
            const int64_t r = (w << 6) + b;
            clist[count + k] = (int32_t)r;
            if (count + k == 0) *sh_first = (int32_t)r;
            if (count + k == B - 1) *sh_cursor = r + 1;
            msk &= msk - 1;
            ++k;
        }
        if (total >= room) {
            count = B;
        } else {
            count += total;
            cur = (w0 + NT) << 6;
        }
    }
    __syncthreads();                                             // clist, sh_first visible to the workgroup
    for (int j = tid; j < count; j += NT) gbl(T.cand)[j] = clist[j];  // coalesced

    int64_t R1 = R0;
    const int64_t m_old = m;
    if (T.settle && count > 0) {
        // The non-landmarks among ranks [R0, R1) are listed in rank order:
        // 64 ranks per thread per round into LDS (the gather's list, free
        // again), then out to idx[m ..] coalesced.  The next resolve pass
        // copies their thresholds, operands and original indices with all its
        // workgroups (settle_copy).
        R1 = ((int64_t)*sh_first >> 5) << 5;
        int32_t *sel = clist;
        constexpr int kSel = MAX_B;                              // listed per pass
        const BM_GLOBAL uint64_t *islm = gbl(T.islm);
        BM_GLOBAL int32_t *sidx = gbl(T.sd.idx);
        for (int64_t w0 = R0 >> 6; (w0 << 6) < R1; w0 += NT) {  // R0 is a multiple of 32
            const int64_t w = w0 + tid;
            uint64_t msk = 0;
            if ((w << 6) < R1) {
                msk = ~islm[w];
                const int64_t lo = w << 6;
                if (lo < R0) msk &= (~0ull) << (R0 - lo);        // R0 - lo is 0 or 32
                if (R1 - lo < 64) msk &= (1ull << (R1 - lo)) - 1;
            }
            int total;
            const int pre = block_excl_scan<NT>((int)__popcll(msk), &total, sh_scan);
            for (int q0 = 0; q0 < total; q0 += kSel) {
                {
                    uint64_t mm = msk;
                    for (int k = pre; mm; ++k) {
                        const int b = __ffsll((unsigned long long)mm) - 1;
                        mm &= mm - 1;
                        if (k >= q0 && k < q0 + kSel) sel[k - q0] = (int32_t)((w << 6) + b);
                    }
                }
                __syncthreads();
                const int cnt = min(kSel, total - q0);
                for (int q = tid; q < cnt; q += NT) sidx[m + q0 + q] = sel[q];
                __syncthreads();                                 // sel is listed again next
            }
            m += total;
        }
    }

    if (tid == 0) {
        st->nc = count;
        st->na = 0;
        st->cursor = (count == B) ? *sh_cursor : n;
        if (count == 0) {
            st->done = 1;
            if (T.ndone) gatomic_add(T.ndone, 1ull);
        } else {
            st->blocks += 1;
            st->candidates += (unsigned long long)count;
            st->resolve_pairs += (unsigned long long)count * (unsigned long long)(count - 1) / 2;
            if (T.settle) {
                st->rlo = R1;
                st->m = m;
                st->settle_from = m_old;
            }
        }
    }
}

// Copy the entries [settle_from, m) the last opening of chain T listed (their
// ranks in idx) into the settled set: thresholds, operands, original index.
// Part `part` of `parts` workgroups takes a contiguous share; neighbouring
// threads copy neighbouring entries, several loads in flight per thread.
// Called by every workgroup of the resolve that follows the opening.
template <int NT>
__device__ void settle_copy(const ChainTask &T, int part, int parts)
{
    const BM_GLOBAL GreedyState *st = gbl(T.st);
    if (!T.settle || st->nc == 0) return;                        // no block was opened
    const int64_t e0 = st->settle_from, e1 = st->m;
    const int64_t per = (e1 - e0 + parts - 1) / parts;
    const int64_t a0 = e0 + (int64_t)part * per, a1 = min(e1, a0 + per);
    if (a0 >= a1) return;
    const int cnt = (int)(a1 - a0);
    const MfmaArgs &a = T.a;
    const int S = a.S, nvec = 2 * S;
    const int tid = (int)threadIdx.x;
    const BM_GLOBAL float *aT3 = gbl(a.T3);
    BM_GLOBAL float *sT3 = gbl(T.sd.T3);
    BM_GLOBAL int32_t *sidx = gbl(T.sd.idx);
    const BM_GLOBAL int32_t *perm = gbl(T.perm);
    const BM_GLOBAL u32x4 *aP = (const BM_GLOBAL u32x4 *)gbl(a.Pop);
    BM_GLOBAL u32x4 *sP = (BM_GLOBAL u32x4 *)gbl(T.sd.Pop);
    // operands first (they read the ranks in idx), vector sv = 2 K-step + half
    // of entry q, entries fastest
    const int nv = cnt * nvec;
    for (int v0 = tid; v0 < nv; v0 += 4 * NT) {
        u32x4 val[4];
        int64_t dof[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int v = min(v0 + u * NT, nv - 1);
            const int sv = v / cnt, q = v - sv * cnt;
            const int ss = sv >> 1, half = sv & 1;
            const int64_t src = sidx[a0 + q], dst = a0 + q;
            val[u] = aP[(((src >> 5) * S + ss) * 64) + (src & 31) + 32 * half];
            dof[u] = (((dst >> 5) * S + ss) * 64) + (dst & 31) + 32 * half;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (v0 + u * NT < nv) sP[dof[u]] = val[u];
    }
    __syncthreads();                                             // every rank in idx has been read
    for (int q = tid; q < cnt; q += NT) {
        const int64_t j = a0 + q;
        const int32_t r = sidx[j];
#pragma unroll
        for (int c3 = 0; c3 < 3; ++c3) sT3[t3_index(j, c3)] = aT3[t3_index(r, c3)];
        sidx[j] = T.perm ? perm[r] : r;
    }
}

// Accept the opened block of chain T in rank order, by rounds: a candidate
// without any earlier conflict (rowflag 0) is accepted at once; otherwise it
// is rejected as soon as one of its earlier conflicts is accepted, and
// accepted once all of them are rejected.  Decisions never change, so a stale
// view only delays one; the earliest undecided candidate always has all its
// conflicts decided, so every round decides at least one.  The result equals
// the sequential scan.  Thread t holds candidates k * NT + t, so each wave's
// lanes cover one bitmap word per k and every load and store coalesces; the
// listing and the compaction take one slot scan each.  In a round one wave
// takes one flagged row, lane w reading conflict words w, w + 64 (coalesced).
// The accepted ranks go to A (the range pass's list), the landmark list
// (original indices) and lm_rank at ordinal st->L, and the block is recorded
// in blog[(st->blocks - 1) % kBlockLogSize].  The conflict words of the
// flagged rows are cleared afterwards: the resolve stores only nonzero words
// (only flagged rows hold any), so the words are all zero between blocks.
// The acceptance of a block of nc <= RUN * NT candidates.
template <int NT, int RUN>
__device__ void accept_run(const ChainTask &T, unsigned char *lds, BM_GLOBAL GreedyState *st, const int nc)
{
    constexpr int NWAVES = NT / 64;
    static_assert(RUN <= 32 && RUN * NT <= MAX_B, "a thread's candidates fit one 32-bit mask");
    unsigned long long *acc = (unsigned long long *)lds;        // [MAX_B / 64] accepted
    unsigned long long *rej = acc + MAX_B / 64;                 // [MAX_B / 64] rejected
    int *sh_undecided = (int *)(rej + MAX_B / 64);
    int *tab = sh_undecided + 4;                                // [MAX_B / 64 + 4] slot bases
    int16_t *flist = (int16_t *)(tab + MAX_B / 64 + 4);         // [MAX_B] flagged rows
    const int tid = (int)threadIdx.x;
    const int64_t L0 = st->L;
    BM_GLOBAL uint64_t *C = gbl(T.C);
    const int nw = (T.B + 63) / 64;
    const int lane = lane_id(), wid = tid >> 6;
    // Candidate j = k * NT + tid: the 64 lanes of a wave hold 64 consecutive
    // candidates, one bitmap word, so loads and stores coalesce and a ballot
    // is that word.  Rows with no earlier conflict are accepted at once.
    uint32_t flagged = 0, inrun = 0;
    {
        // (unconditional loads, clamped into the block, so that all of them
        // are in flight at once instead of one wait per branch)
        int fl[RUN];
#pragma unroll
        for (int k = 0; k < RUN; ++k) fl[k] = gbl(T.rowflag)[min(k * NT + tid, nc - 1)];
#pragma unroll
        for (int k = 0; k < RUN; ++k) {
            if (k * NT + tid < nc) {
                inrun |= 1u << k;
                if (fl[k]) flagged |= 1u << k;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < RUN; ++k) {
        const bool in = (inrun >> k) & 1u, f = (flagged >> k) & 1u;
        const unsigned long long okb = __ballot(in && !f);
        const unsigned long long fb = __ballot(f);
        if (lane == 0) {
            acc[k * NWAVES + wid] = okb;
            rej[k * NWAVES + wid] = 0ull;
            tab[k * NWAVES + wid] = (int)__popcll(fb);
        }
    }
    // the flagged rows in rank order
    const int F = slot_scan<NT, RUN>(tab);
#pragma unroll
    for (int k = 0; k < RUN; ++k) {
        const unsigned long long fb = __ballot((flagged >> k) & 1u);
        if ((flagged >> k) & 1u) flist[tab[k * NWAVES + wid] + mbcnt(fb)] = (int16_t)(k * NT + tid);
    }
    __syncthreads();
    unsigned long long rounds = 0;
    while (F > 0) {                                              // uniform
        if (tid == 0) *sh_undecided = 0;
        __syncthreads();
        for (int q = wid; q < F; q += NWAVES) {
            const int j = flist[q];
            const int wj = j >> 6;
            const unsigned long long bit = 1ull << (j & 63);
            const unsigned long long dj =
                __atomic_load_n(&acc[wj], __ATOMIC_RELAXED) | __atomic_load_n(&rej[wj], __ATOMIC_RELAXED);
            if (__ballot((dj & bit) != 0)) continue;             // decided (decisions are final)
            const int nwj = (j + 63) >> 6;                       // words holding candidates < j
            bool any_acc = false, any_open = false;
            for (int w0 = 0; w0 < nwj; w0 += 64) {               // lane w reads word w0 + w
                const int w = w0 + lane;
                unsigned long long c = 0, av = 0, rv = 0;
                if (w < nwj) {
                    c = C[(int64_t)j * nw + w];
                    if (w == wj) c &= bit - 1ull;                // only i < j (the rest is not written)
                    av = __atomic_load_n(&acc[w], __ATOMIC_RELAXED);
                    rv = __atomic_load_n(&rej[w], __ATOMIC_RELAXED);
                }
                any_acc = any_acc || __ballot((c & av) != 0ull) != 0;
                any_open = any_open || __ballot((c & ~(av | rv)) != 0ull) != 0;
            }
            if (lane == 0) {
                if (any_acc) atomicOr(&rej[wj], bit);
                else if (!any_open) atomicOr(&acc[wj], bit);
                else *sh_undecided = 1;
            }
        }
        __syncthreads();
        ++rounds;
        const int und = *sh_undecided;
        __syncthreads();
        if (!und) break;
        if (rounds > (unsigned long long)nc) {                   // every round decides one: cannot happen
            if (tid == 0) st->error = 1;
            break;
        }
    }
    // back to zero for the next resolve: row j holds words below (j + 63) / 64 only
    for (int q = wid; q < F; q += NWAVES) {
        const int j = flist[q];
        for (int w = lane; w < ((j + 63) >> 6); w += 64) C[(int64_t)j * nw + w] = 0ull;
    }
    // the accepted candidates, compacted in rank order
    uint32_t took = 0;
#pragma unroll
    for (int k = 0; k < RUN; ++k) {
        const int j = k * NT + tid;
        if (((inrun >> k) & 1u) && ((acc[j >> 6] >> (j & 63)) & 1ull)) took |= 1u << k;
    }
    // (the ranks are read again here, not held through the rounds)
    int32_t rank[RUN], orig[RUN];
#pragma unroll
    for (int k = 0; k < RUN; ++k) rank[k] = gbl(T.cand)[min(k * NT + tid, nc - 1)];
    if (T.perm) {                                                // (unconditional loads: all in flight)
#pragma unroll
        for (int k = 0; k < RUN; ++k) orig[k] = gbl(T.perm)[rank[k]];
    } else {
#pragma unroll
        for (int k = 0; k < RUN; ++k) orig[k] = rank[k];
    }
    __syncthreads();                                             // the rounds' reads of tab are over
#pragma unroll
    for (int k = 0; k < RUN; ++k) {
        const int c = (int)__popcll(__ballot((took >> k) & 1u));
        if (lane == 0) tab[k * NWAVES + wid] = c;
    }
    const int total = slot_scan<NT, RUN>(tab);
#pragma unroll
    for (int k = 0; k < RUN; ++k) {
        const unsigned long long tb = __ballot((took >> k) & 1u);
        if (!((took >> k) & 1u)) continue;
        const int pos = tab[k * NWAVES + wid] + mbcnt(tb);
        const int32_t r = rank[k];
        gbl(T.A)[pos] = r;
        gbl(T.landmarks)[L0 + pos] = orig[k];
        gbl(T.lm_rank)[L0 + pos] = r;
    }
    if (tid == 0) {
        st->L0 = L0;
        st->na = total;
        st->L = L0 + total;
        st->rounds += rounds;
        st->range_pairs += (unsigned long long)total * (unsigned long long)(st->m + T.n - st->rlo);
        st->accepted += 1;
        BM_GLOBAL BlockLog &b = gbl(T.blog)[(st->blocks - 1) % kBlockLogSize];
        b.L0 = L0;
        b.na = total;
        b.rlo = st->rlo;
        b.m = st->m;
        b.nkeys_before = *gbl(T.nkeys);
    }
}

template <int NT>
__device__ void block_accept(const ChainTask &T, unsigned char *lds)
{
    constexpr int RUN = MAX_B / NT;
    BM_GLOBAL GreedyState *st = gbl(T.st);
    const int nc = st->nc;
    if (nc == 0) {                                               // no block (the chain is done)
        if (threadIdx.x == 0) st->na = 0;
        return;
    }
    // a block of at most half the largest size takes half the runs
    if (nc <= MAX_B / 2) accept_run<NT, RUN / 2>(T, lds, st, nc);
    else accept_run<NT, RUN>(T, lds, st, nc);
}

} // namespace bm
