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

constexpr int MAX_B = 8192;

// LDS bytes the steps use (from a caller-provided, 16-byte aligned buffer).
template <int NT> constexpr size_t open_lds_bytes() { return 16 + (size_t)NT / 64 * 4 + (size_t)NT * 16; }
template <int NT> constexpr size_t accept_lds_bytes()
{
    return (size_t)MAX_B / 64 * 16 + 16 + (size_t)NT / 64 * 4 + (size_t)MAX_B * 2;
}

// Open a block of chain T:
//  1. Gather: scan the covered bitmap from the cursor, 64 ranks per thread per
//     sweep, and list up to B uncovered ranks in increasing order; clear
//     rowflag[0..B).
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
    int32_t *sel = (int32_t *)(lds + 16 + NT / 64 * 4);
    const int tid = (int)threadIdx.x;
    GreedyState *st = T.st;
    const int64_t n = T.n;
    const int B = T.B;
    if (st->done) {                                              // workgroup-uniform
        if (tid == 0) {
            st->nc = 0;
            st->na = 0;
        }
        return;
    }
    for (int j = tid; j < B; j += NT) T.rowflag[j] = 0;
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
            msk = ~T.covered[w];
            if (w == w0) msk &= (~0ull) << (cur & 63);
            if (w == nwords - 1 && (n & 63)) msk &= (1ull << (n & 63)) - 1;
        }
        int total;
        const int pre = block_excl_scan<NT>((int)__popcll(msk), &total, sh_scan);
        const int room = B - count;
        int k = pre;
        while (msk && k < room) {
            const int b = __ffsll((unsigned long long)msk) - 1;
            const int64_t r = (w << 6) + b;
            T.cand[count + k] = (int32_t)r;
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
    __syncthreads();                                             // cand[], sh_first visible to the workgroup

    int64_t R1 = R0;
    if (T.settle && count > 0) {
        // one bitmap word (64 ranks) per thread per round; the round's
        // non-landmarks are listed in rank order, then their thresholds,
        // indices and operands copied
        const MfmaArgs &a = T.a;
        const SettledSet &sd = T.sd;
        R1 = ((int64_t)*sh_first >> 5) << 5;
        const int S = a.S, nvec = 2 * S;
        constexpr int kSel = NT * 4;                             // listed per pass of the copy
        for (int64_t w0 = R0 >> 6; (w0 << 6) < R1; w0 += NT) {  // R0 is a multiple of 32
            const int64_t w = w0 + tid;
            uint64_t msk = 0;
            if ((w << 6) < R1) {
                msk = ~T.islm[w];
                const int64_t lo = w << 6;
                if (lo < R0) msk &= (~0ull) << (R0 - lo);        // R0 - lo is 0 or 32
                if (R1 - lo < 64) msk &= (1ull << (R1 - lo)) - 1;
            }
            int total;
            const int pre = block_excl_scan<NT>((int)__popcll(msk), &total, sh_scan);
            // thresholds and indices straight away; operands through the LDS list
            for (int k = pre; msk; ++k) {
                const int b = __ffsll((unsigned long long)msk) - 1;
                msk &= msk - 1;
                const int64_t r = (w << 6) + b;
                const int64_t j = m + k;
#pragma unroll
                for (int q = 0; q < 3; ++q) sd.T3[t3_index(j, q)] = a.T3[t3_index(r, q)];
                sd.idx[j] = T.perm ? T.perm[r] : (int32_t)r;
                if (k < kSel) sel[k] = (int32_t)r;
            }
            __syncthreads();
            for (int q0 = 0; q0 < total; q0 += kSel) {
                if (q0 > 0) {                                    // a long round: list the next part again
                    __syncthreads();
                    int k = pre;
                    uint64_t mm = 0;
                    if ((w << 6) < R1) {
                        mm = ~T.islm[w];
                        const int64_t lo = w << 6;
                        if (lo < R0) mm &= (~0ull) << (R0 - lo);
                        if (R1 - lo < 64) mm &= (1ull << (R1 - lo)) - 1;
                    }
                    for (; mm; ++k) {
                        const int b = __ffsll((unsigned long long)mm) - 1;
                        mm &= mm - 1;
                        if (k >= q0 && k < q0 + kSel) sel[k - q0] = (int32_t)((w << 6) + b);
                    }
                    __syncthreads();
                }
                const int cnt = min(kSel, total - q0);
                for (int v = tid; v < cnt * nvec; v += NT) {
                    const int q = v / nvec, rem = v - q * nvec, ss = rem >> 1, half = rem & 1;
                    const int64_t src = sel[q], dst = m + q0 + q;
                    const int64_t so = ((((src >> 5) * S + ss) * 64) + (src & 31) + 32 * half) * 8;
                    const int64_t dof = ((((dst >> 5) * S + ss) * 64) + (dst & 31) + 32 * half) * 8;
                    *(u32x4 *)(sd.Pop + dof) = *(const u32x4 *)(a.Pop + so);
                }
            }
            m += total;
            __syncthreads();
        }
    }

    if (tid == 0) {
        st->nc = count;
        st->na = 0;
        st->cursor = (count == B) ? *sh_cursor : n;
        if (count == 0) {
            st->done = 1;
            if (T.ndone) atomicAdd(T.ndone, 1ull);
        } else {
            st->blocks += 1;
            st->candidates += (unsigned long long)count;
            st->resolve_pairs += (unsigned long long)count * (unsigned long long)(count - 1) / 2;
            if (T.settle) {
                st->rlo = R1;
                st->m = m;
            }
        }
    }
}

// Accept the opened block of chain T in rank order, by rounds: a candidate
// without any earlier conflict (rowflag 0) is accepted at once; otherwise it
// is rejected as soon as one of its earlier conflicts is accepted, and
// accepted once all of them are rejected.  Decisions never change, so a stale
// view only delays one; the earliest undecided candidate always has all its
// conflicts decided, so every round decides at least one.  The result equals
// the sequential scan.  Each thread takes a contiguous run of candidates for
// the listing and the compaction (one block scan each); in a round one wave
// takes one flagged row, lane w reading conflict words w, w + 64 (coalesced).  The accepted ranks go to A (the range pass's list), the
// landmark list (original indices) and lm_rank at ordinal st->L, and the
// block is recorded in blog[(st->blocks - 1) % kBlockLogSize].
template <int NT>
__device__ void block_accept(const ChainTask &T, unsigned char *lds)
{
    constexpr int NWAVES = NT / 64;
    unsigned long long *acc = (unsigned long long *)lds;
    unsigned long long *rej = acc + MAX_B / 64;
    int *sh_undecided = (int *)(rej + MAX_B / 64);
    int *sh_scan = sh_undecided + 4;
    int16_t *flist = (int16_t *)(sh_scan + NT / 64);
    GreedyState *st = T.st;
    const int nc = st->nc;
    const int tid = (int)threadIdx.x;
    if (nc == 0) {                                               // no block (the chain is done)
        if (tid == 0) st->na = 0;
        return;
    }
    const int64_t L0 = st->L;
    const uint64_t *C = T.C;
    const int nw = (T.B + 63) / 64;
    const int lane = lane_id(), wid = tid >> 6;
    uint64_t *islm = T.settle ? T.islm : nullptr;
    for (int t = tid; t < MAX_B / 64; t += NT) acc[t] = rej[t] = 0ull;
    __syncthreads();
    // rows with no earlier conflict are accepted; the flagged ones are listed in
    // rank order.  Thread t takes the contiguous run [t * per, (t + 1) * per),
    // its row flags and ranks loaded up front (independent loads).
    constexpr int RUN = MAX_B / NT;
    const int per = (nc + NT - 1) / NT;                          // <= RUN
    const int j0 = tid * per, j1 = min(nc, j0 + per);
    int32_t rank[RUN];
    uint32_t flagged = 0, inrun = 0;
#pragma unroll
    for (int k = 0; k < RUN; ++k) {
        const int j = j0 + k;
        const bool in = j < j1;
        const int f = in ? T.rowflag[j] : 0;
        rank[k] = in ? T.cand[j] : 0;
        if (in) inrun |= 1u << k;
        if (f) flagged |= 1u << k;
    }
    {
        // the run spans at most two bitmap words: one LDS atomic per word
        uint32_t ok = inrun & ~flagged;
        while (ok) {
            const int k = __builtin_ctz(ok);
            const int w = (j0 + k) >> 6;
            unsigned long long bits = 0;
            while (ok) {
                const int kk = __builtin_ctz(ok);
                if (((j0 + kk) >> 6) != w) break;
                bits |= 1ull << ((j0 + kk) & 63);
                ok &= ok - 1;
            }
            atomicOr(&acc[w], bits);
        }
    }
    const int nfl = __popc(flagged);
    int F;
    int pre = block_excl_scan<NT>(nfl, &F, sh_scan);
    for (uint32_t fl = flagged; fl; fl &= fl - 1) flist[pre++] = (int16_t)(j0 + __builtin_ctz(fl));
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
    // the accepted candidates, compacted in rank order (each thread its run);
    // landmark bits are merged per bitmap word before one atomic
    uint32_t took = 0;
#pragma unroll
    for (int k = 0; k < RUN; ++k)
        if (((inrun >> k) & 1u) && ((acc[(j0 + k) >> 6] >> ((j0 + k) & 63)) & 1ull)) took |= 1u << k;
    int32_t orig[RUN];
#pragma unroll
    for (int k = 0; k < RUN; ++k) orig[k] = ((took >> k) & 1u) && T.perm ? T.perm[rank[k]] : rank[k];
    const int mine = __popc(took);
    int total;
    int pos = block_excl_scan<NT>(mine, &total, sh_scan);
    int64_t word = -1;
    unsigned long long bits = 0;
#pragma unroll
    for (int k = 0; k < RUN; ++k) {
        if (!((took >> k) & 1u)) continue;
        const int32_t r = rank[k];
        T.A[pos] = r;
        T.landmarks[L0 + pos] = orig[k];
        T.lm_rank[L0 + pos] = r;
        ++pos;
        if (islm) {
            if ((r >> 6) != word) {
                if (bits) atomicOr((unsigned long long *)&islm[word], bits);
                word = r >> 6;
                bits = 0;
            }
            bits |= 1ull << (r & 63);
        }
    }
    if (islm && bits) atomicOr((unsigned long long *)&islm[word], bits);
    if (tid == 0) {
        st->L0 = L0;
        st->na = total;
        st->L = L0 + total;
        st->rounds += rounds;
        st->range_pairs += (unsigned long long)total * (unsigned long long)(st->m + T.n - st->rlo);
        st->accepted += 1;
        BlockLog &b = T.blog[(st->blocks - 1) % kBlockLogSize];
        b.L0 = L0;
        b.na = total;
        b.rlo = st->rlo;
        b.m = st->m;
        b.nkeys_before = *T.nkeys;
    }
}

} // namespace bm
