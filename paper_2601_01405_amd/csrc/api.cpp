// api.cpp — the C ABI of libbm.so: validation, device memory, the blocked
// greedy driver, CSR and edge finalisation, result ownership.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "bm.h"
#include "bm_internal.h"
#include "bounds.h"
#include "batch.h"
#include "host_common.h"
#include "kernels.h"

using namespace bm;

namespace {

using namespace bm::host;

// ---- one build ------------------------------------------------------------------------
struct Job {
    const void *points;
    int64_t n;
    int32_t d, dtype;
    double eps;
    const int64_t *order;          // greedy order (ignored in fixed mode)
    const int32_t *fixed;          // fixed landmark list (original indices) or null
    int64_t n_fixed;
};

bm_result *run_job(const Job &job, const bm_options &o)
{
    const auto t_start = clk::now();
    const int64_t n = job.n;
    const int32_t d = job.d;
    bm_result *res = new_result();
    res->stats.path = o.path;
    try {
        Device dev(o);
        res->device = dev.dev;
        const double e2 = job.eps * job.eps;   // RN(eps^2), once, in FP64
        const auto t_prep = clk::now();

        // -- stored points on the device
        const void *Xd = job.points;
        if (!o.points_on_device && n > 0) {
            void *p = dev.raw_alloc((size_t)n * d * dtype_size(job.dtype), true);
            hip_ok(hipMemcpyAsync(p, job.points, (size_t)n * d * dtype_size(job.dtype), hipMemcpyHostToDevice, dev.s),
                   "upload points");
            Xd = p;
        }
        std::vector<int32_t> perm_h = job.fixed ? std::vector<int32_t>() : check_order(job.order, n);
        int32_t *perm_d = nullptr;
        if (!perm_h.empty()) {
            perm_d = dev.alloc<int32_t>((size_t)n);
            hip_ok(hipMemcpyAsync(perm_d, perm_h.data(), (size_t)n * 4, hipMemcpyHostToDevice, dev.s), "upload order");
        }
        PointsView P{Xd, n, d, job.dtype, perm_d};

        // -- validation and statistics on the device
        int32_t path = o.path;
        double max_nu = 0.0, max_abs = 0.0;
        double *nu = nullptr;
        if (n > 0) {
            // maxima of |x|^2 and |x_k|, and (device points) a non-finite flag,
            // read back together (one wait); the statistics of a non-finite
            // input are computed but never used
            struct Stats3 {
                unsigned long long v[3];
            };
            unsigned long long *st3 = dev.zeros<unsigned long long>(3);
            if (o.points_on_device)
                hip_ok(launch_check_finite(Xd, job.dtype, n * (int64_t)d, (int *)(st3 + 2), dev.s), "check_finite");
            nu = dev.alloc<double>((size_t)n);
            hip_ok(launch_point_stats(P, nu, st3, dev.s), "point_stats");
            const Stats3 h = dev.fetch((const Stats3 *)st3);
            if (h.v[2]) fail(BM_ENONFINITE, "a coordinate is NaN or infinite");
            std::memcpy(&max_nu, &h.v[0], 8);
            std::memcpy(&max_abs, &h.v[1], 8);
        }
        MfmaArgs ma{};
        bool ma_ready = false;
        if (path == BM_PATH_AUTO) {
            path = auto_path(job.dtype, d, e2, max_nu, max_abs);
            // the split costs three products per coordinate: past K = 48, see
            // whether one scaled-F16 product leaves few enough pairs to recheck
            if (path == BM_PATH_BF16X3 && n > 0 && split_is_costly(d)) {
                MfmaArgs f = prepare_mfma(dev, P, nu, MFMA_F16, e2, max_nu, max_abs, o.refine);
                if (prefer_f16(d, sample_band_rate(dev, P, f, e2))) {
                    path = BM_PATH_F16;
                    ma = f;
                    ma_ready = true;
                } else {
                    release_mfma(dev, f);
                }
            }
        }
        res->stats.path = path;
        int B = o.block ? o.block : auto_block(n, d, path);

        // -- path preparation
        Fp32Thresholds thr32{};
        float *xf = nullptr;
        if (path == BM_PATH_FP32) {
            thr32 = fp32_thresholds(e2, d, job.dtype, std::sqrt(max_nu), max_abs);
            if (job.dtype == BM_F32 && !perm_d) {
                xf = (float *)Xd;
            } else if (n > 0) {
                xf = dev.alloc<float>((size_t)n * d);
                hip_ok(launch_to_f32(P, xf, dev.s), "to_f32");
            }
        } else if (n > 0 && !ma_ready) {
            ma = prepare_mfma(dev, P, nu, path, e2, max_nu, max_abs, o.refine);
        }
        res->stats.ms_prepare = ms_since(t_prep);

        // -- range passes
        const auto t_greedy = clk::now();
        const int32_t bn = std::max(1, bitlen((uint64_t)std::max<int64_t>(n - 1, 1)));
        unsigned long long cap = o.init_member_capacity
                                     ? (unsigned long long)o.init_member_capacity
                                     : (unsigned long long)std::max<int64_t>(2 * n, 1 << 16);
        if ((!o.init_member_capacity || !o.block) && ma.Pop && !job.fixed && n >= kProbePoints) {
            // big clouds: the mean ball of 64 sampled landmarks sizes the buffer for
            // the first blocks, so that they need no recompute after an overflow,
            // and with large balls (many candidates rejected, many members per
            // pass) an automatic block is smaller, with balls of about one point
            // (every candidate accepted) larger
            const double ball = sample_pass(dev, P, ma, e2, 64).ball_mean;
            if (!o.block && ball >= kLargeBall) B = std::min(B, kLargeBallBlock);
            if (!o.block && ball < kTinyBall) B = std::max(B, kTinyBallBlock);
            if (!o.init_member_capacity)
                cap = std::max<unsigned long long>(cap, (unsigned long long)(1.5 * ball * 4.0 * B) + 65536ull);
        }
        res->stats.block = B;
        uint64_t *keys = dev.alloc<uint64_t>(cap);
        GreedyState *st = dev.zeros<GreedyState>(1);
        const int64_t lm_cap = std::max<int64_t>(job.fixed ? job.n_fixed : n, 1);
        int32_t *lm_d = dev.alloc<int32_t>((size_t)lm_cap);
        int32_t *lm_rank = job.fixed ? lm_d : dev.alloc<int32_t>((size_t)lm_cap);   // fixed mode: ranks = indices
        int32_t *A = dev.alloc<int32_t>((size_t)B);
        int64_t *fixtab = dev.alloc<int64_t>(4 * kUploadBlocks);   // blk[0..3] rows of directly launched passes
        // device task tables: [0] the greedy's range pass, [1] its resolve,
        // [2 + q] directly launched passes of the fixed-landmark / recompute paths
        RangeTask *rtask = dev.alloc<RangeTask>(2 + kUploadBlocks);
        ChainTask *ctask = dev.alloc<ChainTask>(1);
        GreedyState hs{};
        int64_t L = 0;
        RangeOut ro{nullptr, keys, cap, &st->nkeys, st, 0, bn};
        int32_t NGW = 1, chunks = 8;
        const bool mfma = path != BM_PATH_FP32;
        if (mfma) range_grid(B, n, range_target_wg(), &NGW, &chunks);

        // range-pass launches, optionally bracketed by events on the same stream
        std::vector<std::pair<hipEvent_t, hipEvent_t>> evs;
        struct EvGuard {
            std::vector<std::pair<hipEvent_t, hipEvent_t>> &v;
            ~EvGuard()
            {
                for (auto &e : v) {
                    (void)hipEventDestroy(e.first);
                    (void)hipEventDestroy(e.second);
                }
            }
        } ev_guard{evs};
        SettledSet sd{};
        // device-clock execution windows of the range passes (profile = 1)
        // ([0] range passes, [1] resolves)
        KernelClock *kclk = nullptr, *rclk = nullptr;
        if (o.profile) {
            kclk = dev.alloc<KernelClock>(2);
            const KernelClock init[2] = {{~0ull, 0ull, 0ull, 0ull}, {~0ull, 0ull, 0ull, 0ull}};
            dev.upload(kclk, init, sizeof init);
            rclk = kclk + 1;
        }
        auto range_task = [&](const int32_t *Alist, const int64_t *blk, uint64_t *covered) {
            RangeTask t{};
            t.a = ma;
            t.P = P;
            t.n_dev = nullptr;
            t.e2 = e2;
            t.A = Alist;
            t.blk = blk;
            t.o = ro;
            t.o.keys = keys;
            t.o.cap = cap;
            t.o.covered = covered;
            t.sd = sd;
            t.NGW = NGW;
            t.chunks = chunks;
            t.wg0 = 0;
            return t;
        };
        // A range pass on stream `s` (task: its device-side descriptor, matrix-core
        // path); per-launch events only for direct launches (profile = 1).
        auto run_range_on = [&](hipStream_t s, bool events, const RangeTask *task, const int32_t *Alist,
                                const int64_t *blk, uint64_t *covered) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (events && o.profile) {
                hip_ok(hipEventCreate(&e0), "hipEventCreate");
                hip_ok(hipEventCreate(&e1), "hipEventCreate");
                evs.emplace_back(e0, e1);
            }
            const LaunchEvents ev{e0, e1, kclk};
            if (!mfma) {
                RangeOut r = ro;
                r.keys = keys;
                r.cap = cap;
                r.covered = covered;
                hip_ok(launch_range_fp32(xf, P, e2, thr32, o.refine, Alist, blk, B, r, s, ev), "range_fp32");
            } else {
                hip_ok(launch_range_tasks(task, nullptr, (int64_t)NGW * chunks, ma.kind, ma.S, false, s, ev),
                       "range_mfma");
            }
        };
        // Directly launched passes over rows of blocks (L0, na, rlo, m): the
        // fixed-landmark mode and the recompute after a key-buffer overflow.
        int64_t *tab_h = (int64_t *)dev.pinned;       // [0, 2 KB) of the pinned staging
        auto run_rows = [&](const std::vector<BlockLog> &rows, const int32_t *lm_list) {
            for (size_t j = 0; j < rows.size(); j += kUploadBlocks) {
                const size_t m = std::min<size_t>(kUploadBlocks, rows.size() - j);
                dev.sync();
                for (size_t q = 0; q < m; ++q) {
                    tab_h[4 * q] = rows[j + q].L0;
                    tab_h[4 * q + 1] = rows[j + q].na;
                    tab_h[4 * q + 2] = rows[j + q].rlo;
                    tab_h[4 * q + 3] = rows[j + q].m;
                }
                hip_ok(hipMemcpyAsync(fixtab, tab_h, m * 32, hipMemcpyHostToDevice, dev.s), "upload table");
                if (mfma) {
                    std::vector<RangeTask> tv(m);
                    for (size_t q = 0; q < m; ++q) tv[q] = range_task(lm_list + rows[j + q].L0, fixtab + 4 * q, nullptr);
                    dev.upload(rtask + 2, tv.data(), m * sizeof(RangeTask));
                }
                for (size_t q = 0; q < m; ++q) {
                    run_range_on(dev.s, true, rtask + 2 + q, lm_list + rows[j + q].L0, fixtab + 4 * q, nullptr);
                    res->stats.range_launches++;
                }
            }
        };
        // The key buffer overflowed: grow it, then recompute the memberships of
        // the landmark ranges [L0_j, L0_j + na_j) from the first incomplete one on,
        // restarting the key counter where that block began.  The landmark set is
        // unaffected (covered bits do not depend on the key buffer).
        // A bigger key buffer holding the first `keep` keys of the old one.
        auto grow_keys = [&](unsigned long long ncap, unsigned long long keep) {
            uint64_t *nk = dev.alloc<uint64_t>(ncap);
            if (keep) hip_ok(hipMemcpyAsync(nk, keys, keep * 8, hipMemcpyDeviceToDevice, dev.s), "regrow copy");
            dev.sync();
            dev.release(keys);
            keys = nk;
            cap = ncap;
        };
        auto refill = [&](const std::vector<BlockLog> &logs) {
            const unsigned long long need = hs.nkeys;
            const unsigned long long start = logs.front().nkeys_before;
            grow_keys(std::max<unsigned long long>(2 * cap, need + need / 2), start);
            dev.upload(&st->nkeys, &start, 8);
            run_rows(logs, lm_rank);
            const GreedyState chk = dev.fetch(st);
            if (chk.nkeys != need) fail(BM_EINTERNAL, "membership count changed on recompute");
            hs.nkeys = chk.nkeys;
        };

        if (job.fixed) {
            // fixed-landmark mode: landmarks given as original indices (identity order)
            L = job.n_fixed;
            if (L > 0) hip_ok(hipMemcpyAsync(lm_d, job.fixed, (size_t)L * 4, hipMemcpyHostToDevice, dev.s), "upload lm");
            std::vector<BlockLog> all;      // every rank scanned: rlo = 0, no settled list
            for (int64_t a0 = 0; a0 < L; a0 += B) all.push_back(BlockLog{a0, std::min<int64_t>(B, L - a0), 0, 0, 0});
            run_rows(all, lm_d);
            hs = dev.fetch(st);
            if (hs.nkeys > cap) refill(all);    // all[0].nkeys_before = 0: recompute everything
            res->stats.blocks = (int64_t)all.size();
            res->stats.range_pairs = L * n;
            res->stats.pairs_issued = L * n;
        } else if (n > 0) {
            const int nw = (B + 63) / 64;
            uint64_t *covered = dev.zeros<uint64_t>((size_t)((n + 63) / 64));
            int32_t *cand = dev.alloc<int32_t>((size_t)B);
            uint64_t *C = dev.zeros<uint64_t>((size_t)B * nw);      // zero between blocks (the accept clears)
            int *rowflag = dev.alloc<int>((size_t)B);
            // Settled list (refined matrix-core path): landmarks are skipped as
            // points of later range passes, since no landmark is in another's ball.
            // The unrefined predicate is not symmetric, so there every rank is scanned.
            const bool settle = mfma && o.refine;
            uint64_t *islm = nullptr;
            if (settle) {
                islm = dev.zeros<uint64_t>((size_t)((n + 63) / 64));
                const size_t np = (size_t)((n + 31) / 32 * 32);
                const size_t words = mfma_operand_words(n, ma.S);
                sd.Pop = dev.zeros<uint16_t>(words);
                sd.T3 = dev.alloc<float>(t3_floats(n));
                hip_ok(hipMemsetD32Async((hipDeviceptr_t)sd.T3, 0x7f800000, t3_floats(n), dev.s), "fill +inf");
                sd.idx = dev.zeros<int32_t>(np);
            }
            BlockLog *blog = dev.alloc<BlockLog>(kBlockLogSize);
            std::vector<BlockLog> blog_h(kBlockLogSize);
            // the chain's descriptor and its two matrix-core tasks
            ChainTask ct{};
            ct.covered = covered;
            ct.n = n;
            ct.st = st;
            ct.B = B;
            ct.settle = settle ? 1 : 0;
            ct.cand = cand;
            ct.rowflag = rowflag;
            ct.islm = islm;
            ct.a = ma;
            ct.sd = sd;
            ct.perm = perm_d;
            ct.C = C;
            ct.A = A;
            ct.landmarks = lm_d;
            ct.lm_rank = lm_rank;
            ct.blog = blog;
            ct.nkeys = &st->nkeys;
            ct.ndone = nullptr;
            dev.upload(ctask, &ct, sizeof ct);
            // [0]: the greedy's range pass, whose last workgroup opens the next block;
            // [1]: the candidate resolve, whose last workgroup accepts.
            int32_t rNGW = 1, rchunks = 8;
            if (mfma) range_grid(B, B, resolve_target_wg(), &rNGW, &rchunks);
            auto upload_tasks = [&]() {
                RangeTask t[2];
                t[0] = range_task(A, &st->L0, covered);
                t[0].chain = ctask;
                t[1] = RangeTask{};
                t[1].a = ma;
                t[1].P = P;
                t[1].n_dev = &st->nc;
                t[1].e2 = e2;
                t[1].A = cand;
                t[1].o = RangeOut{nullptr, nullptr, 0, &st->nkeys, st, 0, 0};
                t[1].C32 = (uint32_t *)C;
                t[1].c32_stride = 2 * nw;
                t[1].rowflag = rowflag;
                t[1].NGW = rNGW;
                t[1].chunks = rchunks;
                t[1].chain = ctask;
                dev.upload(rtask, t, sizeof t);
            };
            upload_tasks();
            const int64_t res_wgs = (int64_t)rNGW * rchunks;
            // One block of the greedy on stream s.  Matrix-core paths: resolve
            // (+ accept) and range pass (+ open the next block), after a first
            // open before the loop.  FP32 path: open, exact resolve, accept, range.
            auto enqueue_block = [&](hipStream_t s, bool events) {
                if (mfma) {
                    const LaunchEvents rev{nullptr, nullptr, events ? rclk : nullptr};
                    hip_ok(launch_range_tasks(rtask + 1, nullptr, res_wgs, ma.kind, ma.S, true, s, rev),
                           "resolve_mfma");
                    run_range_on(s, events, rtask, A, &st->L0, covered);
                    return;
                }
                hip_ok(launch_block_begin(ctask, 1, s), "block begin");
                hip_ok(launch_resolve_exact(P, e2, cand, st, B, C, rowflag, s), "resolve");
                hip_ok(launch_accept(ctask, 1, B, s), "accept");
                run_range_on(s, events, rtask, A, &st->L0, covered);
            };
            if (mfma) hip_ok(launch_block_begin(ctask, 1, dev.s), "first block");
            // Past the first batch, blocks are replayed from a captured HIP graph of
            // kGraphBlocks blocks (every kernel reads its block from the device-side
            // state, so one graph serves every block; blocks after the last one find
            // no candidate and do nothing).  The FP32 pass takes its key buffer by
            // value, so a graph of that path is captured again when the buffer moves.
            GraphRunner gr;
            // Capturing and instantiating costs about as much as a few hundred
            // microseconds of launches; it pays off where blocks are short (small
            // clouds), not where every block runs for a hundred microseconds.
            const bool use_graph = !o.no_graph && n < kGraphMaxPoints;
            // Blocks are queued back to back; the host looks at the state once per batch.
            // Batches of 1 and 3 blocks launched directly, then 8, 16, 32, 64.  Before
            // each batch the key buffer grows to what the keys per landmark so far
            // predict, so that an overflow (and its recompute) stays rare.
            int batch = 1;
            int nbatch = 0;
            bool direct_batch = true;
            void *graph_keys = nullptr;
            for (;;) {
                const unsigned long long blocks_before = hs.accepted;
                if (hs.L > 0) {
                    const double per_lm = (double)hs.nkeys / (double)hs.L;
                    const double want = (double)hs.nkeys + 1.25 * per_lm * (double)batch * (double)B + 65536.0;
                    if (want > (double)cap) {
                        grow_keys((unsigned long long)(want * 1.25), hs.nkeys);
                        if (mfma) upload_tasks();       // the range task writes to the new buffer
                    }
                }
                if (use_graph && !direct_batch) {
                    if (!gr.ready() || (!mfma && graph_keys != (void *)keys)) {
                        gr.capture([&](hipStream_t cs) {
                            for (int k = 0; k < kGraphBlocks; ++k) enqueue_block(cs, false);
                        });
                        graph_keys = keys;
                    }
                    for (int k = 0; k < batch; k += kGraphBlocks) gr.launch(dev.s);
                } else {
                    for (int k = 0; k < batch; ++k) enqueue_block(dev.s, true);
                }
                res->stats.range_launches += batch;
                direct_batch = ++nbatch < 2;
                hs = dev.fetch(st);
                if (hs.error) fail(BM_EINTERNAL, "candidate acceptance did not converge");
                if (hs.nkeys > cap) {
                    hip_ok(hipMemcpy(blog_h.data(), blog, sizeof(BlockLog) * kBlockLogSize, hipMemcpyDeviceToHost),
                           "read block log");
                    std::vector<BlockLog> logs;
                    // blocks accepted in this batch (a block opened by the batch's last
                    // range pass is not accepted yet: its keys come in the next batch)
                    for (unsigned long long b = blocks_before; b < hs.accepted; ++b)
                        logs.push_back(blog_h[b % kBlockLogSize]);
                    // first block whose keys did not all fit
                    size_t first = 0;
                    while (first < logs.size()) {
                        const unsigned long long end =
                            first + 1 < logs.size() ? logs[first + 1].nkeys_before : hs.nkeys;
                        if (end > cap) break;
                        ++first;
                    }
                    if (first == logs.size()) fail(BM_EINTERNAL, "overflow not attributed to a block");
                    refill(std::vector<BlockLog>(logs.begin() + (long)first, logs.end()));
                    upload_tasks();                 // the greedy's pass writes to the new buffer
                }
                if (hs.done) break;
                // the next batch: the blocks the progress so far predicts for the
                // ranks left (10% more, at least 3, at most 64), so that few batches
                // (host round trips) are needed; graphs take multiples of 8
                {
                    const double done_ranks = (double)std::max<int64_t>(hs.cursor, 1);
                    const double left = (double)(n - hs.cursor) * (double)hs.blocks / done_ranks;
                    int want = (int)std::ceil(1.1 * left) + 1;
                    want = std::max(3, std::min(want, 64));
                    if (use_graph && nbatch >= 2) want = (want + kGraphBlocks - 1) / kGraphBlocks * kGraphBlocks;
                    batch = want;
                }
            }
            L = hs.L;
            res->stats.blocks = (int64_t)hs.blocks;
            res->stats.candidates = (int64_t)hs.candidates;
            res->stats.range_pairs = (int64_t)hs.range_pairs;
            res->stats.pairs_issued = (int64_t)hs.resolve_pairs + (int64_t)hs.range_pairs;
        }
        dev.sync();
        for (auto &e : evs) {
            float ms = 0.f;
            hip_ok(hipEventElapsedTime(&ms, e.first, e.second), "hipEventElapsedTime");
            res->stats.ms_range_events += ms;
        }
        if (kclk) {
            const KernelClock kc = dev.fetch(kclk), rc = dev.fetch(rclk);
            int khz = 0;
            hip_ok(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev.dev), "wall clock rate");
            if (khz > 0) {
                res->stats.ms_range_kernel = (double)kc.ticks / (double)khz;
                res->stats.ms_resolve_kernel = (double)rc.ticks / (double)khz;
                res->stats.ms_serial_steps = (double)(kc.tail + rc.tail) / (double)khz;
            }
        }
        res->stats.band_pairs = (int64_t)hs.band;
        res->stats.pairs_useful = L * n;
        res->stats.ms_greedy = ms_since(t_greedy);

        // -- membership CSR
        const auto t_csr = clk::now();
        const int64_t M = (int64_t)hs.nkeys;
        const int end_bit = bn + std::max(1, bitlen((uint64_t)L));
        uint64_t *skeys = sort_into(dev, keys, M, end_bit);
        dev.release(keys);
        keys = nullptr;
        int64_t *row_ptr = nullptr;
        int32_t *midx = nullptr;
        csr_of(dev, skeys, M, L, bn, &row_ptr, &midx);
        dev.sync();
        res->stats.ms_csr = ms_since(t_csr);

        // -- edges
        const auto t_edges = clk::now();
        int32_t *edges = nullptr;
        // Exact greedy: every point lies in some ball, so M >= n, and M == n
        // means every point lies in exactly one: no two balls meet, no edge.
        int64_t E = 0;
        if (!job.fixed && o.refine && M == n) edges = dev.alloc<int32_t>(1);
        else E = edges_of(dev, skeys, M, L, n, bn, row_ptr, midx, &edges, nullptr);
        dev.sync();
        res->stats.ms_edges = ms_since(t_edges);

        // -- hand over
        const auto t_dl = clk::now();
        res->n_landmarks = L;
        res->n_edges = E;
        if (o.results_on_device) {
            if (!edges) edges = dev.alloc<int32_t>(1);
            res->landmarks = lm_d;
            res->member_ptr = row_ptr;
            res->member_idx = midx;
            res->edges = edges;
            res->on_device = 1;
            dev.detach(lm_d);
            dev.detach(row_ptr);
            dev.detach(midx);
            dev.detach(edges);
        } else {
            res->landmarks = (int32_t *)std::malloc((size_t)std::max<int64_t>(L, 1) * 4);
            res->member_ptr = (int64_t *)std::malloc((size_t)(L + 1) * 8);
            res->member_idx = (int32_t *)std::malloc((size_t)std::max<int64_t>(M, 1) * 4);
            res->edges = (int32_t *)std::malloc((size_t)std::max<int64_t>(2 * E, 1) * 4);
            if (!res->landmarks || !res->member_ptr || !res->member_idx || !res->edges)
                fail(BM_ENOMEM, "host allocation of the result failed");
            if (L) hip_ok(hipMemcpyAsync(res->landmarks, lm_d, (size_t)L * 4, hipMemcpyDeviceToHost, dev.s), "D2H");
            hip_ok(hipMemcpyAsync(res->member_ptr, row_ptr, (size_t)(L + 1) * 8, hipMemcpyDeviceToHost, dev.s), "D2H");
            if (M) hip_ok(hipMemcpyAsync(res->member_idx, midx, (size_t)M * 4, hipMemcpyDeviceToHost, dev.s), "D2H");
            if (E) hip_ok(hipMemcpyAsync(res->edges, edges, (size_t)E * 8, hipMemcpyDeviceToHost, dev.s), "D2H");
            dev.sync();
        }
        res->stats.ms_download = ms_since(t_dl);
        res->stats.ms_total = ms_since(t_start);
        return res;
    } catch (...) {
        bm_result_free(res);
        throw;
    }
}

template <class F> int guarded(F &&f)
{
    try {
        g_last_error.clear();
        return f();
    } catch (const BmError &e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return BM_ENOMEM;
    } catch (...) {
        g_last_error = "unexpected internal error";
        return BM_EINTERNAL;
    }
}

bm_options resolve_options(const bm_options *opt)
{
    bm_options o;
    bm_default_options(&o);
    if (opt) o = *opt;
    return o;
}

} // namespace

extern "C" {

int bm_default_options(bm_options *opt)
{
    if (!opt) return BM_EINVAL;
    std::memset(opt, 0, sizeof(*opt));
    opt->path = BM_PATH_AUTO;
    opt->refine = 1;
    opt->device = -1;
    return BM_OK;
}

int bm_build(const void *points, int64_t n, int32_t d, int32_t dtype, double eps, const int64_t *order,
             const bm_options *opt, bm_result **out)
{
    return guarded([&]() -> int {
        if (!out) fail(BM_EINVAL, "out is NULL");
        *out = nullptr;
        const bm_options o = resolve_options(opt);
        check_common(points, n, d, dtype, eps, o);
        if (order) (void)check_order(order, n);
        if (!o.points_on_device && n > 0 && !host_all_finite(points, n * (int64_t)d, dtype))
            fail(BM_ENONFINITE, "a coordinate is NaN or infinite");
        Job job{points, n, d, dtype, eps, order, nullptr, 0};
        *out = run_job(job, o);
        return BM_OK;
    });
}

int bm_range_sets(const void *points, int64_t n, int32_t d, int32_t dtype, double eps, const int32_t *landmarks,
                  int64_t n_landmarks, const bm_options *opt, bm_result **out)
{
    return guarded([&]() -> int {
        if (!out) fail(BM_EINVAL, "out is NULL");
        *out = nullptr;
        const bm_options o = resolve_options(opt);
        check_common(points, n, d, dtype, eps, o);
        if (n_landmarks < 0 || (n_landmarks > 0 && !landmarks)) fail(BM_EINVAL, "bad landmark list");
        for (int64_t i = 0; i < n_landmarks; ++i)
            if (landmarks[i] < 0 || landmarks[i] >= n) fail(BM_EINVAL, "landmark index out of range");
        if (!o.points_on_device && n > 0 && !host_all_finite(points, n * (int64_t)d, dtype))
            fail(BM_ENONFINITE, "a coordinate is NaN or infinite");
        Job job{points, n, d, dtype, eps, nullptr, landmarks, n_landmarks};
        *out = run_job(job, o);
        return BM_OK;
    });
}

int bm_build_many(const bm_problem *probs, int32_t n_probs, const bm_options *opt, bm_result **outs)
{
    int64_t slots = 0;
    int rc = guarded([&]() -> int {
        if (n_probs < 0 || (n_probs > 0 && (!probs || !outs))) fail(BM_EINVAL, "bad problem list");
        const bm_options o = resolve_options(opt);
        for (int32_t p = 0; p < n_probs; ++p) {
            const bm_problem &pr = probs[p];
            if (pr.n_eps < 0 || (pr.n_eps > 0 && !pr.eps)) fail(BM_EINVAL, "bad eps list");
            for (int32_t e = 0; e < pr.n_eps; ++e) {
                check_common(pr.points, pr.n, pr.d, pr.dtype, pr.eps[e], o);
                outs[slots++] = nullptr;
            }
            if (pr.order) (void)check_order(pr.order, pr.n);
            if (!o.points_on_device && pr.n > 0 && !host_all_finite(pr.points, pr.n * (int64_t)pr.d, pr.dtype))
                fail(BM_ENONFINITE, "a coordinate is NaN or infinite");
        }
        // chains of the problems that can share the device run as one batch;
        // the rest (the plain FP32 path, d past the matrix-core K, n = 0) one by one
        std::vector<const bm_problem *> bp;
        std::vector<int64_t> slot0;
        std::vector<char> in_batch((size_t)n_probs, 0);
        int64_t k = 0;
        for (int32_t p = 0; p < n_probs; ++p) {
            if (batchable(probs[p], o)) {
                bp.push_back(&probs[p]);
                slot0.push_back(k);
                in_batch[(size_t)p] = 1;
            }
            k += probs[p].n_eps;
        }
        if (!bp.empty() && !batch_fits(bp)) {
            bp.clear();
            slot0.clear();
            std::fill(in_batch.begin(), in_batch.end(), 0);
        }
        if (!bp.empty()) run_batch(bp, slot0, o, outs);
        k = 0;
        for (int32_t p = 0; p < n_probs; ++p) {
            const bm_problem &pr = probs[p];
            for (int32_t e = 0; e < pr.n_eps; ++e, ++k) {
                if (in_batch[(size_t)p]) continue;
                Job job{pr.points, pr.n, pr.d, pr.dtype, pr.eps[e], pr.order, nullptr, 0};
                outs[k] = run_job(job, o);
            }
        }
        return BM_OK;
    });
    if (rc != BM_OK && outs)
        for (int64_t k = 0; k < slots; ++k) {
            bm_result_free(outs[k]);
            outs[k] = nullptr;
        }
    return rc;
}

int bm_trim_cache(int32_t device)
{
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) count = 0;
    if (device < -1 || device >= count) {
        g_last_error = "bm_trim_cache: no such device";
        return BM_EINVAL;
    }
    cache_trim(device);
    g_last_error.clear();
    return BM_OK;
}

void bm_result_free(bm_result *r)
{
    if (!r) return;
    if (r->on_device && unshare_result(r)) {       // a slice of a batch's arrays
        std::free(r);
        return;
    }
    if (r->on_device) {
        int prev = -1;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(r->device);
        (void)hipFree(r->landmarks);
        (void)hipFree(r->member_ptr);
        (void)hipFree(r->member_idx);
        (void)hipFree(r->edges);
        if (prev >= 0) (void)hipSetDevice(prev);
    } else {
        std::free(r->landmarks);
        std::free(r->member_ptr);
        std::free(r->member_idx);
        std::free(r->edges);
    }
    std::free(r);
}

int bm_device_selfcheck(int32_t device, int32_t *flags)
{
    return guarded([&]() -> int {
        if (!flags) fail(BM_EINVAL, "flags is NULL");
        bm_options o;
        bm_default_options(&o);
        o.device = device;
        Device dev(o);
        *flags = device_flags(dev.dev, dev.s);
        return BM_OK;
    });
}

int bm_error_bound(int32_t path, int32_t dtype, int32_t d, double eps, double max_sq_norm, double max_abs,
                   bm_bound *out)
{
    return guarded([&]() -> int {
        if (!out) fail(BM_EINVAL, "out is NULL");
        if (d < 1 || !(eps > 0.0) || !std::isfinite(eps) || !(max_sq_norm >= 0.0) || !(max_abs >= 0.0))
            fail(BM_EINVAL, "bad arguments");
        if (dtype != BM_F64 && dtype != BM_F32 && dtype != BM_F16) fail(BM_EINVAL, "unknown dtype");
        const double e2 = eps * eps;
        std::memset(out, 0, sizeof(*out));
        double w;
        if (path == BM_PATH_FP32) {
            const double g32 = gamma_u(d + 2.0, std::ldexp(1.0, -24));
            const double E = (dtype == BM_F64) ? std::ldexp(std::sqrt(max_sq_norm), -23) : 0.0;
            exact_window(e2, d, &out->t_in, &out->t_out);
            out->rel_err = g32;
            out->abs_err = d * std::ldexp(1.0, -125);
            // |s32 - D| <= g32 (sqrt(D) + E)^2 + 2 E sqrt(D) + E^2 + abs at D = e2
            const double se = std::sqrt(e2);
            w = g32 * (se + E) * (se + E) + 2.0 * E * se + E * E + out->abs_err;
            w += std::ldexp(e2, -23);                                   // RN32 of the unrefined threshold
            out->exact_range = e2 >= std::ldexp(1.0, -100) && e2 <= std::ldexp(1.0, 100) && max_abs <= std::ldexp(1.0, 60);
        } else if (path == BM_PATH_BF16 || path == BM_PATH_BF16X3 || path == BM_PATH_F16) {
            const int Kraw = (path == BM_PATH_BF16X3) ? 3 * d : d;
            const int K = (Kraw + 15) / 16 * 16;
            // F16 on wider storage works on data scaled by s (a power of two); report in data units
            const double s = (path == BM_PATH_F16) ? f16_scale(dtype, max_abs) : 1.0;
            const MfmaBound b = mfma_bound(path, d, K, e2 * s * s, std::sqrt(max_sq_norm) * s, max_abs * s,
                                           kF16SubnormalsOk, dtype == BM_F16);
            out->alpha = b.alpha;
            out->beta = b.beta;
            out->abs_err = b.abs_err / (s * s);
            out->t_in = b.t_in / (s * s);
            out->t_out = b.t_out / (s * s);
            out->exact_range = b.sane;
            w = 2.0 * ((b.alpha + b.beta) * max_sq_norm + out->abs_err);   // |D_est - D| = 2 |G - h|
            w += std::ldexp(max_sq_norm + e2, -23);                     // RN32 of the unrefined threshold Z
        } else {
            fail(BM_EINVAL, "path must be FP32, BF16, BF16X3 or F16");
        }
        const double eps_lo = e2 > w ? std::sqrt(e2 - w) : 0.0;
        out->delta = std::max(eps - eps_lo, std::sqrt(e2 + w) - eps);
        return BM_OK;
    });
}

const char *bm_last_error(void) { return g_last_error.c_str(); }

int bm_device_count(void)
{
    int c = 0;
    if (hipGetDeviceCount(&c) != hipSuccess) return 0;
    return c;
}

int bm_abi_version(void) { return BM_ABI_VERSION; }

} // extern "C"
