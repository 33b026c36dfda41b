// batch.cpp — many Ball Mappers (point clouds x radius sweeps) in one device
// pass.  Every (problem, radius) pair is an independent greedy chain (Sec. 2.2).
// All chains advance one block per step in the same launches: one resolve
// launch (its last workgroup per chain accepts) and one range-pass launch (its
// last workgroup per chain opens the chain's next block) per operand class
// (operand kind and K); the steps are replayed from a captured HIP graph until
// every chain is done.  A chain that is done opens empty blocks whose
// workgroups exit at once.  The memberships of all chains go to one key
// buffer; one sort and the single-build CSR and edge kernels, run on the
// disjoint union of the chains, finish them all (batch.hip).
#include "batch.h"

namespace bm {
namespace host {

namespace {

struct Prob {
    const void *X = nullptr;
    int32_t *perm = nullptr;
    double *nu = nullptr;
    int64_t n = 0;
    int32_t d = 0, dtype = 0;
    int32_t path = 0, S = 0;
    double scale = 1.0, max_nu = 0.0, max_abs = 0.0;
    uint16_t *Pop = nullptr, *Qop = nullptr;
};

struct Chain {
    int p = 0;                      // problem
    int64_t slot = 0;               // output slot
    double eps = 0.0, e2 = 0.0;
    int64_t n = 0;
    int32_t B = 0;
    MfmaArgs ma{};
    SettledSet sd{};
    GreedyState *st = nullptr;
    uint64_t *covered = nullptr, *islm = nullptr, *C = nullptr;
    int32_t *cand = nullptr, *rowflag = nullptr, *A = nullptr, *lm = nullptr, *lm_rank = nullptr;
    BlockLog *blog = nullptr;
    size_t z_off = 0, i_off = 0, p_off = 0;     // arena offsets (zeroed, +inf, plain)
};

// Carves aligned sub-buffers out of one allocation.
struct Carve {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    }
};

// Workgroups per chain: about one per 1024 points, 8 to 256.
int64_t chain_target_wg(int64_t n) { return std::max<int64_t>(8, std::min<int64_t>(256, n / 1024)); }
// A chain's resolve: about 256 panel-tile products per workgroup over the
// lower triangle of the B x B candidate matrix ((B/32)^2 / 2 of them), so that
// the per-workgroup set-up is amortised; at least one round of 8.
int64_t resolve_target_wg_of(int64_t B)
{
    return std::max<int64_t>(8, std::min<int64_t>(256, B * B / (1 << 19)));
}

} // namespace

int32_t batch_block(int64_t n, int32_t d, int32_t path)
{
    (void)path;
    if (const int32_t B = tuned_block(n, d, true)) return B;
    if (n >= (1 << 17)) return 4096;
    if (n >= (1 << 15)) return 2048;
    if (n >= (1 << 13)) return 1024;
    return 256;
}

bool batchable(const bm_problem &pr, const bm_options &o)
{
    if (pr.n <= 0 || pr.n_eps <= 0) return false;
    if (o.path == BM_PATH_FP32) return false;                       // the plain baseline runs per build
    const int S1 = (pr.d + 15) / 16, S3 = (3 * pr.d + 15) / 16;
    if (S1 > kMaxMfmaSteps) return false;                           // AUTO takes FP32 there
    if (o.path == BM_PATH_BF16X3 && S3 > kMaxMfmaSteps) return false;   // per-build error path
    return true;
}

bool batch_fits(const std::vector<const bm_problem *> &probs)
{
    int64_t chains = 0, ntot = 0, nmax = 1;
    for (const bm_problem *pr : probs) {
        chains += pr->n_eps;
        ntot += pr->n * pr->n_eps;
        nmax = std::max(nmax, pr->n);
    }
    const int bn = std::max(1, bitlen((uint64_t)(nmax - 1)));
    const int bl = std::max(1, bitlen((uint64_t)nmax));
    const int bc = std::max(1, bitlen((uint64_t)(chains - 1)));
    return chains > 0 && bn + bl + bc <= 64 && ntot <= INT32_MAX && 2 * bitlen((uint64_t)ntot) <= 64;
}

void run_batch(const std::vector<const bm_problem *> &probs, const std::vector<int64_t> &slot0, const bm_options &o,
               bm_result **outs)
{
    const auto t_start = clk::now();
    Device dev(o);
    const int P = (int)probs.size();

    // ---- problems on the device: points, order, norms and maxima
    std::vector<Prob> pv((size_t)P);
    std::vector<std::vector<int32_t>> perms((size_t)P);
    unsigned long long *pstats = dev.zeros<unsigned long long>((size_t)2 * P);
    int *bad = o.points_on_device ? dev.zeros<int>((size_t)P) : nullptr;
    for (int p = 0; p < P; ++p) {
        const bm_problem &pr = *probs[(size_t)p];
        Prob &q = pv[(size_t)p];
        q.n = pr.n;
        q.d = pr.d;
        q.dtype = pr.dtype;
        q.X = pr.points;
        const size_t bytes = (size_t)pr.n * pr.d * dtype_size(pr.dtype);
        if (!o.points_on_device) {
            void *x = dev.raw_alloc(bytes, true);
            hip_ok(hipMemcpyAsync(x, pr.points, bytes, hipMemcpyHostToDevice, dev.s), "upload points");
            q.X = x;
        }
        perms[(size_t)p] = check_order(pr.order, pr.n);
        if (!perms[(size_t)p].empty()) {
            q.perm = dev.alloc<int32_t>((size_t)pr.n);
            hip_ok(hipMemcpyAsync(q.perm, perms[(size_t)p].data(), (size_t)pr.n * 4, hipMemcpyHostToDevice, dev.s),
                   "upload order");
        }
        const PointsView PV{q.X, q.n, q.d, q.dtype, q.perm};
        if (bad) hip_ok(launch_check_finite(q.X, q.dtype, q.n * (int64_t)q.d, bad + p, dev.s), "check_finite");
        q.nu = dev.alloc<double>((size_t)q.n);
        hip_ok(launch_point_stats(PV, q.nu, pstats + 2 * p, dev.s), "point_stats");
    }
    std::vector<unsigned long long> ps_h((size_t)2 * P);
    hip_ok(hipMemcpyAsync(ps_h.data(), pstats, ps_h.size() * 8, hipMemcpyDeviceToHost, dev.s), "stats D2H");
    std::vector<int> bad_h((size_t)P, 0);
    if (bad) hip_ok(hipMemcpyAsync(bad_h.data(), bad, (size_t)P * 4, hipMemcpyDeviceToHost, dev.s), "flags D2H");
    dev.sync();
    for (int p = 0; p < P; ++p) {
        if (bad_h[(size_t)p]) fail(BM_ENONFINITE, "a coordinate is NaN or infinite");
        std::memcpy(&pv[(size_t)p].max_nu, &ps_h[(size_t)2 * p], 8);
        std::memcpy(&pv[(size_t)p].max_abs, &ps_h[(size_t)2 * p + 1], 8);
    }

    // ---- operands: one path per problem, chosen at its smallest radius
    const int flags = device_flags(dev.dev, dev.s);
    if ((flags & 3) != 3) fail(BM_EINTERNAL, "matrix-core layout self-check failed on this device");
    for (int p = 0; p < P; ++p) {
        const bm_problem &pr = *probs[(size_t)p];
        Prob &q = pv[(size_t)p];
        double e2min = INFINITY;
        for (int e = 0; e < pr.n_eps; ++e) e2min = std::min(e2min, pr.eps[e] * pr.eps[e]);
        q.path = o.path != BM_PATH_AUTO ? o.path : auto_path(q.dtype, q.d, e2min, q.max_nu, q.max_abs);
        if (q.path == BM_PATH_FP32) fail(BM_EINTERNAL, "batched problem on the FP32 path");
        const PointsView PV{q.X, q.n, q.d, q.dtype, q.perm};
        bool have = false;
        if (o.path == BM_PATH_AUTO && q.path == BM_PATH_BF16X3 && split_is_costly(q.d)) {
            // one scaled-F16 product instead of the split if its band is thin at
            // the sweep's largest radius
            double e2max = 0.0;
            for (int e = 0; e < pr.n_eps; ++e) e2max = std::max(e2max, pr.eps[e] * pr.eps[e]);
            MfmaArgs f = prepare_mfma(dev, PV, q.nu, MFMA_F16, e2max, q.max_nu, q.max_abs, o.refine);
            if (prefer_f16(q.d, sample_band_rate(dev, PV, f, e2max))) {
                q.path = BM_PATH_F16;
                q.Pop = q.Qop = (uint16_t *)f.Pop;
                dev.release((void *)f.cinit);
                have = true;
            } else {
                release_mfma(dev, f);
            }
        }
        const int Kraw = (q.path == MFMA_BF16X3) ? 3 * q.d : q.d;
        q.S = (Kraw + 15) / 16;
        if (q.S > kMaxMfmaSteps) fail(BM_EINVAL, "d too large for this MFMA path");
        q.scale = (q.path == MFMA_F16) ? f16_scale(q.dtype, q.max_abs) : 1.0;
        if (!have) {
            const size_t words = mfma_operand_words(q.n, q.S);
            q.Pop = dev.alloc<uint16_t>(words);
            q.Qop = (q.path == MFMA_BF16X3) ? dev.alloc<uint16_t>(words) : q.Pop;
            hip_ok(launch_mfma_operands(PV, q.path, q.S, q.scale, q.Pop, q.Qop, dev.s), "mfma_operands");
        }
    }

    // ---- chains and their memory (three arenas: zeroed, +inf, uninitialised)
    std::vector<Chain> ch;
    Carve cz, ci, cp;
    const bool settle = o.refine != 0;
    int64_t nmax = 1, ntot = 0;
    for (int p = 0; p < P; ++p) {
        const bm_problem &pr = *probs[(size_t)p];
        const Prob &q = pv[(size_t)p];
        for (int e = 0; e < pr.n_eps; ++e) {
            Chain c;
            c.p = p;
            c.slot = slot0[(size_t)p] + e;
            c.eps = pr.eps[e];
            c.e2 = c.eps * c.eps;
            c.n = q.n;
            c.B = o.block ? o.block : batch_block(q.n, q.d, q.path);
            const int64_t nwords = (q.n + 63) / 64, np = (q.n + 31) / 32 * 32;
            const int nw = (c.B + 63) / 64;
            c.z_off = cz.off;                                       // (states: one array of their own)
            cz.take(nwords * 8);                                    // covered
            if (settle) {
                cz.take(nwords * 8);                                // islm
                cz.take(mfma_operand_words(q.n, q.S) * 2);          // settled operands
                cz.take(np * 4);                                    // settled indices
                c.i_off = ci.take(t3_floats(q.n) * 4);              // settled thresholds
            }
            cz.take((size_t)c.B * nw * 8);                          // conflict words (kept zero)
            c.p_off = cp.take(((size_t)q.n * 2 + t3_floats(q.n)) * 4);   // scalars
            cp.take((size_t)c.B * 4);                               // cand
            cp.take((size_t)c.B * 4);                               // rowflag
            cp.take((size_t)c.B * 4);                               // A
            cp.take((size_t)q.n * 4);                               // landmarks
            cp.take((size_t)q.n * 4);                               // landmark ranks
            cp.take((size_t)kBlockLogSize * sizeof(BlockLog));
            nmax = std::max(nmax, q.n);
            ntot += q.n;
            ch.push_back(c);
        }
    }
    const int nch = (int)ch.size();
    // the chains' states side by side, so that one copy reads them all back
    GreedyState *states = dev.alloc<GreedyState>((size_t)std::max(nch, 1));
    unsigned char *zero_arena = (unsigned char *)dev.raw_alloc(cz.off, true);
    unsigned char *inf_arena = ci.off ? (unsigned char *)dev.raw_alloc(ci.off, true) : nullptr;
    unsigned char *plain_arena = (unsigned char *)dev.raw_alloc(cp.off, true);
    for (size_t k = 0; k < ch.size(); ++k) {
        Chain &c = ch[k];
        const Prob &q = pv[(size_t)c.p];
        const int64_t nwords = (q.n + 63) / 64, np = (q.n + 31) / 32 * 32;
        const int nw = (c.B + 63) / 64;
        Carve z{c.z_off}, i{c.i_off}, pl{c.p_off};
        c.st = states + k;
        c.covered = (uint64_t *)(zero_arena + z.take(nwords * 8));
        if (settle) {
            c.islm = (uint64_t *)(zero_arena + z.take(nwords * 8));
            c.sd.Pop = (uint16_t *)(zero_arena + z.take(mfma_operand_words(q.n, q.S) * 2));
            c.sd.idx = (int32_t *)(zero_arena + z.take(np * 4));
            c.sd.T3 = (float *)(inf_arena + i.take(t3_floats(q.n) * 4));
        }
        c.C = (uint64_t *)(zero_arena + z.take((size_t)c.B * nw * 8));
        float *sc = (float *)(plain_arena + pl.take(((size_t)q.n * 2 + t3_floats(q.n)) * 4));
        c.cand = (int32_t *)(plain_arena + pl.take((size_t)c.B * 4));
        c.rowflag = (int32_t *)(plain_arena + pl.take((size_t)c.B * 4));
        c.A = (int32_t *)(plain_arena + pl.take((size_t)c.B * 4));
        c.lm = (int32_t *)(plain_arena + pl.take((size_t)q.n * 4));
        c.lm_rank = (int32_t *)(plain_arena + pl.take((size_t)q.n * 4));
        c.blog = (BlockLog *)(plain_arena + pl.take((size_t)kBlockLogSize * sizeof(BlockLog)));
        // this radius's accumulator starts, norm bounds and thresholds
        const double sc2 = q.scale * q.scale;
        const MfmaBound mb = mfma_bound(q.path, q.d, 16 * q.S, c.e2 * sc2, std::sqrt(q.max_nu) * q.scale,
                                        q.max_abs * q.scale, (flags & 4) != 0, q.dtype == BM_F16);
        hip_ok(launch_mfma_scalars(q.n, q.nu, sc2, mb, c.e2 * sc2, q.d, sc, sc + q.n, sc + 2 * q.n, dev.s),
               "mfma_scalars");
        c.ma = MfmaArgs{q.Pop, q.Qop, sc, sc + q.n, sc + 2 * q.n, f32_up(mb.alpha), q.S, q.path, o.refine};
    }

    // ---- one key buffer for every chain: chain << (bl + bn) | ordinal << bn | index
    const int32_t bn = std::max(1, bitlen((uint64_t)(nmax - 1)));
    const int32_t bl = std::max(1, bitlen((uint64_t)nmax));
    const int32_t bc = std::max(1, bitlen((uint64_t)(nch - 1)));
    unsigned long long *counters = dev.alloc<unsigned long long>(2);    // [0] keys, [1] chains done
    unsigned long long cap = o.init_member_capacity ? (unsigned long long)o.init_member_capacity
                                                    : (unsigned long long)std::max<int64_t>(4 * ntot, 1 << 20);
    uint64_t *keys = dev.alloc<uint64_t>(cap);

    // ---- descriptors: chains, and per operand class the range and resolve tasks
    ChainTask *ctask = dev.alloc<ChainTask>((size_t)nch);
    struct Class {
        int kind = 0, S = 0;
        RangeTask *rt = nullptr, *qt = nullptr;
        int32_t *rmap = nullptr, *qmap = nullptr;
        int64_t rwg = 0, qwg = 0;
    };
    std::map<std::pair<int, int>, std::vector<int>> by_class;
    for (int c = 0; c < nch; ++c) {
        const Prob &q = pv[(size_t)ch[(size_t)c].p];
        by_class[{q.path, q.S}].push_back(c);
    }
    std::vector<Class> classes;
    auto upload_tables = [&]() {
        std::vector<ChainTask> cts((size_t)nch);
        for (int c = 0; c < nch; ++c) {
            const Chain &k = ch[(size_t)c];
            const Prob &q = pv[(size_t)k.p];
            ChainTask &t = cts[(size_t)c];
            t = ChainTask{};
            t.covered = k.covered;
            t.n = k.n;
            t.st = k.st;
            t.B = k.B;
            t.settle = settle ? 1 : 0;
            t.cand = k.cand;
            t.rowflag = k.rowflag;
            t.islm = k.islm;
            t.a = k.ma;
            t.sd = k.sd;
            t.perm = q.perm;
            t.C = k.C;
            t.A = k.A;
            t.landmarks = k.lm;
            t.lm_rank = k.lm_rank;
            t.blog = k.blog;
            t.nkeys = counters;
            t.ndone = counters + 1;
        }
        dev.upload(ctask, cts.data(), cts.size() * sizeof(ChainTask));
    };
    auto build_classes = [&]() {
        for (auto &kv : by_class) {
            Class cl;
            cl.kind = kv.first.first;
            cl.S = kv.first.second;
            std::vector<RangeTask> rts, qts;
            std::vector<int32_t> rmap, qmap;
            for (int c : kv.second) {
                const Chain &k = ch[(size_t)c];
                const Prob &q = pv[(size_t)k.p];
                const PointsView PV{q.X, q.n, q.d, q.dtype, q.perm};
                const int nw = (k.B + 63) / 64;
                RangeTask r{};
                r.a = k.ma;
                r.P = PV;
                r.e2 = k.e2;
                r.A = k.A;
                r.blk = &k.st->L0;
                r.o = RangeOut{k.covered, keys, cap, counters, k.st, (uint64_t)c << (bn + bl), bn};
                r.sd = k.sd;
                r.chain = ctask + c;
                range_grid(k.B, k.n, chain_target_wg(k.n), &r.NGW, &r.chunks);
                r.wg0 = (int32_t)cl.rwg;
                cl.rwg += (int64_t)r.NGW * r.chunks;
                rmap.insert(rmap.end(), (size_t)r.NGW * r.chunks, (int32_t)rts.size());
                rts.push_back(r);
                RangeTask v{};
                v.a = k.ma;
                v.P = PV;
                v.n_dev = &k.st->nc;
                v.e2 = k.e2;
                v.A = k.cand;
                v.o = RangeOut{nullptr, nullptr, 0, counters, k.st, 0, 0};
                v.C32 = (uint32_t *)k.C;
                v.c32_stride = 2 * nw;
                v.rowflag = k.rowflag;
                v.chain = ctask + c;
                range_grid(k.B, k.B, resolve_target_wg_of(k.B), &v.NGW, &v.chunks);
                v.wg0 = (int32_t)cl.qwg;
                cl.qwg += (int64_t)v.NGW * v.chunks;
                qmap.insert(qmap.end(), (size_t)v.NGW * v.chunks, (int32_t)qts.size());
                qts.push_back(v);
            }
            if (cl.rwg > 0x7fffffffLL || cl.qwg > 0x7fffffffLL) fail(BM_EINVAL, "batch too large for one launch");
            cl.rt = dev.alloc<RangeTask>(rts.size());
            cl.qt = dev.alloc<RangeTask>(qts.size());
            cl.rmap = dev.alloc<int32_t>(rmap.size());
            cl.qmap = dev.alloc<int32_t>(qmap.size());
            dev.upload(cl.rt, rts.data(), rts.size() * sizeof(RangeTask));
            dev.upload(cl.qt, qts.data(), qts.size() * sizeof(RangeTask));
            dev.upload(cl.rmap, rmap.data(), rmap.size() * 4);
            dev.upload(cl.qmap, qmap.data(), qmap.size() * 4);
            classes.push_back(cl);
        }
    };

    // ---- the greedy of every chain
    const auto t_greedy = clk::now();
    std::vector<GreedyState> sts((size_t)nch);
    auto run_all = [&]() {
        hip_ok(hipMemsetAsync(zero_arena, 0, cz.off, dev.s), "zero arena");
        hip_ok(hipMemsetAsync(states, 0, (size_t)nch * sizeof(GreedyState), dev.s), "zero states");
        if (inf_arena)
            hip_ok(hipMemsetD32Async((hipDeviceptr_t)inf_arena, 0x7f800000, ci.off / 4, dev.s), "fill +inf");
        hip_ok(hipMemsetAsync(counters, 0, 16, dev.s), "zero counters");
        upload_tables();
        build_classes();
        hip_ok(launch_block_begin(ctask, nch, dev.s), "first blocks");
        auto enqueue_step = [&](hipStream_t s) {
            for (const Class &cl : classes)
                hip_ok(launch_range_tasks(cl.qt, cl.qmap, cl.qwg, cl.kind, cl.S, true, s), "resolve");
            for (const Class &cl : classes)
                hip_ok(launch_range_tasks(cl.rt, cl.rmap, cl.rwg, cl.kind, cl.S, false, s), "range");
        };
        constexpr int kGraphSteps = 8;
        GraphRunner gr;
        int reps = 1;
        int64_t steps = 0;
        for (;;) {
            if (!o.no_graph) {
                if (!gr.ready())
                    gr.capture([&](hipStream_t cs) {
                        for (int k = 0; k < kGraphSteps; ++k) enqueue_step(cs);
                    });
                for (int r = 0; r < reps; ++r) gr.launch(dev.s);
            } else {
                for (int k = 0; k < reps * kGraphSteps; ++k) enqueue_step(dev.s);
            }
            steps += (int64_t)reps * kGraphSteps;
            const unsigned long long done = dev.fetch(counters + 1);
            if (done >= (unsigned long long)nch) break;
            if (steps > nmax + 2 * kGraphSteps) fail(BM_EINTERNAL, "a chain did not finish");
            reps = std::min(reps * 2, 8);
        }
        hip_ok(hipMemcpyAsync(sts.data(), states, (size_t)nch * sizeof(GreedyState), hipMemcpyDeviceToHost, dev.s),
               "state D2H");
        dev.sync();
        return dev.fetch(counters);
    };
    unsigned long long M = run_all();
    if (M > cap) {                                                   // too small: once more, with room for all
        dev.release(keys);
        for (Class &cl : classes) {
            dev.release(cl.rt);
            dev.release(cl.qt);
            dev.release(cl.rmap);
            dev.release(cl.qmap);
        }
        classes.clear();
        cap = M;
        keys = dev.alloc<uint64_t>(cap);
        M = run_all();
        if (M != cap) fail(BM_EINTERNAL, "membership count changed on recompute");
    }
    for (const GreedyState &s : sts)
        if (s.error) fail(BM_EINTERNAL, "candidate acceptance did not converge");
    const double ms_greedy = ms_since(t_greedy);

    // ---- CSR and edges of the union of all chains
    const auto t_csr = clk::now();
    std::vector<int64_t> lm_off((size_t)nch + 1, 0), pt_off((size_t)nch + 1, 0);
    for (int c = 0; c < nch; ++c) {
        lm_off[(size_t)c + 1] = lm_off[(size_t)c] + (int64_t)sts[(size_t)c].L;
        pt_off[(size_t)c + 1] = pt_off[(size_t)c] + ch[(size_t)c].n;
    }
    const int64_t Ltot = lm_off[(size_t)nch], Ntot = pt_off[(size_t)nch];
    int64_t *lm_off_d = dev.alloc<int64_t>((size_t)nch + 1);
    int64_t *pt_off_d = dev.alloc<int64_t>((size_t)nch + 1);
    dev.upload(lm_off_d, lm_off.data(), lm_off.size() * 8);
    dev.upload(pt_off_d, pt_off.data(), pt_off.size() * 8);
    uint64_t *skeys = sort_into(dev, keys, (int64_t)M, bc + bl + bn);
    dev.release(keys);
    const int32_t bnu = std::max(1, bitlen((uint64_t)(Ntot - 1)));
    hip_ok(launch_union_keys(skeys, (int64_t)M, bn, bl, lm_off_d, pt_off_d, bnu, dev.s), "union keys");
    int64_t *row_ptr = nullptr;
    int32_t *midx = nullptr;
    csr_of(dev, skeys, (int64_t)M, Ltot, bnu, &row_ptr, &midx);
    dev.sync();
    const double ms_csr = ms_since(t_csr);
    const auto t_edges = clk::now();
    int32_t *edges = nullptr;
    int64_t *eptr = nullptr;
    const int64_t Etot = edges_of(dev, skeys, (int64_t)M, Ltot, Ntot, bnu, row_ptr, midx, &edges, &eptr, lm_off_d, nch);
    dev.release(skeys);
    std::vector<const int32_t *> lm_ptrs((size_t)nch);
    for (int c = 0; c < nch; ++c) lm_ptrs[(size_t)c] = ch[(size_t)c].lm;
    const int32_t **lm_ptrs_d = dev.alloc<const int32_t *>((size_t)nch);
    dev.upload(lm_ptrs_d, lm_ptrs.data(), lm_ptrs.size() * sizeof(void *));
    int32_t *lm_union = dev.alloc<int32_t>((size_t)std::max<int64_t>(Ltot, 1));
    int64_t *mp_union = dev.alloc<int64_t>((size_t)(Ltot + nch));
    int64_t *ranges = dev.alloc<int64_t>((size_t)4 * nch);
    hip_ok(launch_rebase_chains(nch, lm_ptrs_d, lm_off_d, pt_off_d, row_ptr, midx, eptr, edges, lm_union, mp_union,
                                ranges, dev.s),
           "rebase");
    std::vector<int64_t> rg((size_t)4 * nch);
    hip_ok(hipMemcpyAsync(rg.data(), ranges, rg.size() * 8, hipMemcpyDeviceToHost, dev.s), "ranges D2H");
    dev.sync();
    const double ms_edges = ms_since(t_edges);

    // ---- hand over: every result is a slice of the union arrays
    const auto t_dl = clk::now();
    std::vector<bm_result *> res((size_t)nch, nullptr);
    try {
        for (int c = 0; c < nch; ++c) res[(size_t)c] = new_result();
        std::shared_ptr<SharedResults> shared;
        std::vector<int32_t> lm_h, midx_h, edges_h;
        std::vector<int64_t> mp_h;
        if (o.results_on_device) {
            shared = std::make_shared<SharedResults>();
            shared->device = dev.dev;
            for (void *ptr : {(void *)lm_union, (void *)mp_union, (void *)midx, (void *)edges}) {
                dev.detach(ptr);
                shared->ptrs.push_back(ptr);
            }
        } else {
            lm_h.resize((size_t)std::max<int64_t>(Ltot, 1));
            mp_h.resize((size_t)(Ltot + nch));
            midx_h.resize((size_t)std::max<unsigned long long>(M, 1));
            edges_h.resize((size_t)std::max<int64_t>(2 * Etot, 1));
            if (Ltot) hip_ok(hipMemcpyAsync(lm_h.data(), lm_union, (size_t)Ltot * 4, hipMemcpyDeviceToHost, dev.s), "D2H");
            hip_ok(hipMemcpyAsync(mp_h.data(), mp_union, mp_h.size() * 8, hipMemcpyDeviceToHost, dev.s), "D2H");
            if (M) hip_ok(hipMemcpyAsync(midx_h.data(), midx, (size_t)M * 4, hipMemcpyDeviceToHost, dev.s), "D2H");
            if (Etot) hip_ok(hipMemcpyAsync(edges_h.data(), edges, (size_t)Etot * 8, hipMemcpyDeviceToHost, dev.s), "D2H");
            dev.sync();
        }
        const double ms_dl = ms_since(t_dl);
        const double ms_total = ms_since(t_start);
        for (int c = 0; c < nch; ++c) {
            const Chain &k = ch[(size_t)c];
            const GreedyState &s = sts[(size_t)c];
            bm_result *r = res[(size_t)c];
            const int64_t L = lm_off[(size_t)c + 1] - lm_off[(size_t)c];
            const int64_t m0 = rg[(size_t)4 * c], m1 = rg[(size_t)4 * c + 1];
            const int64_t e0 = rg[(size_t)4 * c + 2], e1 = rg[(size_t)4 * c + 3];
            r->n_landmarks = L;
            r->n_edges = e1 - e0;
            r->device = dev.dev;
            if (o.results_on_device) {
                r->landmarks = lm_union + lm_off[(size_t)c];
                r->member_ptr = mp_union + lm_off[(size_t)c] + c;
                r->member_idx = midx + m0;
                r->edges = edges + 2 * e0;
                r->on_device = 1;
                share_result(r, shared);
            } else {
                r->landmarks = (int32_t *)std::malloc((size_t)std::max<int64_t>(L, 1) * 4);
                r->member_ptr = (int64_t *)std::malloc((size_t)(L + 1) * 8);
                r->member_idx = (int32_t *)std::malloc((size_t)std::max<int64_t>(m1 - m0, 1) * 4);
                r->edges = (int32_t *)std::malloc((size_t)std::max<int64_t>(2 * (e1 - e0), 1) * 4);
                if (!r->landmarks || !r->member_ptr || !r->member_idx || !r->edges)
                    fail(BM_ENOMEM, "host allocation of the result failed");
                if (L) std::memcpy(r->landmarks, lm_h.data() + lm_off[(size_t)c], (size_t)L * 4);
                std::memcpy(r->member_ptr, mp_h.data() + lm_off[(size_t)c] + c, (size_t)(L + 1) * 8);
                if (m1 > m0) std::memcpy(r->member_idx, midx_h.data() + m0, (size_t)(m1 - m0) * 4);
                if (e1 > e0) std::memcpy(r->edges, edges_h.data() + 2 * e0, (size_t)(e1 - e0) * 8);
            }
            bm_stats &st = r->stats;
            st.ms_total = ms_total;
            st.ms_greedy = ms_greedy;
            st.ms_csr = ms_csr;
            st.ms_edges = ms_edges;
            st.ms_download = ms_dl;
            st.pairs_useful = L * k.n;
            st.range_pairs = (int64_t)s.range_pairs;
            st.pairs_issued = (int64_t)s.resolve_pairs + (int64_t)s.range_pairs;
            st.band_pairs = (int64_t)s.band;
            st.blocks = (int64_t)s.blocks;
            st.candidates = (int64_t)s.candidates;
            st.path = pv[(size_t)k.p].path;
            st.block = k.B;
        }
    } catch (...) {
        for (bm_result *r : res) bm_result_free(r);
        throw;
    }
    for (int c = 0; c < nch; ++c) outs[ch[(size_t)c].slot] = res[(size_t)c];
}

} // namespace host
} // namespace bm
