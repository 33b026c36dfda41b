// host_common.h — host-side helpers shared by the C-ABI drivers (api.cpp for
// one build, batch.cpp for many): errors, the device context with its
// tracked allocations and pinned staging, HIP graph replay, argument checks,
// the path and block-size choices.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "bm.h"
#include "bm_internal.h"
#include "bounds.h"
#include "kernels.h"
#include "tuned_blocks.h"

namespace bm {
namespace host {


inline thread_local std::string g_last_error;

struct BmError {
    int code;
    std::string msg;
};

[[noreturn]] inline void fail(int code, const std::string &msg) { throw BmError{code, msg}; }

inline void hip_ok(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
            fail(BM_ENOMEM, std::string(what) + ": " + hipGetErrorString(e));
        fail(BM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
}

using clk = std::chrono::steady_clock;
inline double ms_since(clk::time_point t0) { return std::chrono::duration<double, std::milli>(clk::now() - t0).count(); }

inline size_t dtype_size(int32_t dtype) { return dtype == BM_F64 ? 8 : dtype == BM_F32 ? 4 : 2; }

inline int bitlen(uint64_t v) { return v ? 64 - __builtin_clzll(v) : 0; }

// ---- process-wide cache of device memory, pinned staging and streams --------------------
// A build hands what it allocated back here once its stream has drained, and
// later builds on the same device take it instead of calling hipMalloc, hipFree
// (which waits for the whole device), hipHostMalloc and hipStreamCreate again.
// Device memory kept per device is bounded by BM_CACHE_BYTES (bytes; default an
// eighth of the device's memory, 0 keeps nothing); bm_trim_cache frees it.
constexpr size_t kPinnedBytes = 64 * 1024;
struct Cache {
    struct Dev {
        std::vector<std::pair<void *, size_t>> blocks;      // (pointer, size) of free device blocks
        size_t bytes = 0, limit = 0;
        bool limit_set = false;
        std::vector<void *> pinned;                         // free kPinnedBytes host buffers
        std::vector<hipStream_t> streams;                   // idle non-blocking streams
    };
    std::mutex mu;
    std::map<int, Dev> devs;
};
inline Cache &cache()
{
    static Cache *c = new Cache;                            // never destroyed: usable until exit
    return *c;
}
// Allocation sizes: powers of two up to 1 MiB, whole 2 MiB pages above.
inline size_t size_class(size_t b)
{
    if (b <= ((size_t)1 << 20)) {
        size_t c = 256;
        while (c < b) c <<= 1;
        return c;
    }
    const size_t page = (size_t)2 << 20;
    return (b + page - 1) / page * page;
}
// Best fit among `blocks` for a request of class `cls`: at most 50% larger.
inline int best_fit(const std::vector<std::pair<void *, size_t>> &blocks, size_t cls)
{
    int best = -1;
    for (size_t i = 0; i < blocks.size(); ++i) {
        const size_t z = blocks[i].second;
        if (z >= cls && z <= cls + cls / 2 && (best < 0 || z < blocks[(size_t)best].second)) best = (int)i;
    }
    return best;
}
inline Cache::Dev &cache_dev(Cache &c, int dev)             // (c.mu held)
{
    Cache::Dev &d = c.devs[dev];
    if (!d.limit_set) {
        d.limit_set = true;
        const char *env = std::getenv("BM_CACHE_BYTES");
        if (env && *env) {
            d.limit = (size_t)std::strtoull(env, nullptr, 10);
        } else {
            size_t total = 0;
            if (hipDeviceTotalMem(&total, dev) != hipSuccess) total = 0;
            d.limit = total / 8;
        }
    }
    return d;
}
inline void *cache_take(int dev, size_t cls, size_t *got)
{
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    Cache::Dev &d = cache_dev(c, dev);
    const int i = best_fit(d.blocks, cls);
    if (i < 0) return nullptr;
    void *p = d.blocks[(size_t)i].first;
    *got = d.blocks[(size_t)i].second;
    d.bytes -= *got;
    d.blocks.erase(d.blocks.begin() + i);
    return p;
}
// Keep a drained block (device `dev` current), or free it past the limit.
inline void cache_give(int dev, void *p, size_t bytes)
{
    Cache &c = cache();
    {
        std::lock_guard<std::mutex> lk(c.mu);
        Cache::Dev &d = cache_dev(c, dev);
        if (d.bytes + bytes <= d.limit) {
            d.blocks.emplace_back(p, bytes);
            d.bytes += bytes;
            return;
        }
    }
    (void)hipFree(p);
}
// Free the cached device blocks and pinned buffers of one device (-1: all);
// the caller has the device current when dev >= 0.
inline void cache_trim(int dev)
{
    Cache &c = cache();
    std::vector<std::pair<void *, size_t>> blocks;
    std::vector<void *> pinned;
    std::vector<int> owners;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        for (auto &kv : c.devs) {
            if (dev >= 0 && kv.first != dev) continue;
            for (auto &b : kv.second.blocks) {
                blocks.push_back(b);
                owners.push_back(kv.first);
            }
            kv.second.blocks.clear();
            kv.second.bytes = 0;
            pinned.insert(pinned.end(), kv.second.pinned.begin(), kv.second.pinned.end());
            kv.second.pinned.clear();
        }
    }
    int cur = -1;
    (void)hipGetDevice(&cur);
    for (size_t i = 0; i < blocks.size(); ++i) {
        (void)hipSetDevice(owners[i]);
        (void)hipFree(blocks[i].first);
    }
    if (cur >= 0) (void)hipSetDevice(cur);
    for (void *p : pinned) (void)hipHostFree(p);
}

// ---- device context: selected device, stream, tracked allocations ------------------------
constexpr size_t kUploadStage = kPinnedBytes - 4096;
constexpr int kUploadBlocks = 64;                   // blocks per table of directly launched passes
static_assert(kUploadBlocks * 32 <= 2048, "block table staging");
static_assert(kUploadBlocks * sizeof(RangeTask) <= kUploadStage, "task staging");
struct Device {
    int dev = 0, prev_dev = -1;
    hipStream_t s = nullptr;
    bool own_stream = false;
    int64_t budget = 0, used = 0;
    std::vector<std::pair<void *, size_t>> bufs;    // held by this build (size = allocated class)
    std::vector<std::pair<void *, size_t>> spare;   // released during the build: reusable on its stream
    void *pinned = nullptr;

    explicit Device(const bm_options &o)
    {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) fail(BM_ENODEVICE, "no HIP device is visible");
        hip_ok(hipGetDevice(&prev_dev), "hipGetDevice");
        dev = o.device < 0 ? prev_dev : o.device;
        if (dev >= count) fail(BM_ENODEVICE, "options.device is out of range");
        hip_ok(hipSetDevice(dev), "hipSetDevice");
        budget = o.max_device_bytes;
        {
            Cache &c = cache();
            std::lock_guard<std::mutex> lk(c.mu);
            Cache::Dev &d = cache_dev(c, dev);
            if (!o.stream && !d.streams.empty()) {
                s = d.streams.back();
                d.streams.pop_back();
                own_stream = true;
            }
            if (!d.pinned.empty()) {
                pinned = d.pinned.back();
                d.pinned.pop_back();
            }
        }
        if (o.stream) {
            s = (hipStream_t)o.stream;
        } else if (!s) {
            hip_ok(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
            own_stream = true;
        }
        if (!pinned) hip_ok(hipHostMalloc(&pinned, kPinnedBytes, hipHostMallocDefault), "hipHostMalloc");
    }
    ~Device()
    {
        // once the stream has drained, what this build holds goes back to the
        // cache; after a failed wait it is freed instead
        const bool drained = !s || hipStreamSynchronize(s) == hipSuccess;
        for (auto *list : {&bufs, &spare})
            for (auto &b : *list) {
                if (drained) cache_give(dev, b.first, b.second);
                else (void)hipFree(b.first);
            }
        bool kept_pinned = false, kept_stream = false;
        if (drained) {
            Cache &c = cache();
            std::lock_guard<std::mutex> lk(c.mu);
            Cache::Dev &d = cache_dev(c, dev);
            if (pinned) {
                d.pinned.push_back(pinned);
                kept_pinned = true;
            }
            if (own_stream && s) {
                d.streams.push_back(s);
                kept_stream = true;
            }
        }
        if (pinned && !kept_pinned) (void)hipHostFree(pinned);
        if (own_stream && s && !kept_stream) (void)hipStreamDestroy(s);
        if (prev_dev >= 0) (void)hipSetDevice(prev_dev);
    }
    Device(const Device &) = delete;
    Device &operator=(const Device &) = delete;

    // Free the spare blocks (waiting for the stream first).
    void drop_spare()
    {
        if (spare.empty()) return;
        sync();
        for (auto &b : spare) {
            (void)hipFree(b.first);
            used -= (int64_t)b.second;
        }
        spare.clear();
    }
    // A device block of at least `bytes`: from this build's spare blocks, the
    // cache, or hipMalloc (after freeing the cached blocks when that fails).
    void *raw_alloc(size_t bytes, bool tracked)
    {
        if (bytes == 0) bytes = 16;
        const size_t cls = size_class(bytes);
        void *p = nullptr;
        size_t got = 0;
        const int i = best_fit(spare, cls);
        if (i >= 0) {
            p = spare[(size_t)i].first;
            got = spare[(size_t)i].second;
            spare.erase(spare.begin() + i);
        } else {
            if (budget > 0 && used + (int64_t)cls > budget) drop_spare();
            if (budget > 0 && used + (int64_t)cls > budget)
                fail(BM_ENOMEM, "device memory cap (options.max_device_bytes) exceeded");
            p = cache_take(dev, cls, &got);
            if (p && budget > 0 && used + (int64_t)got > budget) {     // larger than the cap allows
                cache_give(dev, p, got);
                p = nullptr;
            }
            if (!p) {
                got = cls;
                hipError_t e = hipMalloc(&p, cls);
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    cache_trim(dev);
                    drop_spare();
                    e = hipMalloc(&p, cls);
                }
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    fail(BM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
                }
            }
            used += (int64_t)got;
        }
        if (tracked) bufs.emplace_back(p, got);
        return p;
    }
    template <class T> T *alloc(size_t count) { return (T *)raw_alloc(count * sizeof(T), true); }
    template <class T> T *zeros(size_t count)
    {
        T *p = alloc<T>(count);
        hip_ok(hipMemsetAsync(p, 0, std::max<size_t>(count * sizeof(T), 1), s), "hipMemsetAsync");
        return p;
    }
    // The block is no longer needed: later allocations of this build may reuse
    // it (they are ordered after its last use on the same stream).
    void release(void *p)
    {
        for (size_t i = 0; i < bufs.size(); ++i)
            if (bufs[i].first == p) {
                spare.push_back(bufs[i]);
                bufs.erase(bufs.begin() + (long)i);
                return;
            }
    }
    // stop tracking (ownership moves to a result)
    void detach(void *p)
    {
        for (size_t i = 0; i < bufs.size(); ++i)
            if (bufs[i].first == p) {
                bufs.erase(bufs.begin() + (long)i);
                return;
            }
    }
    void sync()
    {
        hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize");
        up_used = 0;
    }
    // Pinned host memory: [0, 4 KB) staging of small reads and block tables,
    // [4 KB, kPinnedBytes) staging of uploads.  Both wait for their copy.
    template <class T> T fetch(const T *dptr)
    {
        static_assert(sizeof(T) <= 2048, "fetch staging");
        hip_ok(hipMemcpyAsync((char *)pinned + 2048, dptr, sizeof(T), hipMemcpyDeviceToHost, s), "hipMemcpyAsync D2H");
        sync();
        T v;
        std::memcpy(&v, (char *)pinned + 2048, sizeof(T));
        return v;
    }
    // Uploads take consecutive pieces of the staging area and do not wait; the
    // stream is drained only when the area is full (every wait drains it, so
    // each one frees the whole area).
    void upload(void *dptr, const void *src, size_t bytes)
    {
        for (size_t off = 0; off < bytes; off += kUploadStage) {
            const size_t m = std::min(kUploadStage, bytes - off);
            if (up_used + m > kUploadStage) sync();
            char *stage = (char *)pinned + 4096 + up_used;
            std::memcpy(stage, (const char *)src + off, m);
            hip_ok(hipMemcpyAsync((char *)dptr + off, stage, m, hipMemcpyHostToDevice, s), "hipMemcpyAsync H2D");
            up_used += (m + 255) / 256 * 256;
        }
    }
    size_t up_used = 0;                                 // staging bytes in use since the last wait
};

// ---- argument checks that need no device ----------------------------------------------
inline void check_common(const void *points, int64_t n, int32_t d, int32_t dtype, double eps, const bm_options &o)
{
    if (n < 0) fail(BM_EINVAL, "n must be >= 0");
    if (n > INT32_MAX) fail(BM_EINVAL, "n must be <= INT32_MAX");
    if (d < 1) fail(BM_EINVAL, "d must be >= 1");
    if (dtype != BM_F64 && dtype != BM_F32 && dtype != BM_F16) fail(BM_EINVAL, "unknown dtype");
    if (!std::isfinite(eps) || !(eps > 0.0)) fail(BM_EINVAL, "eps must be finite and > 0");
    if (!(eps * eps > 0.0)) fail(BM_EINVAL, "eps*eps underflows to 0 in FP64");
    if (n > 0 && !points) fail(BM_EINVAL, "points is NULL");
    if (o.path < BM_PATH_AUTO || o.path > BM_PATH_F16) fail(BM_EINVAL, "unknown path");
    if (o.refine != 0 && o.refine != 1) fail(BM_EINVAL, "refine must be 0 or 1");
    if (o.block < 0 || o.block > kMaxBlock) fail(BM_EINVAL, "block must be 0 (automatic) or 1..16384");
    if (o.max_device_bytes < 0 || o.init_member_capacity < 0) fail(BM_EINVAL, "negative size option");
    if ((o.profile != 0 && o.profile != 1) || (o.no_graph != 0 && o.no_graph != 1))
        fail(BM_EINVAL, "profile and no_graph must be 0 or 1");
}

inline bool host_all_finite(const void *points, int64_t count, int32_t dtype)
{
    if (dtype == BM_F64) {
        const double *p = (const double *)points;
        for (int64_t i = 0; i < count; ++i)
            if (!std::isfinite(p[i])) return false;
    } else if (dtype == BM_F32) {
        const float *p = (const float *)points;
        for (int64_t i = 0; i < count; ++i)
            if (!std::isfinite(p[i])) return false;
    } else {
        const uint16_t *p = (const uint16_t *)points;
        for (int64_t i = 0; i < count; ++i)
            if ((p[i] & 0x7c00u) == 0x7c00u) return false;
    }
    return true;
}

inline std::vector<int32_t> check_order(const int64_t *order, int64_t n)
{
    std::vector<int32_t> perm;
    if (!order) return perm;
    std::vector<uint8_t> seen((size_t)n, 0);
    perm.resize((size_t)n);
    for (int64_t r = 0; r < n; ++r) {
        const int64_t p = order[r];
        if (p < 0 || p >= n || seen[(size_t)p]) fail(BM_EINVAL, "order is not a permutation of 0..n-1");
        seen[(size_t)p] = 1;
        perm[(size_t)r] = (int32_t)p;
    }
    return perm;
}

struct Pair64 {
    unsigned long long v[2];
};

inline int64_t range_target_wg()
{
    // about one workgroup per compute unit (256) unless BM_RANGE_WORKGROUPS says otherwise
    static const int64_t env_wg = [] {
        const char *e = getenv("BM_RANGE_WORKGROUPS");
        return e ? atoll(e) : 0LL;
    }();
    return env_wg > 0 ? env_wg : 256;
}
// Workgroups of a candidate resolve (B x B pairs, half of them above the
// diagonal and skipped): BM_RESOLVE_WORKGROUPS, else the range pass's target;
// the workgroups left below the diagonal then run in one round (measured: more
// and shorter workgroups are no faster at B = 8192 and slower at 16384).
inline int64_t resolve_target_wg()
{
    static const int64_t env_wg = [] {
        const char *e = getenv("BM_RESOLVE_WORKGROUPS");
        return e ? atoll(e) : 0LL;
    }();
    return env_wg > 0 ? env_wg : range_target_wg();
}

// A captured sequence of kernels replayed as one HIP graph.  Captured on a
// private stream (the caller's may be the legacy default stream, which cannot
// be captured), launched on any stream.  No memset nodes are captured: the
// block kernels clear what they need themselves.
struct GraphRunner {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    hipStream_t cs = nullptr;
    bool ready() const { return x != nullptr; }
    void reset()
    {
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
        x = nullptr;
        g = nullptr;
    }
    template <class F> void capture(F &&enqueue)
    {
        reset();
        if (!cs) hip_ok(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
        hip_ok(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
        try {
            enqueue(cs);
        } catch (...) {
            hipGraph_t dead = nullptr;
            (void)hipStreamEndCapture(cs, &dead);
            if (dead) (void)hipGraphDestroy(dead);
            throw;
        }
        hip_ok(hipStreamEndCapture(cs, &g), "end capture");
        hip_ok(hipGraphInstantiate(&x, g, nullptr, nullptr, 0), "graph instantiate");
    }
    void launch(hipStream_t s) { hip_ok(hipGraphLaunch(x, s), "graph launch"); }
    ~GraphRunner()
    {
        reset();
        if (cs) (void)hipStreamDestroy(cs);
    }
};
constexpr int kGraphBlocks = 8;                     // greedy blocks per captured graph
constexpr int64_t kGraphMaxPoints = 1 << 17;        // single builds replay graphs below this size
constexpr int64_t kProbePoints = 1 << 17;           // single builds from this size sample ball sizes
constexpr double kLargeBall = 512.0;                // sampled mean ball from which an automatic
constexpr int kLargeBallBlock = 2048;               // block is at most this size,
constexpr double kTinyBall = 2.0;                   // and below which it is at least this size
constexpr int kTinyBallBlock = 16384;

inline bm_result *new_result()
{
    bm_result *r = (bm_result *)std::calloc(1, sizeof(bm_result));
    if (!r) fail(BM_ENOMEM, "host allocation failed");
    return r;
}


// gfx950 matrix cores take float16 (and bf16) subnormal operands exactly; the
// device self-test (bm_device_selfcheck) verifies this before an MFMA path runs.
constexpr bool kF16SubnormalsOk = true;

inline std::mutex g_selfcheck_mu;
inline std::map<int, int> g_selfcheck;     // device -> flags

inline int device_flags(int dev, hipStream_t s)
{
    {
        std::lock_guard<std::mutex> lk(g_selfcheck_mu);
        auto it = g_selfcheck.find(dev);
        if (it != g_selfcheck.end()) return it->second;
    }
    int *fd = nullptr;
    hip_ok(hipMalloc(&fd, sizeof(int)), "hipMalloc");
    int flags = 0;
    hipError_t e = run_selfcheck(fd, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&flags, fd, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(fd);
    hip_ok(e, "device self-check");
    std::lock_guard<std::mutex> lk(g_selfcheck_mu);
    g_selfcheck[dev] = flags;
    return flags;
}

// Candidate block size when the options leave it automatic: the measured
// table (tuned_blocks.h) for the matrix-core paths, by cloud size otherwise.
inline int32_t tuned_block(int64_t n, int32_t d, bool batch)
{
    const TunedBlock *best = nullptr;
    for (const TunedBlock &t : kTunedBlocks) {
        if (n < t.n_min || d > t.d_max) continue;
        if (!best || t.n_min > best->n_min || (t.n_min == best->n_min && t.d_max < best->d_max)) best = &t;
    }
    if (!best) return 0;
    const int32_t B = batch ? best->batch : best->single;
    return std::min<int32_t>(std::max<int32_t>(B, 1), kMaxBlock);
}

inline int auto_block(int64_t n, int32_t d, int path)
{
    if (path == BM_PATH_FP32) {
        if (n >= (1 << 17)) return 1024;
        if (n >= (1 << 13)) return 256;
        return 64;
    }
    if (const int32_t B = tuned_block(n, d, false)) return B;
    if (n >= (1 << 17)) return 8192;
    if (n >= (1 << 13)) return 256;
    return 64;
}

// Path choice from the band each path would have at the largest norm, relative
// to eps^2: float16 storage -> F16 (exact operands); otherwise F16 on scaled
// data when its band is under 2% of eps^2 (same matrix-core cost as BF16 with
// an 8x narrower band), else the three-product BF16 split; FP32 when d is past
// the matrix-core kernel's K.
inline double band_fraction(int kind, int dtype, int d, double e2, double max_nu, double max_abs)
{
    const int K = ((kind == MFMA_BF16X3 ? 3 * d : d) + 15) / 16 * 16;
    const double s = (kind == MFMA_F16) ? f16_scale(dtype, max_abs) : 1.0;
    const MfmaBound b = mfma_bound(kind, d, K, e2 * s * s, std::sqrt(max_nu) * s, max_abs * s, true, dtype == BM_F16);
    const double half_width = 2.0 * ((b.alpha + b.beta) * max_nu * s * s + b.abs_err);
    return half_width / (e2 * s * s);
}

inline int auto_path(int dtype, int d, double e2, double max_nu, double max_abs)
{
    const int S1 = (d + 15) / 16, S3 = (3 * d + 15) / 16;
    if (S1 > kMaxMfmaSteps) return BM_PATH_FP32;
    if (dtype == BM_F16) return BM_PATH_F16;
    if (band_fraction(MFMA_F16, dtype, d, e2, max_nu, max_abs) <= 0.02) return BM_PATH_F16;
    if (S3 <= kMaxMfmaSteps) return BM_PATH_BF16X3;
    return BM_PATH_F16;
}


// ---- matrix-core operands and the automatic path ---------------------------------------------
// Operands of a matrix-core path (kind = BM_PATH_BF16 / BF16X3 / F16) and the
// per-point scalars of radius e2 (squared, data units).
inline MfmaArgs prepare_mfma(Device &dev, const PointsView &P, const double *nu, int kind, double e2, double max_nu,
                             double max_abs, int refine)
{
    const int64_t n = P.n;
    const int d = P.d;
    const int Kraw = (kind == MFMA_BF16X3) ? 3 * d : d;
    const int S = (Kraw + 15) / 16;
    if (S > kMaxMfmaSteps) fail(BM_EINVAL, "d too large for this MFMA path (use FP32, or BF16 for d <= 480)");
    const int flags = device_flags(dev.dev, dev.s);
    if ((flags & 3) != 3) fail(BM_EINTERNAL, "matrix-core layout self-check failed on this device");
    const size_t words = mfma_operand_words(n, S);
    uint16_t *Pop = dev.alloc<uint16_t>(words);
    uint16_t *Qop = (kind == MFMA_BF16X3) ? dev.alloc<uint16_t>(words) : Pop;
    // F16 on float32/float64 storage works in units scaled by a power of two
    const double scale = (kind == MFMA_F16) ? f16_scale(P.dtype, max_abs) : 1.0;
    hip_ok(launch_mfma_operands(P, kind, S, scale, Pop, Qop, dev.s), "mfma_operands");
    const double sc2 = scale * scale;
    const MfmaBound mb = mfma_bound(kind, d, 16 * S, e2 * sc2, std::sqrt(max_nu) * scale, max_abs * scale,
                                    (flags & 4) != 0, P.dtype == BM_F16);
    float *sc = dev.alloc<float>((size_t)n * 2 + t3_floats(n));
    hip_ok(launch_mfma_scalars(n, nu, sc2, mb, e2 * sc2, d, sc, sc + n, sc + 2 * n, dev.s), "mfma_scalars");
    MfmaArgs ma{};
    ma.Pop = Pop;
    ma.Qop = Qop;
    ma.cinit = sc;
    ma.nuup = sc + n;
    ma.T3 = sc + 2 * n;
    ma.alpha = f32_up(mb.alpha);
    ma.S = S;
    ma.kind = kind;
    ma.refine = refine;
    return ma;
}

inline void release_mfma(Device &dev, const MfmaArgs &ma)
{
    if (ma.Qop != ma.Pop) dev.release((void *)ma.Qop);
    dev.release((void *)ma.Pop);
    dev.release((void *)ma.cinit);
}

// One range pass of m landmarks at evenly spaced ranks against every point,
// keeping no membership: the fraction of pairs the filter leaves to the FP64
// recheck, and the mean number of members of a landmark's ball.
struct SampleStats {
    double band_rate = 0.0, ball_mean = 0.0;
};
inline SampleStats sample_pass(Device &dev, const PointsView &P, const MfmaArgs &ma, double e2, int m_max)
{
    SampleStats out;
    const int64_t n = P.n;
    const int m = (int)std::min<int64_t>(n, m_max);
    if (m <= 0) return out;
    std::vector<int32_t> ranks((size_t)m);
    for (int j = 0; j < m; ++j) ranks[(size_t)j] = (int32_t)(((int64_t)j * n) / m);
    int32_t *A = dev.alloc<int32_t>((size_t)m);
    int64_t *blk = dev.alloc<int64_t>(4);
    GreedyState *st = dev.zeros<GreedyState>(1);
    uint64_t *none = dev.alloc<uint64_t>(1);
    const int64_t blk_h[4] = {0, m, 0, 0};
    dev.upload(A, ranks.data(), (size_t)m * 4);
    dev.upload(blk, blk_h, sizeof blk_h);
    RangeTask t{};
    t.a = ma;
    t.P = P;
    t.e2 = e2;
    t.A = A;
    t.blk = blk;
    t.o = RangeOut{nullptr, none, 0, &st->nkeys, st, 0, 1};      // capacity 0: no key is kept
    range_grid(m, n, range_target_wg(), &t.NGW, &t.chunks);
    RangeTask *td = dev.alloc<RangeTask>(1);
    dev.upload(td, &t, sizeof t);
    hip_ok(launch_range_tasks(td, nullptr, (int64_t)t.NGW * t.chunks, ma.kind, ma.S, false, dev.s), "sample pass");
    const GreedyState h = dev.fetch(st);
    for (void *ptr : {(void *)A, (void *)blk, (void *)st, (void *)none, (void *)td}) dev.release(ptr);
    out.band_rate = (double)h.band / ((double)m * (double)n);
    out.ball_mean = (double)h.nkeys / (double)m;
    return out;
}
inline double sample_band_rate(Device &dev, const PointsView &P, const MfmaArgs &ma, double e2)
{
    return sample_pass(dev, P, ma, e2, 512).band_rate;
}

// The three-product split stops being almost free once its K passes 48 (below
// that the pass is bound by its epilogue, not by the matrix cores).
inline bool split_is_costly(int d) { return (3 * d + 15) / 16 > 3; }
// Scaled F16 (one product) instead of the split when its sampled band rate is
// below 5e-5 per matrix-core step saved: one FP64 recheck costs about as much
// as the products of tens of thousands of pairs.  A split past K = 128 does not
// fit the registers and reloads its landmark operands per point tile, which
// makes each of its steps about three times as costly.
inline bool prefer_f16(int d, double band_rate)
{
    const int S1 = (d + 15) / 16, S3 = (3 * d + 15) / 16;
    const double split_steps = (S3 > 8) ? 3.0 * S3 : (double)S3;
    return band_rate <= 5e-5 * (split_steps - S1);
}

// ---- results that share device arrays (a batch) ------------------------------------------
// Device arrays holding the results of one batch; freed with the last of them.
struct SharedResults {
    int device = 0;
    std::vector<void *> ptrs;
    ~SharedResults()
    {
        int prev = -1;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(device);
        for (void *p : ptrs) (void)hipFree(p);
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};
inline std::mutex g_shared_mu;
inline std::map<const bm_result *, std::shared_ptr<SharedResults>> g_shared;
inline void share_result(const bm_result *r, const std::shared_ptr<SharedResults> &s)
{
    std::lock_guard<std::mutex> lk(g_shared_mu);
    g_shared[r] = s;
}
// Drops r's share of a batch's arrays; false if r owns its arrays alone.
inline bool unshare_result(const bm_result *r)
{
    std::shared_ptr<SharedResults> keep;          // released after the lock
    std::lock_guard<std::mutex> lk(g_shared_mu);
    auto it = g_shared.find(r);
    if (it == g_shared.end()) return false;
    keep = std::move(it->second);
    g_shared.erase(it);
    return true;
}

// ---- membership CSR and edges from appended keys ------------------------------------------
// Keys are (row << bn) | column; rows 0..L-1 (landmark ordinals), columns
// 0..N-1 (original point indices).

// Sort the low end_bit bits of M keys into a new buffer.
inline uint64_t *sort_into(Device &dev, const uint64_t *keys, int64_t M, int end_bit)
{
    uint64_t *skeys = dev.alloc<uint64_t>((size_t)std::max<int64_t>(M, 1));
    if (M > 0) {
        size_t tb = 0;
        hip_ok(sort_keys(nullptr, &tb, keys, skeys, (size_t)M, end_bit, dev.s), "sort size");
        void *tmp = dev.raw_alloc(tb, true);
        hip_ok(sort_keys(tmp, &tb, keys, skeys, (size_t)M, end_bit, dev.s), "sort");
        dev.release(tmp);
    }
    return skeys;
}

// Row pointers and columns (ascending within a row) of sorted keys.
inline void csr_of(Device &dev, const uint64_t *skeys, int64_t M, int64_t L, int32_t bn, int64_t **row_ptr,
                   int32_t **midx)
{
    *row_ptr = dev.alloc<int64_t>((size_t)L + 1);
    *midx = dev.alloc<int32_t>((size_t)std::max<int64_t>(M, 1));
    hip_ok(launch_csr_from_sorted(skeys, M, L, bn, *row_ptr, *midx, dev.s), "csr");
}

// Exclusive scan of count values into out[0..count].
inline void scan_into(Device &dev, const int64_t *in, int64_t *out, int64_t count)
{
    size_t tb = 0;
    hip_ok(scan_excl_i64(nullptr, &tb, in, out, (size_t)count, dev.s), "scan size");
    void *tmp = dev.raw_alloc(std::max<size_t>(tb, 16), true);
    hip_ok(scan_excl_i64(tmp, &tb, in, out, (size_t)count, dev.s), "scan");
    dev.release(tmp);
}

// Edges (i, j), i < j, of rows that share a column, lexicographic, through the
// transpose S(x); only rows with a column in another row are visited.  seg (a
// batch's chain offsets, nseg + 1 entries on the device) bounds each row's
// neighbours to its chain.  Returns
// E and sets *edges (2 E ints); if eptr_out, keeps the per-row edge offsets
// (L + 1 entries, zeros for L <= 1 or M == 0).
inline int64_t edges_of(Device &dev, const uint64_t *skeys, int64_t M, int64_t L, int64_t N, int32_t bn,
                        const int64_t *row_ptr, const int32_t *midx, int32_t **edges, int64_t **eptr_out,
                        const int64_t *seg = nullptr, int nseg = 0)
{
    if (L <= 1 || M == 0) {
        *edges = dev.alloc<int32_t>(1);
        if (eptr_out) *eptr_out = dev.zeros<int64_t>((size_t)L + 1);
        return 0;
    }
    int64_t *cnt = dev.zeros<int64_t>((size_t)N);
    hip_ok(launch_point_degree(midx, M, cnt, dev.s), "point_degree");
    int64_t *sptr = dev.alloc<int64_t>((size_t)N + 1);
    scan_into(dev, cnt, sptr, N);
    int32_t *slist = dev.alloc<int32_t>((size_t)M);
    hip_ok(hipMemsetAsync(cnt, 0, (size_t)N * 8, dev.s), "zero fill");
    hip_ok(launch_fill_slists(skeys, M, bn, sptr, cnt, slist, dev.s), "fill_slists");
    dev.release(cnt);
    int *flag = dev.zeros<int>((size_t)L);
    int32_t *rows = dev.alloc<int32_t>((size_t)L);
    unsigned long long *nrows_d = dev.zeros<unsigned long long>(1);
    hip_ok(launch_edge_rows(skeys, M, bn, sptr, L, flag, rows, nrows_d, dev.s), "edge rows");
    const int64_t nrows = (int64_t)dev.fetch(nrows_d);
    dev.release(flag);
    // bitmaps of the large rows kept between the two passes (at most 2 GiB,
    // and a sixteenth of the device's memory)
    EdgeStore store{};
    const int64_t words = (L + 63) / 64;
    size_t total_mem = 0;
    if (hipDeviceTotalMem(&total_mem, dev.dev) != hipSuccess) total_mem = 0;
    const int64_t budget = std::min<int64_t>((int64_t)1 << 31, (int64_t)(total_mem / 16));
    store.cap = std::min<int64_t>(nrows, budget / (words * 8));
    if (store.cap > 0) {
        store.words = words;
        store.bits = dev.alloc<uint64_t>((size_t)(store.cap * words));
        store.count = dev.zeros<unsigned long long>(1);
        store.slots = dev.alloc<int32_t>((size_t)std::max<int64_t>(nrows, 1));
    } else {
        store.cap = 0;
    }
    int64_t *deg = dev.zeros<int64_t>((size_t)L);
    hip_ok(launch_edge_pass(0, nrows, rows, L, seg, nseg, row_ptr, midx, sptr, slist, deg, nullptr, nullptr, store,
                            dev.s),
           "edge count");
    int64_t *eptr = dev.alloc<int64_t>((size_t)L + 1);
    scan_into(dev, deg, eptr, L);
    const int64_t E = (int64_t)dev.fetch(eptr + L);
    *edges = dev.alloc<int32_t>((size_t)std::max<int64_t>(2 * E, 1));
    if (E > 0)
        hip_ok(launch_edge_pass(1, nrows, rows, L, seg, nseg, row_ptr, midx, sptr, slist, deg, eptr, *edges, store,
                                dev.s),
               "edge emit");
    if (store.bits) {
        dev.release(store.bits);
        dev.release(store.count);
        dev.release(store.slots);
    }
    dev.release(deg);
    dev.release(rows);
    dev.release(slist);
    dev.release(sptr);
    if (eptr_out) *eptr_out = eptr;
    else dev.release(eptr);
    return E;
}

} // namespace host
} // namespace bm
