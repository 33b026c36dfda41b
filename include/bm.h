/*
 * bm.h — Ball Mapper construction on one AMD Instinct MI355X (gfx950).
 *
 * C ABI of libbm.so.  Method: arXiv 2601.01405, "Exact and Approximate Range
 * Queries for Efficient Ball Mapper Construction".
 *
 *   - The greedy eps-net of Sec. 2.2: points are visited in `order`; the first
 *     uncovered point becomes a landmark and every point of its open ball
 *     B(l, eps) = { y : d(l, y) < eps } (Sec. 2.1) is marked covered.
 *   - Each landmark's fixed-radius range query R_eps(l) (Sec. 3 and the exact
 *     range set of Sec. 5) compares it with every point; the squared
 *     Euclidean distance is decomposed as |q|^2 + |x|^2 - 2 q.x (Sec. 3.2) and
 *     the inner products run on the matrix cores.
 *   - Memberships are the full balls X_i = X cap B(l_i, eps) (Sec. 2.3).
 *   - Edges are the 1-skeleton of the nerve: (i, j) whenever X_i and X_j share
 *     a point (Sec. 2.1).
 *
 * Exactness.  With refine = 1 (default) every membership decision equals the
 * FP64 predicate  s(a,b) < RN(eps*eps),  where s is the sum over k = 0..d-1,
 * left to right, of RN(RN(a_k - b_k)^2), each operation rounded to nearest,
 * without fused multiply-add, on the coordinates widened exactly to FP64.  A
 * low-precision estimate decides only the pairs provably far from the
 * threshold under a deterministic additive error bound (the delta-accurate
 * oracle of Sec. 5.1); pairs inside the band are recomputed with that FP64
 * sum (the verified range set of Sec. 5.3).  Landmarks, memberships and edges
 * are therefore identical across paths, block sizes and runs.
 * With refine = 0 the low-precision estimate decides every pair: a
 * compressed-distance range oracle of Sec. 5.4 with both false negatives and
 * false positives, bounded by the additive model of Sec. 5.1.
 *
 * Conventions shared by every entry point:
 *   - Return value: a bm_status.  On error *out is set to NULL, nothing is
 *     leaked, and bm_last_error() describes the cause.
 *   - Inputs are borrowed for the duration of the call and never retained.
 *   - Results are allocated by the library and released only by
 *     bm_result_free().  Arrays are host memory (malloc) unless
 *     options.results_on_device = 1, in which case they are device memory
 *     on options.device.
 *   - Calls are synchronous with respect to the host: when a call returns,
 *     all of its device work (on options.stream) has completed.
 *   - Thread safety: calls from different host threads are independent;
 *     bm_last_error() is per thread.
 */
#ifndef BM_H
#define BM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BM_ABI_VERSION 2

typedef enum {
    BM_OK = 0,
    BM_EINVAL = -1,      /* bad argument: n < 0, d < 1, eps not finite or <= 0 or RN(eps^2) == 0,
                            order not a permutation, NULL pointer with n > 0, n > INT32_MAX,
                            unknown dtype/path, bad option value                           */
    BM_ENOMEM = -2,      /* device or host allocation failed, or options.max_device_bytes exceeded */
    BM_ENODEVICE = -3,   /* no HIP device, or options.device out of range                    */
    BM_EDEVICE = -4,     /* a HIP runtime call failed (message has the HIP error string)     */
    BM_ENONFINITE = -5,  /* a coordinate is NaN or infinite                                  */
    BM_EINTERNAL = -6    /* an internal consistency check failed                             */
} bm_status;

typedef enum {           /* stored dtype of the points (row-major n x d)                     */
    BM_F64 = 0,
    BM_F32 = 1,
    BM_F16 = 2           /* IEEE binary16                                                    */
} bm_dtype;

typedef enum {           /* arithmetic of the range pass filter                              */
    BM_PATH_AUTO = 0,    /* F16 for float16 storage; else F16 (scaled) when its band at the
                            data's largest norm is under 2% of eps^2; else BF16X3, except that
                            past K = 48 for the split one sampled F16 pass (512 landmarks)
                            measures the pairs F16 would recheck and F16 is taken when they
                            are few; FP32 past d = 480                                       */
    BM_PATH_FP32 = 1,    /* FP32 direct difference on the vector ALUs (the plain baseline)   */
    BM_PATH_BF16 = 2,    /* one BF16 product per coordinate on MFMA, FP32 accumulation       */
    BM_PATH_BF16X3 = 3,  /* hi/lo BF16 split, three products per coordinate on MFMA          */
    BM_PATH_F16 = 4      /* FP16 operands on MFMA: the stored values for float16 storage
                            (exact); float32/float64 data scaled by a power of two into
                            float16 range and rounded to nearest                          */
} bm_path;

typedef struct {
    int32_t path;                 /* bm_path                                                   */
    int32_t refine;               /* 1 = exact (FP64 recheck of the band), 0 = unrefined       */
    int32_t block;                /* candidate block size B: 0 = automatic, else 1..16384       */
    int32_t device;               /* HIP device ordinal; -1 = the calling thread's current one */
    int32_t points_on_device;     /* 1: `points` is a device pointer on options.device          */
    int32_t results_on_device;    /* 1: result arrays stay in device memory                    */
    int64_t max_device_bytes;     /* 0 = unlimited; else BM_ENOMEM beyond this many bytes      */
    int64_t init_member_capacity; /* 0 = automatic; a small value exercises buffer regrowth    */
    void   *stream;               /* hipStream_t to run on; NULL = a library-owned stream      */
    int32_t profile;              /* 1: time the range passes: device-clock execution windows,
                                     plus HIP events on `stream` around each directly launched
                                     pass (not around passes replayed from a graph)           */
    int32_t no_graph;             /* 0: past its first few blocks the greedy of a cloud under
                                     2^17 points, and every batch, replays a captured HIP graph
                                     of the per-block kernels; 1: every kernel is launched
                                     directly                                                 */
} bm_options;

typedef struct {
    double  ms_total;             /* wall time of the call                                     */
    double  ms_prepare;           /* upload, validation, operand and threshold preparation     */
    double  ms_greedy;            /* candidate gather + resolve + range passes                 */
    double  ms_csr;               /* membership sort and row pointers                          */
    double  ms_edges;             /* edge build                                                */
    double  ms_download;          /* device-to-host copies of the results                      */
    int64_t pairs_useful;         /* n_landmarks * n: every ball over every point (Sec. 2.2)   */
    int64_t pairs_issued;         /* pairs evaluated: range passes + candidate-block resolve   */
    int64_t band_pairs;           /* pairs the low-precision filter could not decide           */
    int64_t blocks;               /* candidate blocks                                          */
    int64_t candidates;           /* candidates gathered over all blocks                       */
    int32_t path;                 /* path actually used                                        */
    int32_t block;                /* block size actually used                                  */
    double  ms_range_kernel;      /* summed execution windows of the range-pass launches, first
                                     wave start to last wave end on the device clock
                                     (profile = 1)                                             */
    int64_t range_launches;       /* range-pass launches                                       */
    int64_t range_pairs;          /* landmark-point pairs they evaluated; below pairs_useful
                                     on the refined matrix-core paths, which skip earlier
                                     landmarks (never in a later landmark's ball)             */
    double  ms_range_events;      /* summed HIP-event intervals around the same launches on the
                                     library's stream (profile = 1); each also holds the
                                     dispatch's wait behind the previous kernel               */
    double  ms_resolve_kernel;    /* summed execution windows of the matrix-core candidate
                                     resolves, first wave start to the last workgroup's exit
                                     before the accept it runs (profile = 1, single builds)   */
    double  ms_serial_steps;      /* summed device time of the serial steps between passes (the
                                     accept after each resolve, the opening of the next block
                                     after each range pass), each run by the last workgroup of
                                     its pass (profile = 1, single builds, matrix-core paths) */
} bm_stats;

typedef struct {
    int64_t  n_landmarks;
    int32_t *landmarks;           /* [n_landmarks] original point indices, selection order      */
    int64_t *member_ptr;          /* [n_landmarks + 1] CSR row pointers                         */
    int32_t *member_idx;          /* [member_ptr[n_landmarks]] original indices, ascending per row */
    int64_t  n_edges;
    int32_t *edges;               /* [2 * n_edges] (i, j) landmark ordinals, i < j, lexicographic */
    int32_t  on_device;           /* 1 if the arrays above are device memory                   */
    int32_t  device;              /* device they live on                                       */
    bm_stats stats;
} bm_result;

/* Fill *opt with the defaults: AUTO path, refine = 1, automatic block, current
 * device, host points and results, no memory cap, library-owned stream. */
int bm_default_options(bm_options *opt);

/*
 * Greedy Ball Mapper of one point cloud (Sec. 2.2 greedy, Sec. 2.1 nerve).
 *   points : n x d row-major coordinates of `dtype`; host pointer, or device
 *            pointer when opt->points_on_device.
 *   eps    : ball radius; membership is s(l, x) < RN(eps * eps).
 *   order  : host array, a permutation of 0..n-1 giving the visiting order;
 *            NULL = index order.
 *   opt    : NULL = defaults.
 *   out    : receives the result.
 * n == 0 gives BM_OK with an empty result.
 */
int bm_build(const void *points, int64_t n, int32_t d, int32_t dtype, double eps,
             const int64_t *order, const bm_options *opt, bm_result **out);

/* One problem of a batch: a point cloud and a sweep of radii. */
typedef struct {
    const void    *points;        /* as in bm_build (opt->points_on_device applies to all)      */
    int64_t        n;
    int32_t        d;
    int32_t        dtype;
    const double  *eps;           /* [n_eps] radii                                             */
    int32_t        n_eps;
    const int64_t *order;         /* NULL = index order                                        */
} bm_problem;

/*
 * Many independent Ball Mappers (every problem at every radius of its sweep).
 * outs must have room for sum(n_eps) pointers, filled problem-major,
 * radius-minor.  Each result is identical to the bm_build of that problem and
 * radius.  On error every slot is NULL.
 */
int bm_build_many(const bm_problem *probs, int32_t n_probs, const bm_options *opt,
                  bm_result **outs);

/*
 * Range sets of a fixed landmark list (the fixed-landmark mode of Sec. 6.2):
 * row i = { x : x in B(landmarks[i], eps) } under the options' path and
 * refine setting, plus the edges of those rows.  landmarks is a host array of
 * original indices in [0, n).  Used to score the unrefined path against the
 * exact one on the same vertex set.
 */
int bm_range_sets(const void *points, int64_t n, int32_t d, int32_t dtype, double eps,
                  const int32_t *landmarks, int64_t n_landmarks, const bm_options *opt,
                  bm_result **out);

/*
 * The deterministic error bound of a path (the additive model of Sec. 5.1,
 * used both to decide pairs exactly and to score the unrefined path).
 * For the MFMA paths the filter value G of landmark a and point x satisfies
 *     |G - (|x|^2 - D(a,x)) / 2| <= alpha |a|^2 + beta |x|^2 + abs_err,
 * D the exact squared distance, |.|^2 the squared norm of the stored point
 * widened to FP64.  For the FP32 path alpha = beta = 0 and rel_err is the
 * relative bound of the FP32 squared distance (the multiplicative model of
 * Sec. 5.2), abs_err its absolute part.  delta is the additive radius error of
 * Sec. 5.1 for points of squared norm <= max_sq_norm:
 *     delta = max(eps - sqrt(eps^2 - w), sqrt(eps^2 + w) - eps),
 * w the bound on |estimated D - D| at D = eps^2, including the FP32 rounding
 * of the unrefined threshold: with refine = 0 every lost or spurious
 * membership has its true distance in [eps - delta, eps + delta).
 * Inputs: path (not AUTO), dtype and d of the stored points, eps, the largest
 * squared norm and the largest |coordinate| of the data.  No device needed.
 */
typedef struct {
    double alpha, beta, abs_err, rel_err;
    double t_in, t_out;           /* D < t_in => s < RN(eps^2); D >= t_out => s >= RN(eps^2) */
    double delta;
    int32_t exact_range;          /* 0 if eps or the data leave the range where the
                                     bound holds (every pair is then rechecked) */
} bm_bound;
int bm_error_bound(int32_t path, int32_t dtype, int32_t d, double eps, double max_sq_norm, double max_abs,
                   bm_bound *out);

/*
 * Checks on `device` (-1 = current) the matrix-core behaviour the error bound
 * relies on and sets *flags: bit 0 bf16 and bit 1 f16 32x32x16 output layout
 * as the kernels assume; bit 2 f16 and bit 3 bf16 subnormal operands
 * multiplied exactly.  The MFMA paths run this once per device and refuse to
 * run (BM_EINTERNAL) if a layout bit is missing.
 */
int bm_device_selfcheck(int32_t device, int32_t *flags);

/*
 * Give back the memory the library keeps between calls.  Each call hands the
 * device blocks, pinned staging buffers and streams it used to a process-wide
 * cache once its stream has drained, and later calls on the same device reuse
 * them instead of allocating again (hipMalloc, hipFree and hipHostMalloc cost
 * tens to hundreds of microseconds each, and hipFree waits for the device).
 * Device memory kept is at most BM_CACHE_BYTES bytes per device (environment,
 * read once per device; default an eighth of the device's memory; 0 keeps
 * none).  This frees the cached device blocks and pinned buffers of `device`
 * (-1: every device); idle streams are kept.  Results are never cached: they
 * belong to the caller until bm_result_free.  Safe to call at any time from
 * any thread; calls in flight keep what they hold.  Returns BM_OK, or
 * BM_EINVAL for a device that does not exist.
 */
int bm_trim_cache(int32_t device);

/* Free a result from any entry point (host or device arrays).  NULL-safe. */
void bm_result_free(bm_result *r);

/* Message for the last failing call on this thread ("" if none). */
const char *bm_last_error(void);

/* Number of visible HIP devices (0 when there is none; never fails). */
int bm_device_count(void);

/* BM_ABI_VERSION of the loaded library. */
int bm_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BM_H */
