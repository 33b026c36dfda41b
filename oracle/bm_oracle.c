/*
 * bm_oracle.c — FP64 brute-force Ball Mapper oracle.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark.  It shares no code with the GPU path and
 * is deliberately plain: every landmark is compared with every point, one
 * coordinate at a time, in FP64.
 *
 * Must be compiled with -ffp-contract=off -fno-fast-math so that
 * `acc + t*t` is a multiply followed by an add, each rounded to nearest.
 *
 * Readings of the paper taken here (arXiv 2601.01405):
 *  - Membership is strict: d(c, y) < eps (open balls, Sec. 2.1 and the exact
 *    range set of Sec. 5).  The squared distance is compared with RN(eps^2);
 *    no square root is taken.
 *  - The greedy of Sec. 2.2 picks "an uncovered point"; we take the first
 *    uncovered point in the caller's order (index order by default).
 *  - A landmark's membership row is its full ball over all of X, including
 *    itself and points already covered by earlier landmarks (Sec. 2.3 X_i;
 *    the nerve of Sec. 2.1 intersects full balls).
 */
#include "bm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- exact widening of stored coordinates to FP64 ---------------------- */

static double half_bits_to_double(uint16_t h)
{
    int sign = (h >> 15) & 1;
    int e = (h >> 10) & 31;
    int m = h & 1023;
    double v;
    if (e == 0)
        v = ldexp((double)m, -24);                 /* zero / subnormal */
    else if (e == 31)
        v = m ? NAN : INFINITY;
    else
        v = ldexp((double)(m + 1024), e - 25);     /* normal */
    return sign ? -v : v;
}

static double coord(const void *pts, int32_t d, int32_t dtype, int64_t i, int32_t k)
{
    int64_t off = i * (int64_t)d + k;
    switch (dtype) {
    case BMO_F64: return ((const double *)pts)[off];
    case BMO_F32: return (double)((const float *)pts)[off];
    default:      return half_bits_to_double(((const uint16_t *)pts)[off]);
    }
}

/* Widen the whole data set once: n x d doubles, row-major. */
static double *widen(const void *pts, int64_t n, int32_t d, int32_t dtype)
{
    double *w = (double *)malloc((size_t)(n > 0 ? n : 1) * (size_t)d * sizeof(double));
    if (!w) return NULL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = 0; k < d; ++k)
            w[i * d + k] = coord(pts, d, dtype, i, k);
    return w;
}

/* ---- the distance (Sec. 3.2: squared Euclidean distance) --------------- */

/* s(a,b) = sum_k RN(RN(a_k - b_k)^2), summed left to right, each step
 * rounded to nearest.  If the partial sum reaches `stop` the loop ends early:
 * every term is >= 0 and rounded addition is monotone, so the full sum would
 * also be >= stop, and the comparison s < stop has the same outcome. */
static double sqdist_w(const double *a, const double *b, int32_t d, double stop)
{
    double acc = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        double t = a[k] - b[k];
        double sq = t * t;
        acc = acc + sq;
        if (acc >= stop) return acc;
    }
    return acc;
}

double bmo_sqdist(const void *pts, int32_t d, int32_t dtype, int64_t a, int64_t b)
{
    double acc = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        double t = coord(pts, d, dtype, a, k) - coord(pts, d, dtype, b, k);
        double sq = t * t;
        acc = acc + sq;
    }
    return acc;
}

/* ---- growable int32 buffer --------------------------------------------- */

typedef struct { int32_t *v; int64_t n, cap; } ibuf;

static int ibuf_push_many(ibuf *b, const int32_t *src, int64_t cnt)
{
    if (b->n + cnt > b->cap) {
        int64_t nc = b->cap ? b->cap : 1024;
        while (nc < b->n + cnt) nc *= 2;
        int32_t *nv = (int32_t *)realloc(b->v, (size_t)nc * sizeof(int32_t));
        if (!nv) return -1;
        b->v = nv; b->cap = nc;
    }
    memcpy(b->v + b->n, src, (size_t)cnt * sizeof(int32_t));
    b->n += cnt;
    return 0;
}

/* ---- one range query: R_eps(p) over all of X, ascending index ---------- */

typedef struct {
    int nthreads;
    int32_t **local;    /* per-thread member lists */
    int64_t *lcount;
    int64_t  chunk;
} rq_scratch;

static int rq_init(rq_scratch *s, int64_t n)
{
    int T = 1;
#ifdef _OPENMP
    T = omp_get_max_threads();
#endif
    s->nthreads = T;
    s->chunk = (n + T - 1) / T;
    if (s->chunk < 1) s->chunk = 1;
    s->local = (int32_t **)calloc((size_t)T, sizeof(int32_t *));
    s->lcount = (int64_t *)calloc((size_t)T, sizeof(int64_t));
    if (!s->local || !s->lcount) return -1;
    for (int t = 0; t < T; ++t) {
        s->local[t] = (int32_t *)malloc((size_t)s->chunk * sizeof(int32_t));
        if (!s->local[t]) return -1;
    }
    return 0;
}

static void rq_free(rq_scratch *s)
{
    if (s->local)
        for (int t = 0; t < s->nthreads; ++t) free(s->local[t]);
    free(s->local);
    free(s->lcount);
}

/* Thread t scans the contiguous index range [t*chunk, (t+1)*chunk) in order,
 * so concatenating the per-thread lists in thread order gives the members in
 * ascending index order. */
static int range_query(const double *w, int64_t n, int32_t d, double e2, int early_exit,
                       int64_t p, rq_scratch *s, ibuf *out, unsigned char *covered)
{
    const double stop = early_exit ? e2 : INFINITY;
    const double *lp = w + p * (int64_t)d;
#pragma omp parallel num_threads(s->nthreads)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        int64_t lo = (int64_t)t * s->chunk, hi = lo + s->chunk;
        if (hi > n) hi = n;
        int64_t c = 0;
        for (int64_t x = lo; x < hi; ++x) {
            double sx = sqdist_w(lp, w + x * (int64_t)d, d, stop);
            if (sx < e2) s->local[t][c++] = (int32_t)x;
        }
        s->lcount[t] = c;
    }
    for (int t = 0; t < s->nthreads; ++t) {
        if (ibuf_push_many(out, s->local[t], s->lcount[t])) return -1;
        if (covered)
            for (int64_t j = 0; j < s->lcount[t]; ++j) covered[s->local[t][j]] = 1;
    }
    return 0;
}

/* ---- edges of the nerve 1-skeleton -------------------------------------- */

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* E = { (i,j) : i < j, row_i and row_j share a point }.  Built through the
 * transpose: S(x) = landmarks whose ball contains x; for each landmark i the
 * neighbours j > i are the union of S(x) over x in row_i. */
int bmo_edges(int64_t n, int64_t L, const int64_t *mptr, const int32_t *midx, bmo_result *out)
{
    out->n_edges = 0;
    out->edges = NULL;
    if (L <= 1) return 0;
    int64_t M = mptr[L];
    int64_t *sptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *slist = (int32_t *)malloc((size_t)(M > 0 ? M : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!sptr || !slist || !fill) { free(sptr); free(slist); free(fill); return -2; }
    for (int64_t m = 0; m < M; ++m) sptr[midx[m] + 1]++;
    for (int64_t x = 0; x < n; ++x) sptr[x + 1] += sptr[x];
    memcpy(fill, sptr, (size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < L; ++i)          /* rows in order => each S(x) ascending */
        for (int64_t m = mptr[i]; m < mptr[i + 1]; ++m) slist[fill[midx[m]]++] = (int32_t)i;
    free(fill);

    int64_t *deg = (int64_t *)calloc((size_t)L + 1, sizeof(int64_t));
    int32_t **nb = (int32_t **)calloc((size_t)L, sizeof(int32_t *));
    int err = (!deg || !nb);
#pragma omp parallel if (!err)
    {
        int32_t *mark = (int32_t *)malloc((size_t)L * sizeof(int32_t));
        ibuf tmp = {0, 0, 0};
        if (!mark) {
#pragma omp atomic write
            err = 1;
        } else {
            for (int64_t j = 0; j < L; ++j) mark[j] = -1;
#pragma omp for schedule(dynamic, 16)
            for (int64_t i = 0; i < L; ++i) {
                tmp.n = 0;
                for (int64_t m = mptr[i]; m < mptr[i + 1]; ++m) {
                    int32_t x = midx[m];
                    for (int64_t q = sptr[x]; q < sptr[x + 1]; ++q) {
                        int32_t j = slist[q];
                        if (j > i && mark[j] != (int32_t)i) {
                            mark[j] = (int32_t)i;
                            if (ibuf_push_many(&tmp, &j, 1)) {
#pragma omp atomic write
                                err = 1;
                            }
                        }
                    }
                }
                qsort(tmp.v, (size_t)tmp.n, sizeof(int32_t), cmp_i32);
                deg[i] = tmp.n;
                if (tmp.n) {
                    nb[i] = (int32_t *)malloc((size_t)tmp.n * sizeof(int32_t));
                    if (nb[i]) memcpy(nb[i], tmp.v, (size_t)tmp.n * sizeof(int32_t));
                    else {
#pragma omp atomic write
                        err = 1;
                    }
                }
            }
        }
        free(mark);
        free(tmp.v);
    }
    int64_t E = 0;
    if (!err) {
        for (int64_t i = 0; i < L; ++i) E += deg[i];
        out->edges = (int32_t *)malloc((size_t)(E > 0 ? 2 * E : 2) * sizeof(int32_t));
        if (!out->edges) err = 1;
    }
    if (!err) {
        int64_t e = 0;
        for (int64_t i = 0; i < L; ++i)
            for (int64_t q = 0; q < deg[i]; ++q) {
                out->edges[2 * e] = (int32_t)i;
                out->edges[2 * e + 1] = nb[i][q];
                ++e;
            }
        out->n_edges = E;
    }
    if (nb)
        for (int64_t i = 0; i < L; ++i) free(nb[i]);
    free(nb);
    free(deg);
    free(sptr);
    free(slist);
    return err ? -2 : 0;
}

/* ---- greedy eps-net (Sec. 2.2) ------------------------------------------ */

static int check_args(const void *pts, int64_t n, int32_t d, int32_t dtype, double eps)
{
    if (n < 0 || d < 1 || n > 2147483647LL) return -1;
    if (n > 0 && !pts) return -1;
    if (dtype < BMO_F64 || dtype > BMO_F16) return -1;
    if (!(eps > 0.0) || !isfinite(eps)) return -1;
    if (!(eps * eps > 0.0)) return -1;
    return 0;
}

int bmo_build(const void *pts, int64_t n, int32_t d, int32_t dtype, double eps,
              const int64_t *order, int32_t early_exit, int64_t max_landmarks,
              bmo_result *out)
{
    memset(out, 0, sizeof(*out));
    if (check_args(pts, n, d, dtype, eps)) return -1;
    const double e2 = eps * eps;   /* RN(eps^2), computed once */

    double *w = widen(pts, n, d, dtype);
    unsigned char *covered = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    ibuf lm = {0, 0, 0}, mi = {0, 0, 0};
    int64_t *ptr = NULL, ptr_n = 0, ptr_cap = 0;
    rq_scratch s;
    memset(&s, 0, sizeof(s));
    int rc = 0;
    if (!w || !covered || rq_init(&s, n)) { rc = -2; goto done; }

    ptr_cap = 1024;
    ptr = (int64_t *)malloc((size_t)ptr_cap * sizeof(int64_t));
    if (!ptr) { rc = -2; goto done; }
    ptr[ptr_n++] = 0;

    for (int64_t r = 0; r < n; ++r) {
        int64_t p = order ? order[r] : r;
        if (covered[p]) continue;
        if (max_landmarks > 0 && lm.n >= max_landmarks) break;
        int32_t p32 = (int32_t)p;
        if (ibuf_push_many(&lm, &p32, 1)) { rc = -2; goto done; }
        covered[p] = 1;  /* p is in its own ball (s = 0 < e2); set explicitly too */
        if (range_query(w, n, d, e2, early_exit, p, &s, &mi, covered)) { rc = -2; goto done; }
        if (ptr_n == ptr_cap) {
            ptr_cap *= 2;
            int64_t *np = (int64_t *)realloc(ptr, (size_t)ptr_cap * sizeof(int64_t));
            if (!np) { rc = -2; goto done; }
            ptr = np;
        }
        ptr[ptr_n++] = mi.n;
    }

    out->n_landmarks = lm.n;
    out->landmarks = lm.v ? lm.v : (int32_t *)calloc(1, sizeof(int32_t));
    out->member_ptr = ptr;
    out->member_idx = mi.v ? mi.v : (int32_t *)calloc(1, sizeof(int32_t));
    lm.v = NULL; mi.v = NULL; ptr = NULL;
    rc = bmo_edges(n, out->n_landmarks, out->member_ptr, out->member_idx, out);

done:
    rq_free(&s);
    free(w);
    free(covered);
    free(lm.v);
    free(mi.v);
    free(ptr);
    if (rc) bmo_free(out);
    return rc;
}

int bmo_range_sets(const void *pts, int64_t n, int32_t d, int32_t dtype, double eps,
                   const int32_t *landmarks, int64_t L, bmo_result *out)
{
    memset(out, 0, sizeof(*out));
    if (check_args(pts, n, d, dtype, eps) || L < 0 || (L > 0 && !landmarks)) return -1;
    for (int64_t i = 0; i < L; ++i)
        if (landmarks[i] < 0 || landmarks[i] >= n) return -1;
    const double e2 = eps * eps;
    double *w = widen(pts, n, d, dtype);
    ibuf mi = {0, 0, 0};
    rq_scratch s;
    memset(&s, 0, sizeof(s));
    int64_t *ptr = (int64_t *)malloc((size_t)(L + 1) * sizeof(int64_t));
    int rc = 0;
    if (!w || !ptr || rq_init(&s, n)) { rc = -2; goto done; }
    ptr[0] = 0;
    for (int64_t i = 0; i < L; ++i) {
        if (range_query(w, n, d, e2, 1, landmarks[i], &s, &mi, NULL)) { rc = -2; goto done; }
        ptr[i + 1] = mi.n;
    }
    out->n_landmarks = L;
    out->landmarks = (int32_t *)malloc((size_t)(L > 0 ? L : 1) * sizeof(int32_t));
    if (!out->landmarks) { rc = -2; goto done; }
    if (L) memcpy(out->landmarks, landmarks, (size_t)L * sizeof(int32_t));
    out->member_ptr = ptr;
    out->member_idx = mi.v ? mi.v : (int32_t *)calloc(1, sizeof(int32_t));
    ptr = NULL; mi.v = NULL;
    rc = bmo_edges(n, L, out->member_ptr, out->member_idx, out);
done:
    rq_free(&s);
    free(w);
    free(mi.v);
    free(ptr);
    if (rc) bmo_free(out);
    return rc;
}

/* ---- target-occupancy eps (Sec. 6.1) ------------------------------------ */

static int cmp_f64(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

int bmo_knn_eps(const void *pts, int64_t n, int32_t d, int32_t dtype, int32_t k,
                double *kdist, double *eps_out)
{
    if (n < 1 || d < 1 || k < 1 || k > n || !pts || !kdist || !eps_out) return -1;
    double *w = widen(pts, n, d, dtype);
    if (!w) return -2;
    int err = 0;
#pragma omp parallel
    {
        double *row = (double *)malloc((size_t)n * sizeof(double));
        if (!row) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 8)
            for (int64_t i = 0; i < n; ++i) {
                for (int64_t j = 0; j < n; ++j)
                    row[j] = sqdist_w(w + i * (int64_t)d, w + j * (int64_t)d, d, INFINITY);
                qsort(row, (size_t)n, sizeof(double), cmp_f64);
                kdist[i] = sqrt(row[k - 1]);   /* row[0] is the point itself */
            }
        }
        free(row);
    }
    free(w);
    if (err) return -2;
    double *srt = (double *)malloc((size_t)n * sizeof(double));
    if (!srt) return -2;
    memcpy(srt, kdist, (size_t)n * sizeof(double));
    qsort(srt, (size_t)n, sizeof(double), cmp_f64);
    *eps_out = (n % 2) ? srt[n / 2] : 0.5 * (srt[n / 2 - 1] + srt[n / 2]);
    free(srt);
    return 0;
}

/* ---- Sec. 6.2 metrics --------------------------------------------------- */

double bmo_covering_radius(const void *pts, int64_t n, int32_t d, int32_t dtype,
                           const int32_t *landmarks, int64_t L)
{
    if (n < 1 || L < 1) return INFINITY;
    double *w = widen(pts, n, d, dtype);
    if (!w) return NAN;
    double worst = 0.0;
#pragma omp parallel for schedule(static) reduction(max : worst)
    for (int64_t x = 0; x < n; ++x) {
        double best = INFINITY;
        for (int64_t i = 0; i < L; ++i) {
            double s2 = sqdist_w(w + x * (int64_t)d, w + (int64_t)landmarks[i] * d, d, best);
            if (s2 < best) best = s2;
        }
        if (best > worst) worst = best;
    }
    free(w);
    return sqrt(worst);
}

double bmo_separation(const void *pts, int64_t n, int32_t d, int32_t dtype,
                      const int32_t *landmarks, int64_t L)
{
    if (L < 2) return INFINITY;
    double *w = widen(pts, n, d, dtype);
    if (!w) return NAN;
    double best = INFINITY;
#pragma omp parallel for schedule(dynamic, 16) reduction(min : best)
    for (int64_t i = 0; i < L; ++i) {
        double b = INFINITY;
        for (int64_t j = i + 1; j < L; ++j) {
            double s2 = sqdist_w(w + (int64_t)landmarks[i] * d, w + (int64_t)landmarks[j] * d, d, b);
            if (s2 < b) b = s2;
        }
        if (b < best) best = b;
    }
    free(w);
    return sqrt(best);
}

int bmo_first_member(const void *pts, int64_t n, int32_t d, int32_t dtype, double eps,
                     const int32_t *landmarks, int64_t L, const int32_t *queries, int64_t nq,
                     int64_t *first)
{
    if (check_args(pts, n, d, dtype, eps) || L < 0 || nq < 0) return -1;
    const double e2 = eps * eps;
    double *w = widen(pts, n, d, dtype);
    if (!w) return -2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nq; ++q) {
        int64_t f = -1;
        const double *xq = w + (int64_t)queries[q] * d;
        for (int64_t i = 0; i < L && f < 0; ++i)
            if (sqdist_w(w + (int64_t)landmarks[i] * d, xq, d, e2) < e2) f = i;
        first[q] = f;
    }
    free(w);
    return 0;
}

int bmo_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void bmo_free(bmo_result *r)
{
    if (!r) return;
    free(r->landmarks);
    free(r->member_ptr);
    free(r->member_idx);
    free(r->edges);
    memset(r, 0, sizeof(*r));
}
