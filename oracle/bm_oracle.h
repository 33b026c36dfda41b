/*
 * bm_oracle.h — FP64 brute-force Ball Mapper oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU path.
 *
 * Every function follows the paper's definitions literally (section numbers
 * refer to arXiv 2601.01405):
 *   - distance: Euclidean, evaluated as the plain squared sum of coordinate
 *     differences in FP64, compared against RN(eps*eps)              (Sec. 3.2, Sec. 2.1)
 *   - open balls B(c, eps) = { y : d(c, y) < eps }                    (Sec. 2.1, Def. of eps-net)
 *   - greedy eps-net: visit points in the given order, an uncovered point
 *     becomes a landmark and every point of its ball is marked covered (Sec. 2.2)
 *   - memberships X_i = X cap B(l_i, eps), the full ball              (Sec. 2.3)
 *   - Ball Mapper graph: edge (i,j) iff X_i cap X_j is non-empty       (Sec. 2.1, nerve 1-skeleton)
 *   - target-occupancy eps: median distance to the k-th nearest
 *     neighbour, the point itself counted first                       (Sec. 6.1)
 *   - covering radius rho(L) and separation s(L)                      (Sec. 6.2)
 */
#ifndef BM_ORACLE_H
#define BM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* stored dtype of the points: 0 = float64, 1 = float32, 2 = float16 (IEEE binary16 bits) */
enum { BMO_F64 = 0, BMO_F32 = 1, BMO_F16 = 2 };

typedef struct {
    int64_t  n_landmarks;
    int32_t *landmarks;   /* original point indices, selection order                     */
    int64_t *member_ptr;  /* n_landmarks + 1 row pointers                                 */
    int32_t *member_idx;  /* member_ptr[L] entries, ascending original index within a row */
    int64_t  n_edges;
    int32_t *edges;       /* 2 * n_edges: (i, j) landmark ordinals, i < j, lexicographic  */
} bmo_result;

/* Squared distance s(a,b) of two stored points: sequential k, no FMA.
 * Exposed so tests can compare it against exact rational arithmetic. */
double bmo_sqdist(const void *pts, int32_t d, int32_t dtype, int64_t a, int64_t b);

/* Greedy Ball Mapper.  order == NULL means index order.  early_exit != 0
 * enables the exact early exit of the distance loop once the partial sum
 * reaches RN(eps^2).  max_landmarks > 0 stops the greedy after that many
 * landmarks (a bounded sample for timing; memberships and edges then cover
 * only those landmarks).  Returns 0 on success, -1 on bad arguments,
 * -2 on allocation failure. */
int bmo_build(const void *pts, int64_t n, int32_t d, int32_t dtype, double eps,
              const int64_t *order, int32_t early_exit, int64_t max_landmarks,
              bmo_result *out);

/* Range sets of a fixed landmark list (no greedy): rows in landmark order. */
int bmo_range_sets(const void *pts, int64_t n, int32_t d, int32_t dtype, double eps,
                   const int32_t *landmarks, int64_t n_landmarks, bmo_result *out);

/* Edges of the nerve 1-skeleton from a membership CSR. */
int bmo_edges(int64_t n, int64_t n_landmarks, const int64_t *member_ptr,
              const int32_t *member_idx, bmo_result *out);

/* Target-occupancy scale: kdist[i] = distance from point i to its k-th
 * nearest neighbour, the point itself counted as the first; *eps_out = the
 * median of kdist (mean of the two middle values when n is even). */
int bmo_knn_eps(const void *pts, int64_t n, int32_t d, int32_t dtype, int32_t k,
                double *kdist, double *eps_out);

/* rho(L) = max over points of the distance to the nearest landmark. */
double bmo_covering_radius(const void *pts, int64_t n, int32_t d, int32_t dtype,
                           const int32_t *landmarks, int64_t n_landmarks);

/* s(L) = min over distinct landmark pairs of their distance (+inf if < 2). */
double bmo_separation(const void *pts, int64_t n, int32_t d, int32_t dtype,
                      const int32_t *landmarks, int64_t n_landmarks);

/* For each query point, the position in `landmarks` of the first landmark
 * whose ball holds it (-1 if none): the cover condition of the greedy. */
int bmo_first_member(const void *pts, int64_t n, int32_t d, int32_t dtype, double eps,
                     const int32_t *landmarks, int64_t n_landmarks, const int32_t *queries,
                     int64_t n_queries, int64_t *first);

/* OpenMP threads the oracle runs with. */
int bmo_threads(void);

void bmo_free(bmo_result *r);

#ifdef __cplusplus
}
#endif
#endif
