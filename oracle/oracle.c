/*
 * Reference oracle for exact k-NN, k-selection, k-means, product quantization
 * and IVFADC search ("Billion-scale similarity search with GPUs", Johnson,
 * Douze, Jegou).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The GPU path never links,
 * calls or shares code with it.
 *
 * Everything here is the plain definition, written to be checked by eye:
 *   - every distance is accumulated in double precision from the float32
 *     inputs (each float widens exactly to double);
 *   - every selection is a full sort of (value, index) pairs followed by
 *     taking the first k, with equal values ordered by the lower index;
 *   - queries are independent, so an OpenMP loop runs over them; nothing else
 *     is blocked, fused or reordered.
 *
 * Status codes: 0 on success, -1 on invalid arguments, -3 on allocation
 * failure.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_L2 0
#define OR_IP 1

typedef struct {
    double v;
    int64_t i;
} pair_t;

/* Ascending value, then ascending index (Section 2: k-selection returns the
 * k lowest values in ascending order; ties go to the lower index). */
static int cmp_asc(const void* pa, const void* pb) {
    const pair_t* a = (const pair_t*)pa;
    const pair_t* b = (const pair_t*)pb;
    if (a->v < b->v) return -1;
    if (a->v > b->v) return 1;
    if (a->i < b->i) return -1;
    if (a->i > b->i) return 1;
    return 0;
}

/* Descending value ("highest values", Section 2, for inner products), then
 * ascending index. */
static int cmp_desc(const void* pa, const void* pb) {
    const pair_t* a = (const pair_t*)pa;
    const pair_t* b = (const pair_t*)pb;
    if (a->v > b->v) return -1;
    if (a->v < b->v) return 1;
    if (a->i < b->i) return -1;
    if (a->i > b->i) return 1;
    return 0;
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Write the first min(k, n) sorted pairs, pad the rest with (+-inf, -1). */
static void emit_topk(const pair_t* p, int64_t n, int32_t k, int largest,
                      double* D, int64_t* I) {
    for (int32_t r = 0; r < k; r++) {
        if (r < n) {
            D[r] = p[r].v;
            I[r] = p[r].i;
        } else {
            D[r] = largest ? -INFINITY : INFINITY;
            I[r] = -1;
        }
    }
}

/* Squared L2 distance in its direct form, sum_t (x_t - y_t)^2, in double. */
static double l2sq_f32(const float* x, const float* y, int32_t d) {
    double s = 0.0;
    for (int32_t t = 0; t < d; t++) {
        double diff = (double)x[t] - (double)y[t];
        s += diff * diff;
    }
    return s;
}

static double dot_f32(const float* x, const float* y, int32_t d) {
    double s = 0.0;
    for (int32_t t = 0; t < d; t++) s += (double)x[t] * (double)y[t];
    return s;
}

/*
 * Exact k-NN (Section 2, Eq. 1; inner products as the "highest values"
 * comparator).  For every query j and every database row i the distance is
 * computed in the direct form (not the norm decomposition of Eq. 2, which is
 * an implementation device), all nb pairs are sorted, and the first k are
 * returned.  Squared L2 is reported (the distance matrix D of Section 2 holds
 * squared distances; the argmin of Eq. 1 is the same).  Missing entries when
 * nb < k are (+inf, -1) for L2 and (-inf, -1) for inner product.
 * exclude, if non-NULL, names one database row per query that is left out of
 * that query's candidates (a node of a k-NN graph is not its own neighbour,
 * Section 6.5).
 */
int oracle_knn(const float* xq, int64_t nq, const float* xb, int64_t nb,
               int32_t d, int32_t k, int32_t metric, const int64_t* exclude,
               double* D, int64_t* I) {
    if (nq < 0 || nb < 0 || d < 1 || k < 1) return -1;
    if (metric != OR_L2 && metric != OR_IP) return -1;
    int fail = 0;
#pragma omp parallel
    {
        pair_t* p = (pair_t*)malloc(sizeof(pair_t) * (size_t)(nb > 0 ? nb : 1));
        if (!p) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = 0; j < nq; j++) {
            if (!p) continue;
            const float* x = xq + j * (int64_t)d;
            const int64_t skip = exclude ? exclude[j] : -1;
            int64_t n = 0;
            for (int64_t i = 0; i < nb; i++) {
                if (i == skip) continue;
                const float* y = xb + i * (int64_t)d;
                p[n].v = metric == OR_L2 ? l2sq_f32(x, y, d) : dot_f32(x, y, d);
                p[n].i = i;
                n++;
            }
            qsort(p, (size_t)n, sizeof(pair_t), metric == OR_L2 ? cmp_asc : cmp_desc);
            emit_topk(p, n, k, metric == OR_IP, D + j * (int64_t)k, I + j * (int64_t)k);
        }
        free(p);
    }
    return fail ? -3 : 0;
}

/*
 * Row-wise k-selection (Section 2): for every row a[0:len] return the k
 * lowest (or, with largest != 0, highest) values with their indices, by a full
 * sort of (a_i, i).
 */
int oracle_kselect(const float* a, int64_t nrows, int64_t len, int32_t k,
                   int32_t largest, double* vals, int64_t* idx) {
    if (nrows < 0 || len < 0 || k < 1) return -1;
    int fail = 0;
#pragma omp parallel
    {
        pair_t* p = (pair_t*)malloc(sizeof(pair_t) * (size_t)(len > 0 ? len : 1));
        if (!p) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < nrows; r++) {
            if (!p) continue;
            for (int64_t i = 0; i < len; i++) {
                p[i].v = (double)a[r * len + i];
                p[i].i = i;
            }
            qsort(p, (size_t)len, sizeof(pair_t), largest ? cmp_desc : cmp_asc);
            emit_topk(p, len, k, largest, vals + r * (int64_t)k, idx + r * (int64_t)k);
        }
        free(p);
    }
    return fail ? -3 : 0;
}

/*
 * k-means assignment step (k = 1 search, Section 6.2): for every point the
 * nearest centroid by squared L2 in double, ties to the lower centroid index.
 * The points are given in double so that residual vectors (exact differences
 * of float32 values) can be clustered without rounding.
 */
int oracle_kmeans_assign(const double* x, int64_t n, int32_t d, const float* c,
                         int32_t K, int64_t* assign, double* dist) {
    if (n < 0 || d < 1 || K < 1) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        const double* xi = x + i * (int64_t)d;
        double best = INFINITY;
        int64_t arg = -1;
        for (int32_t j = 0; j < K; j++) {
            const float* cj = c + (int64_t)j * d;
            double s = 0.0;
            for (int32_t t = 0; t < d; t++) {
                double diff = xi[t] - (double)cj[t];
                s += diff * diff;
            }
            if (s < best) { /* strict: an equal later centroid never wins */
                best = s;
                arg = j;
            }
        }
        assign[i] = arg;
        if (dist) dist[i] = best;
    }
    return 0;
}

/*
 * k-means update step: each centroid becomes the mean of its points, summed
 * in double and rounded once to float32 (round to nearest even).
 *
 * Empty clusters (the paper does not say how to treat them) are handled in
 * increasing index order: the currently largest cluster b (most points, ties
 * to the lower index) is split in two.  Coordinate t of the empty centroid
 * becomes c_b[t] * (1 + s_t * 2^-10) and c_b[t] becomes
 * c_b[t] * (1 - s_t * 2^-10), with s_t = +1 for even t and -1 for odd t,
 * each product formed in double and rounded to float32; the empty cluster
 * takes floor(count_b / 2) of b's count.
 *
 * On input c holds the previous centroids; on output the new ones.
 */
int oracle_kmeans_update(const double* x, int64_t n, int32_t d,
                         const int64_t* assign, int32_t K, float* c,
                         int64_t* counts) {
    if (n < 0 || d < 1 || K < 1) return -1;
    double* sum = (double*)calloc((size_t)K * (size_t)d, sizeof(double));
    if (!sum) return -3;
    for (int32_t j = 0; j < K; j++) counts[j] = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t a = assign[i];
        if (a < 0 || a >= K) {
            free(sum);
            return -1;
        }
        counts[a]++;
        for (int32_t t = 0; t < d; t++) sum[a * d + t] += x[i * (int64_t)d + t];
    }
    for (int32_t j = 0; j < K; j++) {
        if (counts[j] == 0) continue;
        for (int32_t t = 0; t < d; t++)
            c[(int64_t)j * d + t] = (float)(sum[(int64_t)j * d + t] / (double)counts[j]);
    }
    free(sum);
    const double eps = 1.0 / 1024.0;
    for (int32_t j = 0; j < K; j++) {
        if (counts[j] != 0) continue;
        int32_t b = 0;
        for (int32_t q = 1; q < K; q++)
            if (counts[q] > counts[b]) b = q;
        for (int32_t t = 0; t < d; t++) {
            double s = (t % 2 == 0) ? 1.0 : -1.0;
            double v = (double)c[(int64_t)b * d + t];
            c[(int64_t)j * d + t] = (float)(v * (1.0 + s * eps));
            c[(int64_t)b * d + t] = (float)(v * (1.0 - s * eps));
        }
        counts[j] = counts[b] / 2;
        counts[b] -= counts[j];
    }
    return 0;
}

/*
 * Product-quantizer encoding (Section 2, "Product quantizer"): the vector is
 * cut into M contiguous sub-vectors of d/M components; byte m of the code is
 * the index of the nearest of the 256 centroids of sub-quantizer m (squared L2
 * in double, ties to the lower index).  codebooks is [M][256][d/M].
 */
int oracle_pq_encode(const double* r, int64_t n, int32_t d, int32_t M,
                     const float* codebooks, uint8_t* codes) {
    if (n < 0 || d < 1 || M < 1 || d % M != 0) return -1;
    int32_t ds = d / M;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        for (int32_t m = 0; m < M; m++) {
            const double* sub = r + i * (int64_t)d + (int64_t)m * ds;
            double best = INFINITY;
            int32_t arg = 0;
            for (int32_t j = 0; j < 256; j++) {
                const float* cw = codebooks + ((int64_t)m * 256 + j) * ds;
                double s = 0.0;
                for (int32_t t = 0; t < ds; t++) {
                    double diff = sub[t] - (double)cw[t];
                    s += diff * diff;
                }
                if (s < best) {
                    best = s;
                    arg = j;
                }
            }
            codes[i * (int64_t)M + m] = (uint8_t)arg;
        }
    }
    return 0;
}

/*
 * IVFADC batch search (Section 5.3, Algorithm 4, with Eq. 5, Eq. 6 and
 * Eq. 10).  For each query:
 *   1. the probe set is the first nprobe coarse centroids in the order of
 *      (||x - c||^2 in double, centroid index)  -- Eq. 5;
 *   2. for every entry (code, id) of every probed list L the distance is
 *      sum_m || (x - c_L)^m - c_{m, code_m} ||^2 in double, i.e. the
 *      residual form of Eq. 10 (never the three-term split of Eq. 11);
 *   3. all (distance, id) pairs are sorted, ties to the lower id, and the
 *      first k are returned, padded with (+inf, -1)  -- Eq. 6.
 * nprobe_per_query, if non-NULL, gives each query its own nprobe and
 * overrides nprobe.  exclude, if non-NULL, names one id per query whose
 * entries are skipped (the query's own node when a k-NN graph is built by
 * searching the database against itself, Section 6.5).
 * Lists are in CSR form: entries list_offsets[L] .. list_offsets[L+1]-1 of
 * codes ([ntotal][M] bytes) and ids belong to list L.
 */
int oracle_ivfpq_search(const float* xq, int64_t nq, int32_t d,
                        const float* coarse, int32_t nlist, int32_t M,
                        const float* codebooks, const int64_t* list_offsets,
                        const uint8_t* codes, const int64_t* ids, int32_t k,
                        int32_t nprobe, const int32_t* nprobe_per_query,
                        const int64_t* exclude, double* D, int64_t* I) {
    if (nq < 0 || d < 1 || nlist < 1 || M < 1 || d % M != 0 || k < 1) return -1;
    int32_t ds = d / M;
    int64_t ntotal = list_offsets[nlist];
    int fail = 0;
#pragma omp parallel
    {
        pair_t* cp = (pair_t*)malloc(sizeof(pair_t) * (size_t)nlist);
        pair_t* ep = (pair_t*)malloc(sizeof(pair_t) * (size_t)(ntotal > 0 ? ntotal : 1));
        double* res = (double*)malloc(sizeof(double) * (size_t)d);
        if (!cp || !ep || !res) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = 0; j < nq; j++) {
            if (!cp || !ep || !res) continue;
            const float* x = xq + j * (int64_t)d;
            int32_t np = nprobe_per_query ? nprobe_per_query[j] : nprobe;
            if (np > nlist) np = nlist;
            if (np < 0) np = 0;
            for (int32_t c = 0; c < nlist; c++) {
                cp[c].v = l2sq_f32(x, coarse + (int64_t)c * d, d);
                cp[c].i = c;
            }
            qsort(cp, (size_t)nlist, sizeof(pair_t), cmp_asc);
            int64_t ne = 0;
            for (int32_t p = 0; p < np; p++) {
                int64_t L = cp[p].i;
                const float* cL = coarse + L * d;
                for (int32_t t = 0; t < d; t++) res[t] = (double)x[t] - (double)cL[t];
                for (int64_t e = list_offsets[L]; e < list_offsets[L + 1]; e++) {
                    if (exclude && ids[e] == exclude[j]) continue;
                    double s = 0.0;
                    for (int32_t m = 0; m < M; m++) {
                        const float* cw = codebooks + ((int64_t)m * 256 + codes[e * M + m]) * ds;
                        for (int32_t t = 0; t < ds; t++) {
                            double diff = res[m * ds + t] - (double)cw[t];
                            s += diff * diff;
                        }
                    }
                    ep[ne].v = s;
                    ep[ne].i = ids[e];
                    ne++;
                }
            }
            qsort(ep, (size_t)ne, sizeof(pair_t), cmp_asc);
            emit_topk(ep, ne, k, 0, D + j * (int64_t)k, I + j * (int64_t)k);
        }
        free(cp);
        free(ep);
        free(res);
    }
    return fail ? -3 : 0;
}
