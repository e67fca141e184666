/*
 * mi_knn.h -- C ABI of the MI355X (gfx950) k-NN / IVFADC library.
 *
 * The operations follow "Billion-scale similarity search with GPUs"
 * (Johnson, Douze, Jegou): exact k-nearest-neighbour search with fused
 * k-selection (Sections 2 and 5.1) and IVFADC search over product-quantizer
 * codes (Sections 2, 5.2 and 5.3).
 *
 * Conventions for every call
 *   - Array arguments are DEVICE pointers unless the comment says "host".
 *     Matrices are dense, row-major, contiguous.  The caller owns all
 *     argument memory; the library never frees it.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls
 *     enqueue their kernels on it and return; outputs are valid once the
 *     stream has been synchronised.  Calls that must read a device value on
 *     the host (training, adding) synchronise the stream and say so.
 *   - Results of k-selections: row r holds the k best entries sorted best
 *     first -- squared L2 ascending, inner product descending -- with ties
 *     broken by the lower index.  If fewer than k candidates exist the tail
 *     is padded with distance +inf (L2) or -inf (inner product) and index -1.
 *   - The return value is a status; on error the outputs are unspecified,
 *     an index object is left as it was, and mk_last_error() describes the
 *     failure.  No call throws across the ABI.
 *   - k must satisfy 1 <= k <= 1024 (the register-resident selector holds at
 *     most 1024 entries, as WarpSelect in Section 4.2); larger k returns
 *     MK_ERR_UNSUPPORTED.
 *   - Scratch memory is taken from HIP's stream-ordered allocator and given
 *     back on the same stream.
 */
#ifndef MI_KNN_H
#define MI_KNN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MK_OK = 0,
    MK_ERR_INVALID_ARG = -1,
    MK_ERR_UNSUPPORTED = -2,
    MK_ERR_OOM = -3,
    MK_ERR_DEVICE = -4,
    MK_ERR_STATE = -5
} mk_status;

/* Section 2: L2 is the main metric; "highest values" for inner products. */
typedef enum { MK_METRIC_L2 = 0, MK_METRIC_IP = 1 } mk_metric;

typedef void* mk_stream_t; /* a hipStream_t */

/* Message for the last non-OK status returned on the calling thread. */
const char* mk_last_error(void);

/* Library ABI version (major * 100 + minor). */
int32_t mk_version(void);

/*
 * Squared L2 norms ||x_i||^2 of n rows of dimension d (Section 2, Eq. 2: the
 * norm terms take one pass over the matrix).
 *   x   [n, d] float32        out [n] float32
 */
mk_status mk_norms(const float* x, int64_t n, int32_t d, float* out, mk_stream_t stream);

/*
 * Linear pre-processing of rows, such as an OPQ rotation applied to database
 * and query vectors before indexing and search (Section 1: OPQ is a linear
 * transform of the inputs usable as pre-processing; Section 6.4 reduces
 * Deep1B with it): out[i][j] = sum_t rot[j][t] * x[i][t].
 *   x   [n, d] float32     rot [dout, d] float32 (a rotation: dout = d; a
 *                          projection: dout < d)     out [n, dout] float32
 * Device pointers, row-major; out must not overlap x (MK_ERR_INVALID_ARG).
 * FP32 matrix-core products, one fixed summation order per element, so the
 * result is deterministic; it errs from the exact product by at most about
 * d * 2^-24 * sum_t |rot[j][t] x[i][t]|.  Learning the rotation is not part
 * of the library.
 */
mk_status mk_rotate_rows(const float* x, int64_t n, int32_t d, const float* rot, int32_t dout,
                         float* out, mk_stream_t stream);

/*
 * Row-wise k-selection (Section 2 problem statement; Section 4.2 WarpSelect,
 * rebuilt for 64-lane wavefronts): for each row of a resident matrix return
 * the k lowest values (largest = 0) or the k highest (largest != 0) with
 * their column indices.
 *   a    [nrows, len] float32 (finite values)
 *   vals [nrows, k] float32   idx [nrows, k] int64
 * len may be smaller than k (padded as above).  nrows = 0 is a no-op.
 */
mk_status mk_kselect(const float* a, int64_t nrows, int64_t len, int32_t k, int32_t largest,
                     float* vals, int64_t* idx, mk_stream_t stream);

/*
 * Exact k-NN search (Section 2 Eq. 1-2; Section 5.1): distances of every
 * query to every database row, with the q.y GEMM term computed by FP32 MFMA
 * tiles whose outputs feed a register-resident k-selection in the same
 * kernel, followed by a merge of database-chunk partial results.
 *   xq [nq, d] float32, xb [nb, d] float32
 *   D  [nq, k] float32 -- squared L2 (ascending) or inner product
 *                         (descending), recomputed in the direct form
 *                         sum_t (x_t - y_t)^2 (or sum_t x_t y_t) in FP32 for
 *                         the returned rows
 *   I  [nq, k] int64
 * The selection keeps extra candidates beyond k (up to the 1024-entry
 * selector) and re-ranks them by the direct form, which removes the
 * cancellation error of ||x||^2 + ||y||^2 - 2<x,y>.  nb must be < 2^31.
 * Supported d: 1..256.  Scratch (device): nq x nchunks x S keys of 8 bytes,
 * nchunks <= 16, S = 64 R with R the smallest power of two such that 64 R
 * >= min(k + 16, 1024), doubled when 64 R >= 256 (candidate pools); plus
 * 16 bytes per (query, chunk) of shared rank points and, for L2 without
 * supplied norms, 4 bytes per database row.
 */
mk_status mk_knn_search(const float* xq, int64_t nq, const float* xb, int64_t nb, int32_t d,
                        int32_t k, mk_metric metric, float* D, int64_t* I, mk_stream_t stream);

/*
 * Exact k-NN against a database held in host memory (Section 5.1: inputs
 * larger than the GPU's memory stream in from the CPU).  The database is
 * copied in chunks of chunk_rows rows into two device buffers on a second
 * stream, the copy of chunk c + 1 overlapping the fused search of chunk c
 * on `stream`; each chunk's k best (mk_knn_search semantics, rows numbered
 * globally) are kept and one final k-selection over the chunks' lists keyed
 * (distance, row) gives the result.  Same contract as mk_knn_search (squared
 * L2 ascending or inner product descending, ties to the lower row, padding).
 *   xq [nq, d] float32 DEVICE, xb_host [nb, d] float32 HOST memory (pinned,
 *   e.g. hipHostMalloc, for the copies to overlap the searches),
 *   D [nq, k] float32 and I [nq, k] int64 DEVICE.
 * nb < 2^32 - 1; 1 <= chunk_rows < 2^31.  Device scratch: two chunk buffers
 * (2 chunk_rows d 4 bytes), nq k 12 bytes per chunk plus 8 bytes per key of
 * nq k ceil(nb / chunk_rows), and mk_knn_search's scratch for one chunk.
 * Synchronises `stream` before returning (the internal copy stream and its
 * events are released).
 */
mk_status mk_knn_search_host(const float* xq, int64_t nq, const float* xb_host, int64_t nb,
                             int32_t d, int32_t k, mk_metric metric, int64_t chunk_rows,
                             float* D, int64_t* I, mk_stream_t stream);

/*
 * As mk_knn_search, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Results are identical to mk_knn_search on the same arguments.  The call
 * allocates nothing: its scratch (the database norms for L2, the chunk partial
 * keys and the rank points, sized as documented for mk_knn_search) is carved
 * from one fixed device array of MK_NOALLOC_SCRATCH_BYTES per GPU, which the
 * library holds until the process ends.  A call whose scratch would exceed it
 * returns MK_ERR_UNSUPPORTED before anything is enqueued (split the queries).
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (concurrent streams or host threads) race and must be serialised by the
 * caller; successive calls on one stream are safe.  The first call on a
 * device looks up the array's device address (no allocation).
 */
#define MK_NOALLOC_SCRATCH_BYTES (64u << 20)
mk_status mk_knn_search_noalloc(const float* xq, int64_t nq, const float* xb, int64_t nb,
                                int32_t d, int32_t k, mk_metric metric, float* D, int64_t* I,
                                mk_stream_t stream);

/*
 * As mk_knn_search, with the database norms ||y_i||^2 supplied by the caller
 * (e.g. from mk_norms on a resident database; ignored for MK_METRIC_IP and
 * may then be NULL).  yn [nb] float32.
 */
mk_status mk_knn_search_prenorm(const float* xq, int64_t nq, const float* xb, const float* yn,
                                int64_t nb, int32_t d, int32_t k, mk_metric metric, float* D,
                                int64_t* I, mk_stream_t stream);

/*
 * Rows node0 .. node0 + nnodes - 1 of the exact k-nearest-neighbour graph of
 * the database (Section 6.5: every vector searched against the whole
 * database): for each node i the k best rows j != i by the metric of
 * mk_knn_search (squared L2 ascending or inner product descending, ties to the
 * lower row), the node itself left out.  Computed as the k + 1 best, with the
 * node removed from them if present.
 *   xb [nb, d] float32 (nodes are its rows), D [nnodes, k] float32,
 *   I [nnodes, k] int64 (padded (+-inf, -1) when nb - 1 < k).
 * 1 <= k <= 1023 (one entry of the 1024-entry selector goes to the node).
 * Scratch: nnodes (k + 1) 12 bytes plus that of mk_knn_search with k + 1.
 */
mk_status mk_knn_graph(const float* xb, int64_t nb, int32_t d, int32_t k, mk_metric metric,
                       int64_t node0, int64_t nnodes, float* D, int64_t* I, mk_stream_t stream);

/*
 * k-means assignment step (Section 6.2: exact search with k = 1): for each
 * point the nearest centroid (squared L2, ties to the lower index) and that
 * squared distance (direct form, FP32).
 *   x [n, d] float32, c [K, d] float32, assign [n] int64, dist [n] float32
 *   (dist may be NULL).
 */
mk_status mk_kmeans_assign(const float* x, int64_t n, int32_t d, const float* c, int32_t K,
                           int64_t* assign, float* dist, mk_stream_t stream);

/*
 * k-means update step (Section 2 "The quantizers": q1 is trained by k-means):
 * each centroid becomes the mean of its points, accumulated in FP64 and
 * rounded once to FP32.  Empty clusters are processed in increasing index
 * order: the currently largest cluster b (ties to the lower index) is split,
 * coordinate t of the empty centroid becoming c_b[t] * (1 + s_t 2^-10) and
 * c_b[t] becoming c_b[t] * (1 - s_t 2^-10), s_t = +1 for even t and -1 for
 * odd t (products in FP64, rounded to FP32); the empty cluster takes
 * floor(count_b / 2) of b's count.
 *   x [n, d], assign [n] int64 in [0, K) (points with other values are
 *   ignored), c [K, d] float32 in/out, counts [K] int64 out (may be NULL).
 * Every step, the empty-cluster rule included, runs on the device.
 */
mk_status mk_kmeans_update(const float* x, int64_t n, int32_t d, const int64_t* assign,
                           int32_t K, float* c, int64_t* counts, mk_stream_t stream);

/*
 * Product-quantizer encoding (Section 2 "Product quantizer"): byte m of a
 * vector's code is the nearest (squared L2, ties to the lower index) of the
 * 256 centroids of sub-quantizer m over components [m d/M, (m+1) d/M).
 *   r [n, d] float32, codebooks [M, 256, d/M] float32, codes [n, M] uint8
 */
mk_status mk_pq_encode(const float* r, int64_t n, int32_t d, int32_t M, const float* codebooks,
                       uint8_t* codes, mk_stream_t stream);

/* ------------------------------------------------------------------------
 * Low-precision brute force with exact re-rank (an extension of the exact
 * search of Section 5.1; the paper computes distances in FP32 only).
 * ------------------------------------------------------------------------ */
typedef enum { MK_PREC_FP32 = 0, MK_PREC_BF16 = 1, MK_PREC_FP8E4M3 = 2, MK_PREC_FP16 = 3 } mk_precision;

/* Row stride, in elements, of low-precision copies: d rounded up to 16. */
int32_t mk_lowp_stride(int32_t d);

/*
 * Low-precision copy of n rows of dimension d (d <= 256):
 *   MK_PREC_BF16:    out [n, ld] of BF16 (2 bytes, round to nearest even);
 *   MK_PREC_FP8E4M3: out [n, ld] of OCP E4M3 (1 byte, round to nearest even)
 *                    of the row multiplied by a power of two s_i with
 *                    max_t |x_it| s_i in (224, 448] (s_i = 1 for a zero row);
 *                    inv_scales [n] float32 receives 1 / s_i.
 * ld = mk_lowp_stride(d); elements d..ld-1 are zero.  inv_scales may be NULL
 * for BF16 (otherwise it receives 1).
 */
mk_status mk_quantize_rows(const float* x, int64_t n, int32_t d, int32_t prec, void* out,
                           float* inv_scales, mk_stream_t stream);

/*
 * Brute-force k-NN whose q.y term runs on BF16 or FP8-E4M3 matrix cores with
 * FP32 accumulation (queries quantized inside the call as above, the FP8
 * product rescaled by both rows' 1/s): the rerank_R best candidates per query
 * by that approximate score are kept, their distances are recomputed from the
 * FP32 rows in the direct form, and the k best of them are returned exactly
 * as mk_knn_search reports them.
 *   xq [nq, d], xb [nb, d] float32; xb_lp / xb_inv: mk_quantize_rows(xb);
 *   yn [nb] FP32 norms of xb (L2; NULL: computed); k <= rerank_R <= 1024.
 *   D [nq, k] float32, I [nq, k] int64.
 */
mk_status mk_knn_search_lowp(const float* xq, int64_t nq, const float* xb, const void* xb_lp,
                             const float* xb_inv, const float* yn, int64_t nb, int32_t d,
                             int32_t k, int32_t rerank_R, mk_metric metric, int32_t prec,
                             float* D, int64_t* I, mk_stream_t stream);

/* ------------------------------------------------------------------------
 * IVFADC index (Section 2 Eq. 3-6; Section 5.2-5.3): coarse quantizer q1
 * with nlist centroids, product quantizer q2 with M sub-quantizers of 256
 * centroids (8-bit codes) on the residual y - q1(y), inverted lists holding
 * codes and ids.  L2 only.  All index storage is resident in device memory
 * and owned by the object.
 * ------------------------------------------------------------------------ */
typedef struct mk_ivfpq mk_ivfpq;

/* d >= 1, nlist >= 1, M in {4, 8, ..., 128} with d % M == 0 (Section 5.2
 * allows any multiple of 4 up to 64 sub-quantizers; M > 64 needs the
 * 16-bit lookup tables of mk_ivfpq_set_scan_options to search).  Allocates nothing on
 * the device until training. */
mk_status mk_ivfpq_create(int32_t d, int32_t nlist, int32_t M, mk_ivfpq** out);

void mk_ivfpq_destroy(mk_ivfpq* index);

/*
 * Train q1 by k-means on xt (nt >= nlist rows, nt >= 256) then q2 by M
 * independent 256-centroid k-means on the sub-vectors of the residuals of xt
 * to the final coarse centroids, niter iterations each.  Initial centroids
 * are rows of xt given by the caller (host arrays):
 *   coarse_init_rows [nlist] int64, pq_init_rows [M, 256] int64.
 * Also builds the query-independent term-1 table of Eq. 11.  Synchronises.
 * Training again discards any added vectors.
 */
mk_status mk_ivfpq_train(mk_ivfpq* index, const float* xt, int64_t nt, int32_t niter,
                         const int64_t* coarse_init_rows, const int64_t* pq_init_rows,
                         mk_stream_t stream);

/*
 * Encode nb vectors and append them to their inverted lists with ids
 * ntotal, ntotal+1, ... (entries of a list stay in id order).  Synchronises.
 */
mk_status mk_ivfpq_add(mk_ivfpq* index, const float* xb, int64_t nb, mk_stream_t stream);

/* Number of vectors added so far. */
int64_t mk_ivfpq_ntotal(const mk_ivfpq* index);

/*
 * IVFADC search (Algorithm 4 of Section 5.3): probe the nprobe nearest
 * coarse centroids (Eq. 5), scan their lists with PQ lookup tables built
 * from the three-term split of Eq. 11 and staged in LDS, select the k
 * nearest of the scanned entries (Eq. 6).  D are ADC squared distances
 * (FP32), I the ids.  1 <= nprobe <= min(nlist, 1024).  The tables and the
 * per-list merge buffers must fit 64 KiB of LDS: 1024 M + 32 k <= 65536
 * bytes (any k for M <= 32, k <= 256 for M = 64); with 16-bit tables
 * (mk_ivfpq_set_scan_options) 512 M + 32 k <= 65536.
 *   xq [nq, d] float32, D [nq, k] float32, I [nq, k] int64
 */
mk_status mk_ivfpq_search(mk_ivfpq* index, const float* xq, int64_t nq, int32_t k,
                          int32_t nprobe, float* D, int64_t* I, mk_stream_t stream);

/*
 * Rows node0 .. node0 + nnodes - 1 of the approximate k-NN graph of the
 * indexed vectors (Section 6.5): each added vector with id i (row i of xb,
 * the array that was added, ids 0 .. ntotal - 1) is searched against the
 * index as by mk_ivfpq_search, and entries with id i are skipped, so a node
 * is never its own neighbour.  With R > 0 each node's short list of the R
 * best entries by ADC distance (itself excluded) is re-ranked exactly
 * against xb as by mk_ivfpq_search_rerank.  Nodes are processed in batches
 * of 32768 queries on `stream`.
 *   xb [ntotal, d] float32, D [nnodes, k] float32 (ADC distances, or exact
 *   squared distances when R > 0), I [nnodes, k] int64.
 * node0 + nnodes <= ntotal; R = 0 or k <= R <= 1024.
 */
mk_status mk_ivfpq_knn_graph(mk_ivfpq* index, const float* xb, int64_t node0, int64_t nnodes,
                             int32_t k, int32_t nprobe, int32_t R, float* D, int64_t* I,
                             mk_stream_t stream);

/*
 * IVFADC search as above for a short list of the R best entries by ADC
 * distance, then an exact re-rank of that list: each entry's squared L2
 * distance is recomputed in FP32 from the full-precision database row
 * xb[id] (direct form, as in mk_knn_search) and the k best by
 * (distance, id) are returned.  The re-rank is an extension of Algorithm 4,
 * not part of it: ADC distances are only accurate to the quantisation error,
 * which bounds how well neighbours inside one cluster can be told apart.
 *   xq [nq, d], xb [nb, d] float32 (device; nb >= ntotal, row i is the
 *   vector added with id i), D [nq, k] float32, I [nq, k] int64.
 * 1 <= k <= R <= 1024; the LDS bound of mk_ivfpq_search holds with R in
 * place of k.  Entries short of R (probed lists too short) are skipped;
 * a tail with fewer than k candidates is padded with (+inf, -1).
 */
mk_status mk_ivfpq_search_rerank(mk_ivfpq* index, const float* xq, int64_t nq, int32_t k,
                                 int32_t nprobe, int32_t R, const float* xb, int64_t nb,
                                 float* D, int64_t* I, mk_stream_t stream);

/*
 * Copy the trained quantizers to host arrays (any pointer may be NULL):
 *   coarse [nlist, d] float32, codebooks [M, 256, d/M] float32.
 * Synchronises.
 */
mk_status mk_ivfpq_get_quantizers(const mk_ivfpq* index, float* coarse, float* codebooks);

/*
 * Replace the quantizers with host arrays of the same shapes (as after
 * training; the term-1 table is rebuilt and any added vectors are
 * discarded).  Synchronises.
 */
mk_status mk_ivfpq_set_quantizers(mk_ivfpq* index, const float* coarse, const float* codebooks,
                                  mk_stream_t stream);

/*
 * Copy the inverted lists to host arrays (any pointer may be NULL):
 *   offsets [nlist + 1] int64 (CSR), codes [ntotal, M] uint8,
 *   ids [ntotal] int64.  Synchronises.
 */
mk_status mk_ivfpq_get_lists(const mk_ivfpq* index, int64_t* offsets, uint8_t* codes,
                             int64_t* ids);

/*
 * Write a trained index to the file `path` (Section 5.3's resident layout:
 * the quantizers and the inverted lists).  Format, little-endian: 8-byte
 * magic "MKIVFPQ\0", u32 version 1, i32 d, i32 nlist, i32 M, i64 ntotal,
 * coarse centroids f32 [nlist, d], codebooks f32 [M, 256, d / M], list
 * offsets i64 [nlist + 1], codes u8 [ntotal, M], ids i64 [ntotal].
 * Tables derived from these (centroid norms, the term-1 tables of Eq. 11)
 * are not stored.  Synchronises the device.  MK_ERR_STATE before training;
 * MK_ERR_INVALID_ARG when the file cannot be written.
 */
mk_status mk_ivfpq_save(const mk_ivfpq* index, const char* path);

/*
 * Create an index from a file written by mk_ivfpq_save; the caller owns
 * *out (mk_ivfpq_destroy).  The derived tables are rebuilt on the device
 * with the kernels of train and add, so searches of the loaded index equal
 * those of the saved one bit for bit.  Synchronises.  A file that is not an
 * index file, is truncated, has trailing bytes or inconsistent list offsets
 * gives MK_ERR_INVALID_ARG (checked on the host; the header before any
 * device work) and *out = NULL.  Ids are taken as stored.
 */
mk_status mk_ivfpq_load(const char* path, mk_ivfpq** out);


/* ------------------------------------------------------------------------
 * Learned probe count.  An extension of the fixed probe count tau of
 * Section 2 (Eq. 5 probes the tau nearest coarse centroids of every query):
 * a perceptron with two ReLU hidden layers predicts log2(tau) per query from
 * the query and its 32 smallest squared coarse distances, and the search
 * probes tau_q = clamp(ceil(2^(prediction + delta)), 1, cap) lists.
 * Features are standardised per column with a stored mean and standard
 * deviation before the first layer.  Matrix products run on the matrix cores
 * in FP32 or BF16 (FP32 accumulation); weights, gradients and the Adam
 * moments are FP32.  All arrays are device memory unless stated otherwise.
 * ------------------------------------------------------------------------ */

typedef struct mk_mlp mk_mlp;

/*
 * din inputs (d + 32 for an index of dimension d), hidden units per layer,
 * prec MK_PREC_FP32 or MK_PREC_BF16.  Parameters start at zero and the
 * standardisation at mean 0, deviation 1.
 */
mk_status mk_mlp_create(int32_t din, int32_t hidden, mk_precision prec, mk_mlp** out);
void mk_mlp_destroy(mk_mlp* net);

/* Length of the flat parameter vector: W1 [hidden, din] row-major, b1
 * [hidden], W2 [hidden, hidden], b2 [hidden], w3 [hidden], b3 [1]. */
int64_t mk_mlp_num_params(const mk_mlp* net);

/* Load parameters from a host array (the caller draws the initial values);
 * resets the Adam moments and step count.  Synchronises. */
mk_status mk_mlp_set_params(mk_mlp* net, const float* theta);

/* Copy parameters and the last gradient to host arrays (either may be
 * NULL).  Synchronises. */
mk_status mk_mlp_get_params(const mk_mlp* net, float* theta, float* grad);

/* Per-column mean and population standard deviation of n raw feature rows
 * F [n, din] (device), summed in FP64 on the host after one copy of F (a
 * column without spread gets deviation 1).  Synchronises. */
mk_status mk_mlp_fit_standardization(mk_mlp* net, const float* F, int64_t n,
                                     mk_stream_t stream);

/* Copy the stored means and 1/deviations to host arrays [din] (either may
 * be NULL).  Synchronises. */
mk_status mk_mlp_get_standardization(const mk_mlp* net, float* mean, float* inv_std);

/* yhat [n] = network(standardised F [n, din]). */
mk_status mk_mlp_forward(const mk_mlp* net, const float* F, int64_t n, float* yhat,
                         mk_stream_t stream);

/*
 * Mean squared error of the batch rows F[rows[i]] (rows may be NULL: rows
 * 0 .. B-1) against targets y[rows[i]], and its gradient, which is kept as
 * the network's last gradient (read it with mk_mlp_get_params).  loss: a
 * device float, may be NULL.
 */
mk_status mk_mlp_loss_grad(mk_mlp* net, const float* F, const int64_t* rows, int64_t B,
                           const float* y, float* loss, mk_stream_t stream);

/*
 * One pass over n rows in the order perm [n] (a permutation drawn by the
 * caller): batches of `batch` rows, each a forward pass, the gradient of
 * its mean squared error and one Adam step (beta1 0.9, beta2 0.999,
 * eps 1e-8, learning rate lr).  losses: device floats, one per batch, may
 * be NULL.
 */
mk_status mk_mlp_train_epoch(mk_mlp* net, const float* F, int64_t n, const float* y,
                             const int64_t* perm, int32_t batch, float lr, float* losses,
                             mk_stream_t stream);

/*
 * Write / read a network: 8-byte magic "MKMLP\0\0\0", u32 version 1, i32 din,
 * i32 hidden, i32 precision, i64 Adam step count, then f32 arrays: the
 * parameters, both Adam moments (mk_mlp_num_params each), the feature means
 * and 1 / standard deviations [din].  A loaded network predicts and trains
 * on exactly as the saved one.  The caller owns *out (mk_mlp_destroy).  Both
 * synchronise the device; bad or truncated files give MK_ERR_INVALID_ARG.
 */
mk_status mk_mlp_save(const mk_mlp* net, const char* path);
/* din, hidden and precision of a network; any output pointer may be NULL. */
mk_status mk_mlp_shape(const mk_mlp* net, int32_t* din, int32_t* hidden, int32_t* prec);
mk_status mk_mlp_load(const char* path, mk_mlp** out);

/* Raw network features of nq queries: F [nq, d + 32] = [xq ; the 32
 * smallest squared coarse distances, ascending].  Needs nlist >= 32. */
mk_status mk_ivfpq_probe_features(const mk_ivfpq* index, const float* xq, int64_t nq, float* F,
                                  mk_stream_t stream);

/*
 * Training labels: for query q with nearest-neighbour id nn_ids[q], the
 * 1-based rank of the list holding that id in the query's coarse order
 * (cap when it is not among the first cap); label [nq] int32 (may be NULL)
 * and target [nq] float = log2(label).  1 <= cap <= min(nlist, 1024).
 */
mk_status mk_ivfpq_probe_labels(const mk_ivfpq* index, const float* xq, int64_t nq,
                                const int64_t* nn_ids, int32_t cap, float* target,
                                int32_t* label, mk_stream_t stream);

/*
 * IVFADC search probing tau_q lists per query (see above) with
 * 32 <= cap <= min(nlist, 1024).  R = 0: ADC distances as in
 * mk_ivfpq_search; R >= k: exact re-rank of an R-entry short list against
 * xb [nb, d] as in mk_ivfpq_search_rerank.  nprobe_used [nq] int32 (may be
 * NULL) receives tau_q.  Asynchronous like the other searches.
 */
mk_status mk_ivfpq_search_learned(mk_ivfpq* index, const mk_mlp* net, float delta,
                                  const float* xq, int64_t nq, int32_t k, int32_t cap, int32_t R,
                                  const float* xb, int64_t nb, float* D, int64_t* I,
                                  int32_t* nprobe_used, mk_stream_t stream);

/* Dimension d of an index. */
int32_t mk_ivfpq_dim(const mk_ivfpq* index);

/*
 * List-scan options of an index, used by every later search call on it
 * (fixed or learned probe count, re-rank, k-NN graph, serving):
 *   lut_precision  MK_PREC_FP32 (default) or MK_PREC_FP16: the per-query
 *                  table -2 term3 of Eq. 11 staged in LDS in 16-bit floats
 *                  (Section 5.3 notes 16-bit tables as the way to larger M):
 *                  half the LDS and half the bytes per lookup, each entry
 *                  rounded once (relative error 2^-11), sums in FP32.  The
 *                  ADC distance then errs by up to 2^-11 sum_m |2 term3_m| --
 *                  outside the 1e-5 FP32 tolerance.  Needed for M > 64
 *                  (FP32 tables of M <= 64 fill at most 64 KiB of LDS).
 *                  Entries must satisfy |2 term3| < 65504.
 *   lists_per_group  probed lists of one query scanned by one workgroup:
 *                  0 (default) chosen from the launch size: as many
 *                  lists per workgroup as keep 1024 or more workgroups
 *                  (512 or more for short lists of k or R >= 512; all of
 *                  a query's lists from about 1024 / 512 queries on),
 *                  -1 all of a query's lists (the per-query fused scan of
 *                  Section 5.3), or a count 1..1024.
 * Results do not depend on lists_per_group (candidates are keyed by
 * (distance, id)).  MK_ERR_UNSUPPORTED for another precision.
 */
mk_status mk_ivfpq_set_scan_options(mk_ivfpq* index, mk_precision lut_precision,
                                    int32_t lists_per_group);

/* d, nlist and M of an index (e.g. one created by mk_ivfpq_load); any
 * output pointer may be NULL. */
mk_status mk_ivfpq_shape(const mk_ivfpq* index, int32_t* d, int32_t* nlist, int32_t* M);

/*
 * Upper bound on the device workspace (bytes) that one search of nq queries
 * allocates: mk_ivfpq_search (R = 0), mk_ivfpq_search_rerank (R > 0) or
 * mk_ivfpq_search_learned (nprobe = cap; not counting the network's hidden
 * activations, two rows of its hidden width per query).  Used for admission
 * control and to size the serving loop's workspaces.
 */
mk_status mk_ivfpq_search_workspace_bytes(const mk_ivfpq* index, int64_t nq, int32_t k,
                                          int32_t nprobe, int32_t R, size_t* bytes);

/* ------------------------------------------------------------------------
 * Serving loop (continuous batching; not part of the paper).  Requests of
 * host query rows are queued and packed in arrival order into batches of at
 * most max_batch rows whose search workspace stays within workspace_budget
 * bytes (the first request of a batch is always admitted); nstreams
 * batches are in flight at once, each on its own HIP stream with pinned
 * staging buffers, so transfers and kernels of consecutive batches overlap.
 * Each stream also holds a device workspace of
 * mk_ivfpq_search_workspace_bytes for max_batch rows (at most
 * workspace_budget when that is set) plus a quarter and 64 MiB, allocated at
 * creation, from which its batches' scratch is carved (scratch that does not
 * fit, or all of it when the device has no room for the workspace, is
 * allocated per search as usual).
 * A request's results equal those of searching it alone.
 * ------------------------------------------------------------------------ */

typedef struct mk_server mk_server;

typedef struct {
    int32_t k;                /* neighbours per query */
    int32_t nprobe;           /* probe count when net is NULL */
    int32_t R;                /* > 0: exact re-rank depth (needs xb) */
    int32_t max_batch;        /* rows per batch (and per request) */
    int32_t nstreams;         /* batches in flight, 1 .. 8 */
    int32_t cap;              /* learned probe count: largest tau */
    float delta;              /* learned probe count: offset */
    const mk_mlp* net;        /* non-NULL: learned probe count */
    const float* xb;          /* device database rows for the re-rank */
    int64_t nb;
    int64_t workspace_budget; /* device bytes per batch; 0: no limit */
} mk_server_config;

/* Start the loop's threads on the current device; the index (and net, xb)
 * must outlive the server. */
mk_status mk_server_create(mk_ivfpq* index, const mk_server_config* cfg, mk_server** out);

/*
 * Queue nq query rows xq [nq, d] (host) with result buffers D [nq, k],
 * I [nq, k] (host); all three stay owned by the caller and must stay valid
 * until mk_server_wait returns for the ticket.  1 <= nq <= max_batch.
 */
mk_status mk_server_submit(mk_server* server, const float* xq, int64_t nq, float* D,
                           int64_t* I, uint64_t* ticket);

/* Block until the request completes; latency_s (may be NULL) receives the
 * time from submission to completion.  Each ticket is collected once. */
mk_status mk_server_wait(mk_server* server, uint64_t ticket, double* latency_s);

/* Batches launched and rows searched so far (either may be NULL). */
mk_status mk_server_stats(mk_server* server, int64_t* batches, int64_t* rows);

/* Finish every queued request, stop the threads, free the buffers. */
void mk_server_destroy(mk_server* server);

/*
 * Debug check of the candidate pools of the fused exact search (queues of 256
 * entries and more, Section 4.2's selection replaced by an unsorted pool cut
 * back by radix selection): the number of candidates, over every search on
 * the current device since the library was loaded, that a full pool had to
 * drop.  Pools are cut before they can fill, so the count is 0 unless the
 * selection is broken.  Synchronises the device.
 */
mk_status mk_debug_pool_drops(int64_t* count);

/* ------------------------------------------------------------------------
 * Kernel timing.  While enabled, every launch of the library's main kernels
 * is bracketed by a pair of HIP events recorded on the launch stream, so the
 * measured time is that kernel's own execution on the device.
 * ------------------------------------------------------------------------ */

/* on != 0 starts recording (and clears earlier records); 0 stops. */
mk_status mk_profile_enable(int32_t on);

/*
 * Total device time in milliseconds and number of launches recorded for the
 * kernel called `name` (e.g. "knn_tile_select", "kselect_pass1",
 * "ivf_scan"); waits for the recorded events.  Unknown names give 0 and 0.
 */
mk_status mk_profile_read(const char* name, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* MI_KNN_H */
