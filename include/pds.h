/*
 * pds.h -- preconditioned data sparsification on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the one-pass compression of Pourkamali-Anaraki & Becker,
 * "Preconditioned Data Sparsification for Big Data with Applications to PCA
 * and K-means" (arXiv 1511.00152), and of the two estimators computed on the
 * compressed data: the rescaled, diagonal-corrected covariance (Sec. V) and
 * sparsified Lloyd K-means (Sec. VI, Alg. 1).
 *
 * Layout conventions (all calls):
 *   - X is row-major n x p, one sample per row (the paper stores samples as
 *     columns of a p x n matrix; this is the same data transposed in memory so
 *     that each sample is contiguous).  Indices are 0-based.
 *   - Compressed data is "ELL without padding": vals is n x m (row-major) and
 *     idx is n x m uint16, the kept coordinates of each sample in ascending
 *     order.  Every sample keeps exactly m coordinates, so no row pointers.
 *   - Device pointers are HIP device (or managed) memory; "host" pointers are
 *     ordinary CPU memory.  The caller owns every buffer; the library never
 *     allocates device memory.  Hot calls (compress, covariance, kmeans_step,
 *     unmix) only enqueue kernels on `stream` (a hipStream_t passed as void*;
 *     NULL = the legacy default stream) and return without synchronising.
 *
 * Error behaviour: every call validates its arguments on the host first and
 * returns a negative pds_status without launching anything (and without
 * writing any output) when they are invalid.  PDS_E_HIP reports a launch
 * failure; the text of the last error of the calling thread is available from
 * pds_last_error().  Device faults surface at the caller's next
 * synchronisation.  n == 0 is a valid no-op for the hot calls.
 */
#ifndef PDS_H_
#define PDS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PDS_OK = 0,
    PDS_E_ARG = -1,         /* null pointer, negative size, bad leading dimension, bad K, ... */
    PDS_E_UNSUPPORTED = -2, /* p not a power of two, p < 2 or p > 65536 */
    PDS_E_M = -3,           /* m < 1 or m > p; m < 2 for the covariance */
    PDS_E_WORKSPACE = -4,   /* workspace smaller than pds_workspace_size() */
    PDS_E_HIP = -5          /* a HIP runtime call failed (see pds_last_error) */
} pds_status;

/* Precision of a plan.
 *   PDS_F64        X and vals are double; transform, Gram and K-means in FP64.
 *   PDS_F32        X and vals are float; transform in FP32 on the vector ALUs,
 *                  Gram on FP32 matrix cores (FP64 reduction across sample
 *                  ranges), K-means distances in FP32 with an FP64 recheck of
 *                  near ties, centers in FP64.
 *   PDS_SPLIT_BF16 X and vals are float; the transform is applied as
 *                  Kronecker-factored Hadamard blocks H_a (x) H_b on BF16
 *                  matrix cores with each FP32 operand split into three BF16
 *                  parts (hi, mid, lo) and FP32 accumulation; the Gram runs on
 *                  BF16 matrix cores with each value split into hi + lo and the
 *                  three products hi*hi, hi*lo, lo*hi accumulated in FP32;
 *                  diagonal correction, centroid division and all reductions
 *                  across sample ranges stay in FP64.  K-means as PDS_F32.   */
typedef enum { PDS_F64 = 0, PDS_F32 = 1, PDS_SPLIT_BF16 = 2 } pds_prec;

/* How pds_covariance accumulates G = sum_i w_i w_i^T (Sec. V, the definition
 * of C_emp_hat) for FP32 and split plans.
 *   PDS_GRAM_DENSE  the precision's matrix-core form above: dense output
 *                   tiles over chunks of samples, p^2 / 2 multiply-adds per
 *                   sample (x 3 products for split plans), of which only the
 *                   m^2 / 2 between kept entries are non-zero.
 *   PDS_GRAM_SPARSE only the m^2 / 2 products between each sample's kept
 *                   entries: exact FP32 products of the FP32 values, summed
 *                   as 32-bit fixed point over ranges of at most 2048 samples
 *                   (scale from the range's largest |value|, every sum exact
 *                   and independent of the order of addition) and then in
 *                   FP64; deterministic.  A non-finite value makes the
 *                   affected tiles NaN.  Not available for FP64 plans.
 *   PDS_GRAM_AUTO   (the default) the form a cost model of both on MI355X
 *                   predicts to be faster for (p, m, n): the sparse form at
 *                   small m / p, the dense form as m approaches p.        */
typedef enum { PDS_GRAM_AUTO = 0, PDS_GRAM_DENSE = 1, PDS_GRAM_SPARSE = 2 } pds_gram_algo;

/* Operation selector for pds_workspace_size. */
typedef enum {
    PDS_OP_COMPRESS = 0,
    PDS_OP_COVARIANCE = 1,
    PDS_OP_KMEANS = 2,
    PDS_OP_KMEANS2 = 3,
    PDS_OP_MEAN = 4,
    PDS_OP_KMEANSPP = 5,
    PDS_OP_KMEANS_BEST = 6,
    PDS_OP_KMEANS_RUN = 7
} pds_op;

typedef struct pds_plan_s* pds_plan;

/* The plan's preconditioning transform (Sec. III): the normalized Hadamard
 * matrix (eq. ROS; p a power of two) or the orthonormal DCT-II, which Sec. III
 * allows as another fast orthonormal transform with entries O(1/sqrt(p))
 * (Thm. 1 with eta = 1/2) and Sec. VII uses for p = 784. */
typedef enum { PDS_TRANSFORM_HADAMARD = 0, PDS_TRANSFORM_DCT = 1 } pds_transform;
#define PDS_DCT_MAX_P 8192

/* Creates a plan for samples of dimension p keeping m coordinates each
 * (compression factor gamma = m / p, Sec. I setup), with random seed `seed`
 * and precision `prec`.  Host-only (no device work); *out receives the plan.
 * Errors: PDS_E_ARG (out NULL or prec unknown), PDS_E_UNSUPPORTED (p),
 * PDS_E_M (m). */
pds_status pds_plan_create(pds_plan* out, int64_t p, int64_t m, uint64_t seed, int32_t prec);

/* Creates a plan whose preconditioner is the orthonormal DCT-II in place of
 * H (pds_transform): y_i = C D x_i with
 *     C[j][k] = s_j cos(pi (2k + 1) j / (2p)),  s_0 = sqrt(1/p), s_j = sqrt(2/p),
 * for any p in [2, PDS_DCT_MAX_P] (no power-of-two restriction), the same
 * signs D (pds_signs) and the same kept sets as a Hadamard plan of this
 * (p, m, seed).  Every plan call takes it: pds_compress transforms with C in
 * FP64, rounded once to the plan's value type -- for p = 2^a 3^b 5^c 7^d <=
 * 2048 in O(p log p) (Makhoul's reordering of the DCT-II into one complex DFT,
 * two samples per mixed-radix FFT; its workspace holds 2p complex twiddles and
 * rotations), for every other p as a dense product of p^2 multiply-adds per
 * sample (its workspace holds the p x p table) -- pds_unmix applies
 * D C^T, and the covariance accumulates its Gram over the next power of two
 * pg >= p (pds_covariance_acc_size is pg x pg doubles; kept indices are < p,
 * so the extra rows and columns stay zero) and finalizes the p x p C_n.  The
 * m-selector calls take Hadamard plans only.  Host-only.
 * Errors: PDS_E_ARG (out NULL or prec unknown), PDS_E_UNSUPPORTED (p),
 * PDS_E_M (m). */
pds_status pds_plan_create_dct(pds_plan* out, int64_t p, int64_t m, uint64_t seed, int32_t prec);

/* The plan's pds_transform into *transform.  Host-only.
 * Errors: PDS_E_ARG (NULL plan or transform). */
pds_status pds_plan_transform(pds_plan plan, int32_t* transform);

/* Frees a plan (NULL is accepted). */
pds_status pds_plan_destroy(pds_plan plan);

/* Host copy of the plan's random sign diagonal D of the ROS y = H D x
 * (Sec. III, eq. ROS): D_host receives p entries, each +1 or -1.  D is drawn
 * once per seed and shared by all samples (Alg. 1 applies one H D to X).
 * D_j = +1 iff bit (j mod 64) of 64-bit word ((j div 64) mod 4) of the
 * Philox4x64-10 block with key (seed, 0) and counter (j div 256, 0, 1, 0) is
 * zero.  Host-only. */
pds_status pds_signs(pds_plan plan, int8_t* D_host);

/* Sets the plan's Gram form (pds_gram_algo; the plan starts with
 * PDS_GRAM_AUTO).  Host-only.  Errors: PDS_E_ARG (unknown value),
 * PDS_E_UNSUPPORTED (PDS_GRAM_SPARSE on an FP64 plan). */
pds_status pds_plan_set_gram(pds_plan plan, int32_t algo);

/* The form pds_covariance will run for a call with n samples
 * (PDS_GRAM_DENSE or PDS_GRAM_SPARSE) into *algo.  Host-only.
 * Errors: PDS_E_ARG (NULL algo, n < 0). */
pds_status pds_plan_gram(pds_plan plan, int64_t n, int32_t* algo);

/* Device workspace bytes that `op` needs for n samples (and K clusters for
 * PDS_OP_KMEANS and PDS_OP_KMEANS2); PDS_OP_COVARIANCE also reports what its accumulator needs
 * through pds_covariance_acc_size.  Host-only. */
pds_status pds_workspace_size(pds_plan plan, int32_t op, int64_t n, int32_t K, size_t* bytes);

/* Bytes of the covariance accumulator `acc` (p x p doubles; pg x pg for DCT
 * plans, pg the next power of two >= p). */
pds_status pds_covariance_acc_size(pds_plan plan, size_t* bytes);

/* One-pass compression (Alg. 1, first loop; Sec. I setup; Sec. III eq. ROS):
 * for each row r of X (sample i = i0 + r)
 *     y_i = H D x_i            H = normalized Sylvester Walsh-Hadamard matrix,
 *                              H[j][k] = (-1)^popcount(j & k) / sqrt(p)
 *     keep m of the p entries of y_i chosen uniformly without replacement:
 *     idx[r][0..m-1] = the kept coordinates, ascending; vals[r][t] = y_i[idx[r][t]].
 * The kept set of sample i depends only on (seed, i, p, m): Floyd's algorithm
 * with draws by Lemire's method from the 32-bit words (low half, then high
 * half, of each 64-bit word) of Philox4x64-10 blocks with key (seed, 0) and
 * counter (b, i, 0, 0), b = 0, 1, ...  So chunked calls (i0 > 0) reproduce a
 * one-shot call bit for bit.
 *   X     device, n x p row-major with leading dimension ldx >= p (elements),
 *         double for PDS_F64, float otherwise.
 *   vals  device, n x m, same element type as X.
 *   idx   device, n x m uint16.
 *   ws    device, >= pds_workspace_size(COMPRESS, n) bytes; NULL when that
 *         size is 0 (Hadamard plans whose row buffer fits in LDS, i.e. every
 *         p up to 8192 in FP32 and 4096 in FP64).  Larger Hadamard p need a
 *         row buffer per workgroup; DCT plans the FFT form's tables or the
 *         dense form's p x p table.
 * Errors: PDS_E_ARG (null pointers with n > 0, n < 0, ldx < p). */
pds_status pds_compress(pds_plan plan, const void* X, int64_t n, int64_t ldx, uint64_t i0, void* vals,
                        uint16_t* idx, void* ws, size_t ws_bytes, void* stream);

/* Covariance estimator of Sec. V on compressed data, streamed:
 *   acc += sum over the n given samples of w_i w_i^T   (w_i = the zero-filled
 *          compressed sample), accumulated in FP64.  Only the upper triangle
 *          (by tiles) of acc is maintained; acc must be zeroed by the caller
 *          before the first batch and is caller-owned (p x p doubles, device).
 *   if finalize != 0, C_out (device, p x p doubles, full symmetric) receives
 *          C_n = C_emp_hat - (p-m)/(p-1) diag(C_emp_hat),
 *          C_emp_hat = p(p-1)/(m(m-1)) * acc / n_total,
 *          i.e. C_n[j][j] = p/(m n_total) acc[j][j] and
 *               C_n[j][k] = p(p-1)/(m(m-1) n_total) acc[j][k] for j != k,
 *          unbiased for C_emp = (1/n_total) sum_i y_i y_i^T (Thm. "covariance").
 *          C_n is in the preconditioned domain (eigenvalues are the same as in
 *          the original domain; eigenvectors map back by (H D)^T).
 * n may be 0 (finalize only).  ws: device, >= pds_workspace_size(COVARIANCE, n);
 * for FP32 and split plans it holds the batch's kept entries re-packed by
 * 32-sample chunk and 128-coordinate block (6 bytes per kept entry) and FP32
 * partial tiles per sample range, so it grows linearly with n: large inputs
 * can be streamed in batches into the same acc.
 * Errors: PDS_E_M (m < 2: the rescaling divides by m - 1), PDS_E_ARG (null
 * pointers, n < 0, finalize with n_total < 1), PDS_E_WORKSPACE. */
pds_status pds_covariance(pds_plan plan, const void* vals, const uint16_t* idx, int64_t n, double* acc,
                          int32_t finalize, int64_t n_total, double* C_out, void* ws, size_t ws_bytes,
                          void* stream);

/* Sample-mean estimator of Sec. IV (Thm. "sampleMean") on compressed data,
 * streamed:
 *   acc += sum over the n given samples of w_i (w_i = the zero-filled
 *          compressed sample), per coordinate, in FP64.  acc: device, p
 *          doubles, caller-owned, zeroed by the caller before the first batch.
 *   if finalize != 0, mean_out (device, p doubles) receives
 *          (p / (m n_total)) * acc, unbiased for the mean of the y_i over all
 *          n_total samples.  It is in the preconditioned domain: pds_unmix
 *          with K = 1 maps it back to the mean of the x_i.
 * vals / idx as written by pds_compress (n x m; FP64 values for PDS_F64
 * plans, FP32 otherwise; indices < p).  Sums inside a work-group are added in
 * no fixed order, so the last bits may differ from run to run.
 * n may be 0 (finalize only).  ws: device, >= pds_workspace_size(MEAN, n)
 * (p doubles per sample range, about 4 ranges per compute unit).
 * Errors: PDS_E_ARG (null pointers, n < 0, finalize with n_total < 1,
 * mean_out aliasing acc), PDS_E_WORKSPACE. */
pds_status pds_sample_mean(pds_plan plan, const void* vals, const uint16_t* idx, int64_t n, double* acc,
                           int32_t finalize, int64_t n_total, double* mean_out, void* ws, size_t ws_bytes,
                           void* stream);

/* Rows of a dimension that is not a power of two, widened for a plan: Xp[r][j]
 * = X[r][j] for j < p_data and 0 for p_data <= j < p_pad.  The Hadamard
 * transform of Sec. III needs p a power of two (the paper used a DCT for
 * p = 784); compressing the zero-padded rows with a plan of p = p_pad keeps
 * norms, and the padded coordinates of means, covariances and centers mapped
 * back by pds_unmix estimate zero (drop them).
 *   X: device, n x p_data rows, leading dimension ldx >= p_data; Xp: device,
 *   n x p_pad rows, contiguous; double when x_prec = PDS_F64, float when
 *   PDS_F32.  Must not alias.
 * Errors: PDS_E_ARG (null pointers, n < 0, p_data < 1, p_pad < p_data,
 * ldx < p_data, x_prec, aliasing). */
pds_status pds_pad_rows(const void* X, int32_t x_prec, int64_t n, int64_t p_data, int64_t ldx, void* Xp, int64_t p_pad,
                        void* stream);

/* Fraction of explained variance of k principal components (Sec. II,
 * comparison with column sampling; PCA on the estimate of Sec. V), FP64:
 *   out2[0] = sum_i sum_j (x_i . U[j])^2 = ||X U^T||_F^2,
 *   out2[1] = sum_i ||x_i||^2 = ||X||_F^2,
 * so the fraction is out2[0] / out2[1] when the rows of U are orthonormal.
 * Summed in a fixed order (run-to-run identical).
 *   U:  device, k x p doubles, row j = component j in the original domain
 *       (e.g. eigenvectors of C_n mapped back by pds_unmix), 1 <= k <= 32.
 *   X:  device, n x p rows with leading dimension ldx >= p; double when
 *       x_prec = PDS_F64, float when x_prec = PDS_F32.
 *   out2: device, 2 doubles.  ws: device, >= PDS_EXPLAINED_WS_BYTES bytes.
 * Errors: PDS_E_ARG (null pointers, n < 1, p < 1, k out of range, ldx < p,
 * x_prec), PDS_E_WORKSPACE. */
#define PDS_EXPLAINED_WS_BYTES 16384
pds_status pds_explained_variance(const double* U, int32_t k, const void* X, int32_t x_prec, int64_t n, int64_t p,
                                  int64_t ldx, double* out2, void* ws, size_t ws_bytes, void* stream);

/* K-means++ seeding on compressed data (Alg. 1 seeds with K-means++; D^2
 * sampling of Arthur & Vassilvitskii with the sparsified distance of Sec. VI):
 *   center 0 = sample floor(u_0 n) (at most n - 1);
 *   center k = the first sample i whose running sum of D^2 (ascending i)
 *              exceeds u_k sum_j D^2, else sample n - 1, where D^2(i) is the
 *              smallest sum over sample i's kept coordinates l of
 *              (vals_i,l - center[l])^2 over the centers chosen so far;
 *   centers[k] = the chosen sample's zero-filled compressed vector.
 * u_k = (w_k >> 11) 2^-53 with w_k word (k mod 4) of the Philox4x64-10 block
 * with key (plan seed, 0) and counter (k div 4, replicate, 2, 0): each
 * replicate >= 0 is an independent starting point.  Distances are the
 * FP64 sequential sums (fused multiply-adds in ascending l); the running sums
 * are formed per block of samples, so a draw within rounding of a boundary
 * between two samples may take the neighbour a sequential scan would take.
 *   vals / idx: as written by pds_compress (n x m, indices < p).
 *   centers: device, K x p doubles.  chosen: device, K int64 (or NULL).
 *   ws: device, >= pds_workspace_size(KMEANSPP, n).
 * Errors: PDS_E_ARG (null pointers, n < 1, K < 1 or K > 1024,
 * replicate < 0), PDS_E_WORKSPACE. */
pds_status pds_kmeanspp(pds_plan plan, const void* vals, const uint16_t* idx, int64_t n, int32_t K, int32_t replicate,
                        double* centers, int64_t* chosen, void* ws, size_t ws_bytes, void* stream);

/* Sparsified K-means from R starting points on one compression (Alg. 1; the
 * experiments of Sec. VII keep the best of several random starts): for
 * r = 0 .. R-1, K-means++ seeding with replicate r (pds_kmeanspp), then T
 * rounds of pds_kmeans_step; objectives[r*T + t] = round t's objective of
 * start r.  The kept start is the one whose last round reports the smallest
 * objective (the earliest on ties): centers_out (device, K x p doubles,
 * preconditioned domain) and assign_out (device, n int32) receive its final
 * centers and last assignments, best (device, 1 int32) its index.  Every
 * decision is taken on the device; nothing returns to the host in between.
 * ws: device, >= pds_workspace_size(KMEANS_BEST, n, K).
 * Errors: PDS_E_ARG (null pointers, n < 1, K out of [1, 1024], T < 1, R out of
 * [1, 1024]), PDS_E_WORKSPACE. */
pds_status pds_kmeans_best(pds_plan plan, const void* vals, const uint16_t* idx, int64_t n, int32_t K, int32_t T,
                           int32_t R, double* centers_out, int32_t* assign_out, double* objectives, int32_t* best,
                           void* ws, size_t ws_bytes, void* stream);

/* T iterations of sparsified K-means (Alg. 1, the loop; Sec. VI) from
 * centers_in: the same rounds as T successive pds_kmeans_step calls, each
 * round reading the previous round's centers, with results equal to theirs
 * bit for bit.  After the first round the rounds reuse the per-workgroup
 * fixed-point scales the first one took from the compressed values (they are
 * the same values), which saves one read of the values per round.
 *   centers_out: device, K x p doubles, the last round's centers (must not
 *   alias centers_in); assign: device, n int32, the last round's assignments;
 *   objectives: device, T doubles, round t's objective (eq. CK_means) with the
 *   centers entering that round.  ws: device, >= pds_workspace_size(KMEANS_RUN,
 *   n, K) (the step's workspace and one center buffer).
 * Errors: PDS_E_ARG (null pointers with n > 0, n < 0, K out of [1, 1024],
 * T < 1, aliasing), PDS_E_WORKSPACE. */
pds_status pds_kmeans_run(pds_plan plan, const void* vals, const uint16_t* idx, int64_t n, int32_t K, int32_t T,
                          const double* centers_in, double* centers_out, int32_t* assign, double* objectives, void* ws,
                          size_t ws_bytes, void* stream);

/* One iteration of sparsified K-means (Sec. VI; Alg. 1, loop body) on
 * compressed data, centers in the preconditioned domain:
 *   step 1 (eq. assignments): assign[i] = argmin_k sum_{l in idx_i}
 *          (vals_i,l - centers_in[k][l])^2, ties to the lowest k; the sum runs
 *          over the sample's own kept coordinates only.
 *   step 2 (eq. mu_update_two): centers_out[k][l] = mean of vals_i,l over the
 *          samples i assigned to k that kept coordinate l; where that count is
 *          zero the coordinate cannot be estimated and keeps centers_in[k][l].
 *   objective (device, 1 double) = sum_i distance(i, assign[i]) (eq. CK_means).
 *   centers_in / centers_out: device, K x p doubles (must not alias).
 *   assign: device, n int32.   ws: device, >= pds_workspace_size(KMEANS, n, K).
 * FP32 plans compute distances in FP32 and recompute every sample whose best
 * and second-best distances are closer than a rounding bound in FP64 with the
 * same summation order as an FP64 plan, so assignments equal the FP64 argmin.
 * Errors: PDS_E_ARG (null pointers with n > 0, n < 0, K < 1 or K > 1024),
 * PDS_E_WORKSPACE. */
pds_status pds_kmeans_step(pds_plan plan, const void* vals, const uint16_t* idx, int64_t n, int32_t K,
                           const double* centers_in, double* centers_out, int32_t* assign, double* objective,
                           void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * K-means iteration as pds_kmeans_step, same kernels and results, with its
 * workspace taken from a scratch array the library holds in device memory
 * (PDS_NOALLOC_SCRATCH_BYTES per GPU, reserved when the library is loaded and
 * kept until the process ends) instead of a caller's buffer.  The call
 * allocates nothing.  Every call on one GPU shares that GPU's array: calls
 * that may overlap on one GPU (two streams, two threads) race and must be
 * ordered by the caller.  Arguments as for pds_kmeans_step without ws.
 * Errors: as pds_kmeans_step; PDS_E_WORKSPACE when the workspace
 * pds_workspace_size(KMEANS, n, K) would exceed PDS_NOALLOC_SCRATCH_BYTES
 * (64 MiB covers, e.g., n = 2^20, p = 1024, K = 10 in FP32). */
#define PDS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
pds_status pds_kmeans_step_noalloc(pds_plan plan, const void* vals, const uint16_t* idx, int64_t n, int32_t K,
                                   const double* centers_in, double* centers_out, int32_t* assign,
                                   double* objective, void* stream);

/* Unmixing of centers (eq. mu-mu'; Alg. 1, last step): centers_out[k] =
 * (H D)^T centers_pre[k] = D H centers_pre[k] (H is symmetric), FP64; for
 * DCT plans (C D)^T centers_pre[k] = D C^T centers_pre[k].
 * centers_pre / centers_out: device, K x p doubles (may not alias).
 * Errors: PDS_E_ARG (null pointers, K < 1). */
pds_status pds_unmix(pds_plan plan, const double* centers_pre, int32_t K, double* centers_out, void* stream);

/* Second pass of two-pass sparsified K-means (Alg. "Sparsified K-means,
 * 2-pass"), one more pass over the original rows after the one-pass run:
 *   c_out[i]  = argmin_k sum_j (X[i][j] - mu_hat[k][j])^2 over all p
 *               coordinates, ties to the lowest k (FP32 plans: FP32 distances,
 *               rows closer to a tie than a rounding bound decided in FP64 in
 *               ascending coordinate order, so the result is the FP64 argmin);
 *   mu_out[k] = mean of the rows X[i] with c_hat[i] == k; a cluster with no
 *               rows keeps mu_hat[k].  Rows with c_hat outside [0, K) count
 *               for no center.
 * X: device, n x p row-major with leading dimension ldx >= p, FP64 for FP64
 * plans, FP32 otherwise (the original, not preconditioned, data).
 * c_hat: device, n int32, the one-pass assignments.  mu_hat: device, K x p
 * doubles, the one-pass centers in the original domain (pds_unmix output).
 * mu_out: device, K x p doubles (must not alias mu_hat).  c_out: device, n
 * int32.  ws: device, >= pds_workspace_size(KMEANS2, n, K).
 * Errors: PDS_E_ARG (null pointers with n > 0, n < 0, ldx < p, K < 1 or
 * K > 1024, aliasing), PDS_E_WORKSPACE. */
pds_status pds_kmeans_2pass(pds_plan plan, const void* X, int64_t n, int64_t ldx, int32_t K, const int32_t* c_hat,
                            const double* mu_hat, double* mu_out, int32_t* c_out, void* ws, size_t ws_bytes,
                            void* stream);

/* ---------------------------------------------------------------------------
 * Learned m-selector.  Not part of the paper's method: a small model that
 * chooses m for a data block so that the covariance estimator of Sec. V meets
 * a relative Frobenius error target, trained on labels the method itself
 * defines.  All calls below are asynchronous on `stream`, validate on the host
 * first and return PDS_E_ARG on null pointers or out-of-range sizes.
 * ------------------------------------------------------------------------- */

/* Per-row moments (FP64): out[3r] = sum_j X[r][j]^2, out[3r+1] = sum_j
 * X[r][j]^4, out[3r+2] = max_j X[r][j]^2.  X: device float, n x p, leading
 * dimension ldx >= p; out: device, n x 3 doubles.  p >= 1. */
pds_status pds_row_moments(const float* X, int64_t n, int64_t p, int64_t ldx, double* out, void* stream);

/* Frobenius distance, FP64 with a fixed summation order: out2[0] =
 * sum_e (A[e] - B[e])^2, out2[1] = sum_e B[e]^2 over len >= 1 doubles.
 * A, B, out2: device.  ws: device, >= PDS_FROB_WS_BYTES bytes.  A may equal B. */
#define PDS_FROB_WS_BYTES 4096
pds_status pds_frob_diff(const double* A, const double* B, int64_t len, double* out2, void* ws, size_t ws_bytes,
                         void* stream);

/* Device workspace bytes for pds_msel_label on n rows or pds_msel_features
 * with nsub = n rows.  The plan must keep every coordinate (m = p) and be
 * PDS_F32: with m = p the compression is the exact transform y = H D x and the
 * estimator of Sec. V is exactly C_emp (Sec. V setup).  Host-only. */
pds_status pds_msel_workspace_size(pds_plan plan, int64_t n, size_t* bytes);

/* Training label of a block X (device float, n x p, ldx >= p, n >= 2): the
 * smallest m in [2, p] whose expected squared relative Frobenius error
 *   E||C_n - C_emp||_F^2 / ||C_emp||_F^2
 *     = [(1/q2 - 1) sum_i (||y_i||^4 - sum_j y_ij^4) + (1/q1 - 1) sum_ij y_ij^4]
 *       / (n^2 ||C_emp||_F^2),      q1 = m/p, q2 = m(m-1)/(p(p-1)),
 * is at most target^2, with y_i = H D x_i under the plan's D.  The inclusion
 * probabilities are those of Lemma B and Thm. B; the expectation is over the
 * sampling only, the data and D being fixed.  m_out: device, one int32.
 * C_out: NULL, or device p x p doubles receiving C_emp.  A block with
 * C_emp = 0 gets m = 2.  target > 0.  Errors: PDS_E_M (plan m != p),
 * PDS_E_ARG, PDS_E_WORKSPACE. */
pds_status pds_msel_label(pds_plan plan, const float* X, int64_t n, int64_t ldx, double target, int32_t* m_out,
                          double* C_out, void* ws, size_t ws_bytes, void* stream);

/* The 32 features of a block of n rows computed from its first nsub rows
 * (2 <= nsub <= min(n, 1024)), written to feats (device, 32 floats):
 *   0       log mean ||x||^2
 *   1..8    quantiles of ||x_i||^2 / mean ||x||^2
 *   9..16   quantiles of log(p max_j x_ij^2 / ||x_i||^2)   (coherence, Sec. III)
 *   17..24  quantiles of log(p max_j y_ij^2 / ||y_i||^2)   (after H D)
 *   25      log mean_i p sum_j y_ij^4 / ||y_i||^4
 *   26      log mean_i p sum_j x_ij^4 / ||x_i||^4
 *   27      log(U / (mean ||y||^2)^2), U = (nsub^2 ||C_sub||_F^2 - sum_i ||y_i||^4)
 *           / (nsub (nsub - 1)), C_sub = (1/nsub) sum_i y_i y_i^T
 *   28      log(||C_sub||_F^2 / (mean ||y||^2)^2)
 *   29, 30  log n, log p
 *   31      log(m'/p), m' = the label rule of pds_msel_label evaluated with the
 *           subset's moments scaled to n rows and ||C_emp||_F^2 predicted as
 *           (mean ||y||^4 + (n - 1) U) / n
 * Quantile levels are 0.05 0.15 0.3 0.5 0.7 0.85 0.95 1; level q takes sorted
 * entry floor(q (nsub - 1)).  A zero row counts as ratio 1 (log 0).
 * Errors: PDS_E_M (plan m != p), PDS_E_ARG, PDS_E_WORKSPACE. */
pds_status pds_msel_features(pds_plan plan, const float* X, int64_t n, int64_t ldx, int64_t nsub, double target,
                             float* feats, void* ws, size_t ws_bytes, void* stream);

/* The selector's network: 32 -> 64 -> 64 -> 1, ReLU hidden layers, inputs
 * standardized as (f - mu) / sd, output log(gamma).  Parameters are packed
 * FP32: W1[64][32], b1[64], W2[64][64], b2[64], W3[64], b3 (row-major,
 * W[out][in]); pds_mlp_param_count() of them. */
int32_t pds_mlp_param_count(void);

/* Forward pass in FP32 for B >= 1 rows of feats (device, B x 32): pred
 * (device, B floats) = network output; acts (device, B x 160 floats) keeps
 * the standardized input and both hidden layers for pds_mlp_backward.
 * params, mu, sd: device (mu, sd: 32 floats each). */
pds_status pds_mlp_forward(const float* params, const float* feats, const float* mu, const float* sd, int64_t B,
                           float* acts, float* pred, void* stream);

/* Gradient of the expectile loss L = (1/B) sum_b |tau - [r_b < 0]| r_b^2,
 * r_b = target_b - pred_b, with respect to the parameters (device,
 * pds_mlp_param_count() floats, summed over the batch in a fixed order) and
 * the loss itself (device, 1 float).  acts and pred come from pds_mlp_forward
 * with the same params.  ws: device, >= B x 130 floats.  0 < tau < 1. */
pds_status pds_mlp_backward(const float* params, const float* acts, const float* pred, const float* target, int64_t B,
                            float tau, float* ws, size_t ws_bytes, float* grad, float* loss, void* stream);

/* One Adam update (Kingma & Ba, ICLR 2015) of every parameter, FP32:
 * m1 = b1 m1 + (1 - b1) g, m2 = b2 m2 + (1 - b2) g^2,
 * params -= lr (m1 / (1 - b1^step)) / (sqrt(m2 / (1 - b2^step)) + eps).
 * step >= 1 counts updates; m1, m2 start at zero.  All device. */
pds_status pds_mlp_adam(float* params, const float* grad, float* m1, float* m2, int32_t step, float lr, float beta1,
                        float beta2, float eps, void* stream);

/* BF16 copy of the parameters (round to nearest even), device -> device. */
pds_status pds_mlp_pack_bf16(const float* params, uint16_t* params_bf16, void* stream);

/* Inference with BF16 parameters: standardized inputs and the first hidden
 * layer rounded to BF16, FP32 accumulation; gamma[b] = clamp(exp(output),
 * gamma_min, gamma_max), or gamma_fallback (then clamped) when a feature or
 * the output is not finite.  feats: device B x 32; gamma: device B floats.
 * 0 < gamma_min <= gamma_max. */
pds_status pds_msel_predict(const uint16_t* params_bf16, const float* feats, const float* mu, const float* sd,
                            int64_t B, float gamma_min, float gamma_max, float gamma_fallback, float* gamma,
                            void* stream);

/* ---------------------------------------------------------------------------
 * Batched form: many independent data sets, each with its own p, m, K and
 * seed, compressed in one persistent launch and clustered by T rounds of
 * sparsified K-means (Sec. VI; Alg. 1) replayed from one captured HIP graph.
 * Results equal what the single-set calls produce for each set: the same kept
 * sets (a set's kept sets and D depend on (seed, sample, p, m) only), values
 * within FP32 rounding, assignments the FP64 argmin.  FP32 data only.
 * ------------------------------------------------------------------------- */
typedef struct {
    const float* X;       /* device, n x p row-major, leading dimension ldx >= p; for p >= 256
                             X and ldx * 4 must be multiples of 16 bytes */
    int64_t n;            /* samples, >= 0 */
    int64_t ldx;
    int32_t p;            /* power of two in [128, 2048] */
    int32_t m;            /* kept coordinates, 1 <= m <= p */
    int32_t K;            /* clusters, 1 <= K <= 1024 */
    int32_t reserved;     /* must be 0 */
    uint64_t seed;        /* as pds_plan_create's seed */
    float* vals;          /* device, n x m: compressed values (output) */
    uint16_t* idx;        /* device, n x m: kept coordinates, ascending (output) */
    double* centers;      /* device, K x p: initial centers in the preconditioned domain on entry to
                             pds_batch_kmeans, the centers after T rounds on return */
    double* centers_alt;  /* device, K x p: scratch */
    int32_t* assign;      /* device, n: assignments of the last round (output) */
    double* objective;    /* device, T doubles: J' of each round (output) */
} pds_batch_desc;

typedef struct pds_batch_s* pds_batch;

/* Creates a batch over count >= 1 descriptors (host array, copied) with T >= 0
 * K-means rounds.  Host-only.  Errors: PDS_E_ARG (a descriptor's pointers,
 * sizes or alignment), PDS_E_UNSUPPORTED (p), PDS_E_M (m). */
pds_status pds_batch_create(pds_batch* out, const pds_batch_desc* descs, int32_t count, int32_t T);
pds_status pds_batch_destroy(pds_batch b);

/* Device workspace bytes the batch needs (descriptor and work tables,
 * transposed FP32 centers, per-chunk partial sums).  Host-only. */
pds_status pds_batch_workspace_size(pds_batch b, size_t* bytes);

/* Binds a workspace (device, >= pds_batch_workspace_size bytes, owned by the
 * caller and kept alive and unmodified while the batch is used): uploads the
 * tables on `stream` and captures the T K-means rounds into a graph.
 * Errors: PDS_E_WORKSPACE, PDS_E_HIP. */
pds_status pds_batch_bind(pds_batch b, void* ws, size_t ws_bytes, void* stream);

/* Compression of every set (Alg. 1, first loop; as pds_compress with i0 = 0)
 * in one persistent launch. */
pds_status pds_batch_compress(pds_batch b, void* stream);

/* Seeds each set's centers with its first K compressed samples, zero-filled
 * (center k = w_k for k < n, zero beyond).  A simple seeding, not K-means++. */
pds_status pds_batch_init_centers(pds_batch b, void* stream);

/* T rounds of sparsified K-means on every set (as T calls of pds_kmeans_step
 * alternating between centers and centers_alt, the last writing centers):
 * one graph launch.  Needs pds_batch_compress first. */
pds_status pds_batch_kmeans(pds_batch b, void* stream);

/* Times candidate launch shapes (samples per compression group, samples per
 * assignment item and per accumulation chunk) on the bound data and keeps the
 * fastest; re-captures the graph.  Runs the compression and one K-means round
 * per candidate, so it overwrites vals and idx (with the same values),
 * centers_alt, assign and objective[0]; call it after pds_batch_compress and
 * with initial centers in place.  Synchronizes `stream`. */
pds_status pds_batch_autotune(pds_batch b, void* stream);

/* Text summary: sets, samples, work items, chosen shapes, kernel launches per
 * pds_batch_kmeans (writes a NUL-terminated line into buf, len bytes). */
pds_status pds_batch_info(pds_batch b, char* buf, size_t len);

/* Measurement hooks (not part of the method).  pds_profile_enable(1) clears
 * any previous records and starts bracketing every kernel the library launches
 * with a pair of HIP events on the launch stream; pds_profile_enable(0) stops
 * recording.  pds_profile_report waits for the recorded events, writes one
 * text line per kernel name, "name launches total_ms min_ms max_ms\n", into
 * buf (host, len bytes, NUL-terminated, truncated if short; *needed receives
 * the full length + 1 when non-NULL) and clears the records.  Recording costs
 * two event records per launch and allocates host-side event objects, so leave
 * it off outside measurement.  Errors: PDS_E_ARG (buf NULL with len > 0),
 * PDS_E_HIP. */
pds_status pds_profile_enable(int32_t on);
pds_status pds_profile_report(char* buf, size_t len, size_t* needed);

/* Text of the last error reported to the calling thread ("" if none). */
const char* pds_last_error(void);

/* Library version string. */
const char* pds_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PDS_H_ */
