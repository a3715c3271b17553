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

/* Operation selector for pds_workspace_size. */
typedef enum { PDS_OP_COMPRESS = 0, PDS_OP_COVARIANCE = 1, PDS_OP_KMEANS = 2 } pds_op;

typedef struct pds_plan_s* pds_plan;

/* Creates a plan for samples of dimension p keeping m coordinates each
 * (compression factor gamma = m / p, Sec. I setup), with random seed `seed`
 * and precision `prec`.  Host-only (no device work); *out receives the plan.
 * Errors: PDS_E_ARG (out NULL or prec unknown), PDS_E_UNSUPPORTED (p),
 * PDS_E_M (m). */
pds_status pds_plan_create(pds_plan* out, int64_t p, int64_t m, uint64_t seed, int32_t prec);

/* Frees a plan (NULL is accepted). */
pds_status pds_plan_destroy(pds_plan plan);

/* Host copy of the plan's random sign diagonal D of the ROS y = H D x
 * (Sec. III, eq. ROS): D_host receives p entries, each +1 or -1.  D is drawn
 * once per seed and shared by all samples (Alg. 1 applies one H D to X).
 * D_j = +1 iff bit (j mod 64) of 64-bit word ((j div 64) mod 4) of the
 * Philox4x64-10 block with key (seed, 0) and counter (j div 256, 0, 1, 0) is
 * zero.  Host-only. */
pds_status pds_signs(pds_plan plan, int8_t* D_host);

/* Device workspace bytes that `op` needs for n samples (and K clusters for
 * PDS_OP_KMEANS); PDS_OP_COVARIANCE also reports what its accumulator needs
 * through pds_covariance_acc_size.  Host-only. */
pds_status pds_workspace_size(pds_plan plan, int32_t op, int64_t n, int32_t K, size_t* bytes);

/* Bytes of the covariance accumulator `acc` (p x p doubles). */
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
 *   ws    may be NULL (compress needs no workspace; ws_bytes ignored).
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
 * n may be 0 (finalize only).  ws: device, >= pds_workspace_size(COVARIANCE, n).
 * Errors: PDS_E_M (m < 2: the rescaling divides by m - 1), PDS_E_ARG (null
 * pointers, n < 0, finalize with n_total < 1), PDS_E_WORKSPACE. */
pds_status pds_covariance(pds_plan plan, const void* vals, const uint16_t* idx, int64_t n, double* acc,
                          int32_t finalize, int64_t n_total, double* C_out, void* ws, size_t ws_bytes,
                          void* stream);

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

/* Unmixing of centers (eq. mu-mu'; Alg. 1, last step): centers_out[k] =
 * (H D)^T centers_pre[k] = D H centers_pre[k] (H is symmetric), FP64.
 * centers_pre / centers_out: device, K x p doubles (may not alias).
 * Errors: PDS_E_ARG (null pointers, K < 1). */
pds_status pds_unmix(pds_plan plan, const double* centers_pre, int32_t K, double* centers_out, void* stream);

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
