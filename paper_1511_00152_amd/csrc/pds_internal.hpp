// Internal launch interface between the C ABI (api.hip) and the kernels.
// Arguments are validated by the caller; launchers only size grids and launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pds {

struct DeviceInfo {
    int cus;       // compute units
    int device;    // ordinal
};

hipError_t device_info(DeviceInfo& info);

// Optional per-kernel event timing (pds_profile_enable).  Construct right
// before a launch and destroy right after it, on the launch stream.
class ProfScope {
public:
    ProfScope(const char* name, hipStream_t s);
    ~ProfScope();

private:
    int slot_;
    hipStream_t s_;
};

// ---- compression --------------------------------------------------------
// Kept coordinates (ascending) of samples i0 .. i0+n-1 into idx (n x m).
hipError_t launch_sample_indices(uint64_t seed, int p, int m, int64_t n, uint64_t i0, uint16_t* idx,
                                 const DeviceInfo& dev, hipStream_t s);

// y = H D x per row, then vals[r][t] = y[idx[r][t]].  prec: 0 f64, 1 f32,
// 2 split-bf16 (matrix-core transform).  ws: scratch for very large p.
hipError_t launch_compress(int prec, uint64_t seed, int p, int m, const void* X, int64_t n, int64_t ldx,
                           const uint16_t* idx, void* vals, void* ws, size_t ws_bytes, const DeviceInfo& dev,
                           hipStream_t s);
size_t compress_workspace(int prec, int p, int64_t n, const DeviceInfo& dev);
// FP32 values at p in [512, 2048] with aligned rows: sampler and transform in
// one launch (writes idx and vals; no launch_sample_indices before it)
bool compress_fused_ok(int prec, int p, const void* X, int64_t ldx);
hipError_t launch_compress_fused(uint64_t seed, int p, int m, const float* X, int64_t n, int64_t ldx, uint64_t i0,
                                 float* vals, uint16_t* idx, const DeviceInfo& dev, hipStream_t s);
// split-BF16 matrix-core transform (p = 4096)
bool kron_transform_ok(int p, const void* X, int64_t ldx);
hipError_t launch_compress_kron(uint64_t seed, int m, const float* X, int64_t n, int64_t ldx, const uint16_t* idx,
                                float* vals, const DeviceInfo& dev, hipStream_t s);

// DCT plans: y = C D x (orthonormal DCT-II) for any p <= 8192; ws holds the
// FFT twiddle tables (p = 2^a 3^b 5^c 7^d <= 2048) or the p x p FP64 table
// of the dense form (dct_compress_workspace bytes)
size_t dct_compress_workspace(int p);
bool dct_fast_ok(int p);
hipError_t launch_dct_compress(int prec, uint64_t seed, int p, int m, const void* X, int64_t n, int64_t ldx,
                               const uint16_t* idx, void* vals, void* ws, const DeviceInfo& dev, hipStream_t s);
hipError_t launch_dct_unmix(uint64_t seed, int p, const double* cpre, int K, double* cout, hipStream_t s);

// ---- covariance -----------------------------------------------------------
// algo: 0 = the faster form by the cost model, 1 = dense tiles, 2 = sparse
size_t covariance_workspace(int prec, int p, int m, int64_t n, const DeviceInfo& dev, int algo);
bool covariance_is_sparse(int prec, int p, int m, int64_t n, const DeviceInfo& dev, int algo);
hipError_t launch_covariance_accumulate(int prec, int p, int m, const void* vals, const uint16_t* idx, int64_t n,
                                        double* acc, void* ws, size_t ws_bytes, const DeviceInfo& dev,
                                        hipStream_t s, int algo);
// C (p x p) from the accumulated Gram acc (row stride lda >= p)
hipError_t launch_covariance_finalize(int prec, int p, int lda, int m, int64_t n_total, const double* acc, double* C,
                                      hipStream_t s);

// ---- sample mean -------------------------------------------------------------
size_t mean_workspace(int p, int m, int64_t n, const DeviceInfo& dev);
hipError_t launch_mean(int prec, int p, int m, const void* vals, const uint16_t* idx, int64_t n, double* acc,
                       int finalize, int64_t n_total, double* mean_out, void* ws, const DeviceInfo& dev,
                       hipStream_t s);

hipError_t launch_pad_rows(int x_f64, const void* X, int64_t n, int64_t p_data, int64_t ldx, void* Xp, int64_t p_pad,
                           const DeviceInfo& dev, hipStream_t s);

// ---- PCA quality -------------------------------------------------------------
size_t explained_workspace();
int explained_max_k();
hipError_t launch_explained(const double* U, int k, const void* X, int x_f64, int64_t n, int p, int64_t ldx,
                            double* out2, void* ws, hipStream_t s);

// ---- K-means++ seeding ------------------------------------------------------
size_t kmeanspp_workspace(int64_t n);
hipError_t launch_kmeanspp(int prec, int p, int m, const void* vals, const uint16_t* idx, int64_t n, int K,
                           uint64_t seed, uint64_t rep, double* centers, int64_t* chosen, void* ws, hipStream_t s);
hipError_t launch_keep_best(int r, int T, const double* obj, const double* centers, int64_t kp, const int32_t* assign,
                            int64_t n, double* centers_best, int32_t* assign_best, int32_t* best, const DeviceInfo& dev,
                            hipStream_t s);

// ---- K-means ----------------------------------------------------------------
size_t kmeans_workspace(int prec, int p, int m, int64_t n, int K, const DeviceInfo& dev);
// reuse_scale: the workspace holds the per-workgroup scales that an earlier
// round recorded for these same vals / idx / n / K (rounds of one call)
hipError_t launch_kmeans_step(int prec, int p, int m, const void* vals, const uint16_t* idx, int64_t n, int K,
                              const double* cin, double* cout, int32_t* assign, double* objective, void* ws,
                              size_t ws_bytes, const DeviceInfo& dev, hipStream_t s, bool reuse_scale = false);

// ---- two-pass K-means -------------------------------------------------------
size_t kmeans2_workspace(int prec, int p, int64_t n, int K, const DeviceInfo& dev);
bool kmeans2_supported(int K);
hipError_t launch_kmeans_2pass(int prec, int p, const void* X, int64_t n, int64_t ldx, int K, const int32_t* c_hat,
                               const double* mu_hat, double* mu_out, int32_t* c_out, void* ws, size_t ws_bytes,
                               const DeviceInfo& dev, hipStream_t s);

// ---- unmix ------------------------------------------------------------------
hipError_t launch_unmix(uint64_t seed, int p, const double* cpre, int K, double* cout, hipStream_t s);

// ---- learned m-selector -----------------------------------------------------
// per-row (sum x^2, sum x^4, max x^2) in FP64, out is n x 3
hipError_t launch_row_moments(const float* X, int64_t n, int p, int64_t ldx, double* out, const DeviceInfo& dev,
                              hipStream_t s);
// out2 = (sum (A-B)^2, sum B^2); part holds frob_workspace() bytes
size_t frob_workspace();
hipError_t launch_frob_diff(const double* A, const double* B, int64_t len, double* out2, double* part, hipStream_t s);
hipError_t launch_msel_label(const double* mom, int64_t n, int p, const double* F2, double t, int32_t* m_out,
                             hipStream_t s);
hipError_t launch_msel_features(const double* mr, const double* my, int s_rows, int64_t n, int p, const double* F2s,
                                double t, float* feats, hipStream_t s);
hipError_t launch_zero_f64(double* a, int64_t len, const DeviceInfo& dev, hipStream_t s);

// MLP 32 -> 64 -> 64 -> 1 (packed FP32 parameters, mlp_param_count() of them)
int mlp_param_count();
hipError_t launch_mlp_forward(const float* P, const float* feats, const float* mu, const float* sd, int B, float* acts,
                              float* out, hipStream_t s);
hipError_t launch_mlp_backward(const float* P, const float* acts, const float* pred, const float* target, int B,
                               float tau, float* sig, float* lossb, float* grad, float* loss, hipStream_t s);
hipError_t launch_adam(float* P, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s);
hipError_t launch_pack_bf16(const float* P, int n, unsigned short* Pb, hipStream_t s);
hipError_t launch_mlp_predict_bf16(const unsigned short* Pb, const float* feats, const float* mu, const float* sd,
                                   int B, float gmin, float gmax, float fallback, float* gamma, hipStream_t s);

}  // namespace pds
