// Learned m-selector support: per-row moments, Frobenius distances between
// p x p matrices, the training label and the 32 block features.
//
// The label is the smallest m whose EXPECTED squared Frobenius error of the
// covariance estimator, relative to the exact empirical covariance, is at most
// t^2.  The expectation is over the method's sampling (Lemma B and Theorem B:
// a coordinate is kept with probability q1 = m/p, a pair with probability
// q2 = m(m-1)/(p(p-1)); samples draw independently).  Each entry of the
// estimator is an unbiased sum of independent per-sample terms, so
//   E||C_n - C_emp||_F^2 = n^-2 sum_i [ (1/q2 - 1) sum_{j!=k} y_ij^2 y_ik^2
//                                      + (1/q1 - 1) sum_j y_ij^4 ]
//                        = n^-2 [ (1/q2 - 1) A + (1/q1 - 1) B ],
//   A = sum_i (||y_i||^4 - sum_j y_ij^4),  B = sum_i sum_j y_ij^4,
// a decreasing function of m that is zero at m = p.
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

constexpr int kFeat = 32;
constexpr int kFrobBlocks = 256;

// (1/q2 - 1) A + (1/q1 - 1) B, divided by n^2 F2
__device__ inline double msel_expected_e2(int m, int p, double n, double A, double B, double F2)
{
    const double P = p, M = m;
    const double r1 = (P - M) / M;
    const double r2 = (P * (P - 1.0) - M * (M - 1.0)) / (M * (M - 1.0));
    return (r2 * A + r1 * B) / (n * n * F2);
}

// smallest m in [2, p] with e2(m) <= t^2 (e2 is non-increasing, e2(p) = 0)
__device__ inline int msel_smallest_m(int p, double n, double A, double B, double F2, double t)
{
    if (!(F2 > 0.0)) return 2;
    const double t2 = t * t;
    int lo = 2, hi = p;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (msel_expected_e2(mid, p, n, A, B, F2) <= t2)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// fixed-order tree sum over a workgroup of NT threads; every thread returns the total
template <int NT>
__device__ inline double block_sum(double v, double* red)
{
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// Row moments: out[i] = (sum_j x_ij^2, sum_j x_ij^4, max_j x_ij^2) in FP64.
// One wave per row; lanes stride over the row, then a butterfly reduction.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_row_moments(const float* __restrict__ X, int64_t n, int p, int64_t ldx,
                                                     double* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < n; r += nw) {
        const float* x = X + r * ldx;
        double s2 = 0.0, s4 = 0.0, mx = 0.0;
        for (int j = lane; j < p; j += 64) {
            const double v = (double)x[j];
            const double v2 = v * v;
            s2 += v2;
            s4 = fma(v2, v2, s4);
            mx = fmax(mx, v2);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            s2 += __shfl_xor(s2, o);
            s4 += __shfl_xor(s4, o);
            mx = fmax(mx, __shfl_xor(mx, o));
        }
        if (lane == 0) {
            out[r * 3 + 0] = s2;
            out[r * 3 + 1] = s4;
            out[r * 3 + 2] = mx;
        }
    }
}

// ---------------------------------------------------------------------------
// Frobenius distance: (sum (A-B)^2, sum B^2) over len entries, two stages with
// a fixed summation order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_frob_partial(const double* __restrict__ A, const double* __restrict__ B,
                                                      int64_t len, double* __restrict__ part)
{
    __shared__ double red[256];
    double d2 = 0.0, b2 = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < len; e += (int64_t)kFrobBlocks * 256) {
        const double b = B[e];
        const double d = A[e] - b;
        d2 = fma(d, d, d2);
        b2 = fma(b, b, b2);
    }
    d2 = block_sum<256>(d2, red);
    b2 = block_sum<256>(b2, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 2 + 0] = d2;
        part[blockIdx.x * 2 + 1] = b2;
    }
}

__global__ __launch_bounds__(256) void k_frob_final(const double* __restrict__ part, double* __restrict__ out)
{
    __shared__ double red[256];
    const double d2 = block_sum<256>(part[threadIdx.x * 2 + 0], red);
    const double b2 = block_sum<256>(part[threadIdx.x * 2 + 1], red);
    if (threadIdx.x == 0) {
        out[0] = d2;
        out[1] = b2;
    }
}

// ---------------------------------------------------------------------------
// Label: A and B from the preconditioned rows' moments, F2 = ||C_emp||_F^2.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_msel_label(const double* __restrict__ mom, int64_t n, int p,
                                                    const double* __restrict__ F2p, double t,
                                                    int32_t* __restrict__ m_out)
{
    __shared__ double red[256];
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double s2 = mom[i * 3 + 0], s4 = mom[i * 3 + 1];
        a += fma(s2, s2, -s4);
        b += s4;
    }
    a = block_sum<256>(a, red);
    b = block_sum<256>(b, red);
    if (threadIdx.x == 0) *m_out = msel_smallest_m(p, (double)n, a, b, *F2p, t);
}

// ---------------------------------------------------------------------------
// Features of a block from its first s rows (2 <= s <= 1024): moments of the
// raw rows (mr) and of the preconditioned rows (my), F2s = ||C_sub||_F^2 with
// C_sub = (1/s) sum_i y_i y_i^T.  Layout of the 32 features:
//   0      log mean ||x||^2
//   1..8   quantiles of ||x_i||^2 / mean ||x||^2
//   9..16  quantiles of log(p max_j x_ij^2 / ||x_i||^2)      (raw coherence)
//   17..24 quantiles of log(p max_j y_ij^2 / ||y_i||^2)      (preconditioned)
//   25     log mean_i p sum_j y_ij^4 / ||y_i||^4
//   26     log mean_i p sum_j x_ij^4 / ||x_i||^4
//   27     log(U / (mean ||y||^2)^2), U = (s^2 F2s - sum ||y_i||^4) / (s(s-1)),
//          the unbiased pair statistic of ||E y y^T||_F^2
//   28     log(F2s / (mean ||y||^2)^2)
//   29, 30 log n, log p
//   31     log(m'/p), m' the label rule applied to the subset's plug-in moments
// Quantile levels 0.05 0.15 0.3 0.5 0.7 0.85 0.95 1: sorted entry
// floor(q (s-1)) in integer arithmetic.  A row with zero norm counts as flat
// (ratio 1).
// ---------------------------------------------------------------------------
constexpr int kQuantPerMille[8] = {50, 150, 300, 500, 700, 850, 950, 1000};

__device__ inline void bitonic_sort_1024(double* v)
{
    const int t = threadIdx.x;
    for (int k = 2; k <= 1024; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int o = t ^ j;
            if (o > t) {
                const double a = v[t], b = v[o];
                const bool up = (t & k) == 0;
                if ((a > b) == up) {
                    v[t] = b;
                    v[o] = a;
                }
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(1024) void k_msel_features(const double* __restrict__ mr, const double* __restrict__ my,
                                                        int s, int64_t n, int p, const double* __restrict__ F2s_p,
                                                        double t, float* __restrict__ feats)
{
    __shared__ double red[1024];
    __shared__ double srt[3][1024];
    const int i = threadIdx.x;
    const double P = p;
    double v0 = INFINITY, v1 = INFINITY, v2 = INFINITY;
    double s2r = 0.0, s2y = 0.0, fr = 0.0, fy = 0.0, a = 0.0, b = 0.0, q = 0.0;
    if (i < s) {
        s2r = mr[i * 3 + 0];
        const double s4r = mr[i * 3 + 1], mxr = mr[i * 3 + 2];
        s2y = my[i * 3 + 0];
        const double s4y = my[i * 3 + 1], mxy = my[i * 3 + 2];
        v0 = s2r;
        v1 = (s2r > 0.0) ? log(P * mxr / s2r) : 0.0;
        v2 = (s2y > 0.0) ? log(P * mxy / s2y) : 0.0;
        fr = (s2r > 0.0) ? P * s4r / (s2r * s2r) : 1.0;
        fy = (s2y > 0.0) ? P * s4y / (s2y * s2y) : 1.0;
        a = fma(s2y, s2y, -s4y);
        b = s4y;
        q = s2y * s2y;
    }
    srt[0][i] = v0;
    srt[1][i] = v1;
    srt[2][i] = v2;
    const double S2r = block_sum<1024>(s2r, red);
    const double S2y = block_sum<1024>(s2y, red);
    const double Fr = block_sum<1024>(fr, red);
    const double Fy = block_sum<1024>(fy, red);
    const double Sa = block_sum<1024>(a, red);
    const double Sb = block_sum<1024>(b, red);
    const double Sq = block_sum<1024>(q, red);
    bitonic_sort_1024(srt[0]);
    bitonic_sort_1024(srt[1]);
    bitonic_sort_1024(srt[2]);
    const double ds = s;
    const double mean_r = S2r / ds, mean_y = S2y / ds;
    if (i < 8) {
        const int k = (int)(((int64_t)kQuantPerMille[i] * (s - 1)) / 1000);
        feats[1 + i] = (float)(srt[0][k] / mean_r);
        feats[9 + i] = (float)srt[1][k];
        feats[17 + i] = (float)srt[2][k];
    }
    if (i == 0) {
        const double F2s = *F2s_p;
        const double dn = (double)n;
        const double U = (ds * ds * F2s - Sq) / (ds * (ds - 1.0));
        feats[0] = (float)log(mean_r);
        feats[25] = (float)log(Fy / ds);
        feats[26] = (float)log(Fr / ds);
        feats[27] = (float)log(fmax(U, 1e-300) / (mean_y * mean_y));
        feats[28] = (float)log(F2s / (mean_y * mean_y));
        feats[29] = (float)log(dn);
        feats[30] = (float)log(P);
        // plug-in: E||C_emp||^2 = (E||y||^4 + (n-1) ||E yy^T||^2) / n
        const double F2n = (Sq / ds) / dn + (dn - 1.0) / dn * U;
        const int mp = (F2n > 0.0) ? msel_smallest_m(p, dn, dn * Sa / ds, dn * Sb / ds, F2n, t) : p;
        feats[31] = (float)log((double)mp / P);
    }
}

// zero a double buffer (a fill kernel rather than a memset node)
__global__ __launch_bounds__(256) void k_zero_f64(double* __restrict__ a, int64_t len)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < len; e += (int64_t)gridDim.x * 256) a[e] = 0.0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_row_moments(const float* X, int64_t n, int p, int64_t ldx, double* out, const DeviceInfo& dev,
                              hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t grid = (n + 3) / 4;
    const int64_t cap = (int64_t)dev.cus * 8;
    if (grid > cap) grid = cap;
    ProfScope ps_("row_moments", s);
    hipLaunchKernelGGL(k_row_moments, dim3((unsigned)grid), dim3(256), 0, s, X, n, p, ldx, out);
    return hipGetLastError();
}

size_t frob_workspace() { return (size_t)kFrobBlocks * 2 * sizeof(double); }

hipError_t launch_frob_diff(const double* A, const double* B, int64_t len, double* out2, double* part, hipStream_t s)
{
    ProfScope ps_("frob_diff", s);
    hipLaunchKernelGGL(k_frob_partial, dim3(kFrobBlocks), dim3(256), 0, s, A, B, len, part);
    hipLaunchKernelGGL(k_frob_final, dim3(1), dim3(256), 0, s, part, out2);
    return hipGetLastError();
}

hipError_t launch_msel_label(const double* mom, int64_t n, int p, const double* F2, double t, int32_t* m_out,
                             hipStream_t s)
{
    ProfScope ps_("msel_label", s);
    hipLaunchKernelGGL(k_msel_label, dim3(1), dim3(256), 0, s, mom, n, p, F2, t, m_out);
    return hipGetLastError();
}

hipError_t launch_msel_features(const double* mr, const double* my, int s_rows, int64_t n, int p, const double* F2s,
                                double t, float* feats, hipStream_t s)
{
    ProfScope ps_("msel_features", s);
    hipLaunchKernelGGL(k_msel_features, dim3(1), dim3(1024), 0, s, mr, my, s_rows, n, p, F2s, t, feats);
    return hipGetLastError();
}

hipError_t launch_zero_f64(double* a, int64_t len, const DeviceInfo& dev, hipStream_t s)
{
    if (len <= 0) return hipSuccess;
    int64_t grid = (len + 255) / 256;
    const int64_t cap = (int64_t)dev.cus * 8;
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)grid), dim3(256), 0, s, a, len);
    return hipGetLastError();
}

}  // namespace pds
