// Two-pass sparsified K-means (Alg. "Sparsified K-means, 2-pass"): after the
// one-pass run, one more pass over the original rows X re-assigns every row to
// the nearest one-pass center mu_hat (in the original domain) and recomputes
// each center as the mean of the rows of its one-pass cluster c_hat (a cluster
// with no rows keeps its one-pass center).
//
// Three launches:
//   prep    FP32 copy of mu_hat (FP32 plans) and the largest |center| entry,
//           the scale of the near-tie bound
//   assign  sixteen lanes per row: lanes over coordinates, clusters in
//           windows of 16 with per-lane partial distances, then sums across
//           the sixteen lanes (centers in LDS when they fit); a row whose two
//           best distances are closer than the rounding bound is decided again
//           in FP64 with every lane summing one cluster's distance in ascending
//           coordinate order (the oracle's order, ties to the lowest index)
//   sums    workgroup = (row range, block of columns): each thread owns a column
//           and keeps one FP64 sum per cluster in LDS, adding the range's rows
//           in ascending order; per-range partial sums and counts
//   update  fixed-order FP64 sum of the range partials, division by the count
// Rows are read twice (assign, sums): the second read replaces FP64 atomics.
// Rows whose one-pass cluster lies outside [0, K) take no part in the centers.
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

constexpr int kK2Window = 16;          // clusters per assignment window
constexpr int kK2SumLds = 131072;      // LDS bytes of the per-column cluster sums (the K counts come on top)
constexpr int kK2AssignThreads = 256;  // sixteen rows at a time per workgroup
constexpr int kK2CenterLds = 65536;    // centers in LDS up to this size (else read from memory)

template <typename T>
struct K2Center;  // center element type of the assignment
template <>
struct K2Center<float> {
    using type = float;
};
template <>
struct K2Center<double> {
    using type = double;
};

// FP32 centers (float plans) and the largest |mu_hat| entry (float bits), by
// one workgroup (the result is written, not accumulated: nothing to clear).
__global__ __launch_bounds__(1024) void k_km2_prep(const double* __restrict__ mu_hat, int64_t KP,
                                                   float* __restrict__ ct, uint32_t* __restrict__ cmax)
{
    __shared__ uint32_t red[1024];
    uint32_t mx = 0u;
    for (int64_t e = threadIdx.x; e < KP; e += 1024) {
        const double v = mu_hat[e];
        if (ct) ct[e] = (float)v;
        mx = max(mx, __float_as_uint(fabsf((float)v)));
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *cmax = red[0];
}

template <typename T>
__device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Nearest one-pass center of each row: sixteen lanes per row (four rows per
// wave), each lane over every sixteenth coordinate, clusters in windows of 16
// with per-lane partial distances summed across the sixteen lanes (xor
// butterflies, every lane gets the totals).  With LDS set, the centers sit in
// LDS (the four rows of a wave read the same words: broadcasts).
template <typename T, bool LDS>
__global__ __launch_bounds__(kK2AssignThreads) void k_km2_assign(const T* __restrict__ X, int64_t n, int64_t ldx,
                                                                 int p, int K,
                                                                 const typename K2Center<T>::type* __restrict__ ct,
                                                                 const double* __restrict__ mu_hat,
                                                                 const uint32_t* __restrict__ cmax_bits,
                                                                 int32_t* __restrict__ c_out)
{
    using C = typename K2Center<T>::type;
    extern __shared__ __align__(16) unsigned char k2_smem[];
    const C* cs = ct;
    if constexpr (LDS) {
        C* l = reinterpret_cast<C*>(k2_smem);
        for (int64_t e = threadIdx.x; e < (int64_t)K * p; e += kK2AssignThreads) l[e] = ct[e];
        __syncthreads();
        cs = l;
    }
    const int sl = threadIdx.x & 15;
    constexpr int kRows = kK2AssignThreads / 16;
    const int64_t nr = (int64_t)gridDim.x * kRows;
    const T cmax = (T)__uint_as_float(*cmax_bits);
    // unit roundoff of the distance arithmetic
    const T u = sizeof(T) == 4 ? (T)5.9604645e-8 : (T)1.1102230246251565e-16;
    for (int64_t i = (int64_t)blockIdx.x * kRows + (threadIdx.x >> 4); i < n; i += nr) {
        const T* x = X + i * ldx;
        T best = (T)INFINITY, second = (T)INFINITY, sx = 0;
        int bestk = 0;
        for (int kc = 0; kc < K; kc += kK2Window) {
            T d[kK2Window];
#pragma unroll
            for (int q = 0; q < kK2Window; ++q) d[q] = 0;
            // 256 coordinates of the row at a time: the lane's sixteen loads
            // are issued together, then used
            for (int j0 = 0; j0 < p; j0 += 256) {
                T xb[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int j = j0 + sl + 16 * u;
                    xb[u] = j < p ? x[j] : (T)0;
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int j = j0 + sl + 16 * u;
                    if (j < p) {
                        const T v = xb[u];
                        if (kc == 0) sx = fma(v, v, sx);
#pragma unroll
                        for (int q = 0; q < kK2Window; ++q) {
                            if (kc + q < K) {
                                const T diff = v - (T)cs[(int64_t)(kc + q) * p + j];
                                d[q] = fma(diff, diff, d[q]);
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < kK2Window; ++q) {
                if (kc + q < K) {
                    T dq = d[q];
#pragma unroll
                    for (int off = 8; off > 0; off >>= 1) dq += __shfl_xor(dq, off, 16);
                    if (dq < best) {
                        second = best;
                        best = dq;
                        bestk = kc + q;
                    } else if (dq < second) {
                        second = dq;
                    }
                }
            }
        }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) sx += __shfl_xor(sx, off, 16);
        bool flag = false;
        if (K > 1) {
            // |d - d_exact| <= u (8 (sum x^2 + p max|mu|^2) + 1.01 p d) per
            // candidate (any summation order: every term passes through at
            // most p additions); two candidates, factor 2 of slack
            const T pf = (T)p;
            const T bound = (T)2 * u * ((T)16 * (sx + pf * cmax * cmax) + (T)1.01 * pf * (best + second));
            flag = !(second - best > bound);
        }
        if (flag) {
            // FP64, one cluster per lane of the row, ascending coordinates (the
            // oracle's sums), ties to the lowest index
            double bd = INFINITY;
            int bk = 0x7fffffff;
            for (int k = sl; k < K; k += 16) {
                const double* mu = mu_hat + (int64_t)k * p;
                double dd = 0.0;
                for (int j = 0; j < p; ++j) {
                    const double diff = (double)x[j] - mu[j];
                    dd = fma(diff, diff, dd);
                }
                if (dd < bd) {  // k ascends within a lane: ties keep the lower k
                    bd = dd;
                    bk = k;
                }
            }
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) {
                const double od = __shfl_xor(bd, off, 16);
                const int ok = __shfl_xor(bk, off, 16);
                if (od < bd || (od == bd && ok < bk)) {
                    bd = od;
                    bk = ok;
                }
            }
            bestk = bk;
        }
        if (sl == 0) c_out[i] = bestk;
    }
}

// Per-range sums of the rows of each one-pass cluster, one column per thread.
template <typename T>
__global__ void k_km2_sums(const T* __restrict__ X, int64_t n, int64_t ldx, int p, int K,
                           const int32_t* __restrict__ c_hat, int64_t rows_per, int cols,
                           double* __restrict__ psum, uint32_t* __restrict__ pcnt)
{
    extern __shared__ __align__(16) double ksum[];  // [K][cols], then K row counts
    uint32_t* kcnt = reinterpret_cast<uint32_t*>(ksum + K * cols);
    const int t = threadIdx.x;
    const int64_t r = blockIdx.x;
    const int j = blockIdx.y * cols + t;
    const bool counter = blockIdx.y == 0 && t == 0;  // counts the range's rows per cluster
    for (int e = t; e < K * cols; e += blockDim.x) ksum[e] = 0.0;
    for (int e = t; e < K; e += blockDim.x) kcnt[e] = 0u;
    __syncthreads();
    const int64_t i0 = r * rows_per;
    const int64_t i1 = i0 + rows_per < n ? i0 + rows_per : n;
    const bool live = j < p;
    // eight rows' loads in flight; each thread adds its column in row order
    int64_t i = i0;
    for (; i + 8 <= i1; i += 8) {
        T v[8];
        int k[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            k[u] = c_hat[i + u];
            v[u] = live ? X[(i + u) * ldx + j] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if ((unsigned)k[u] < (unsigned)K) {  // rows outside [0, K) take no part
                ksum[k[u] * cols + t] += (double)v[u];
                if (counter) kcnt[k[u]] += 1u;
            }
        }
    }
    for (; i < i1; ++i) {
        const int k = c_hat[i];
        if ((unsigned)k < (unsigned)K) {
            ksum[k * cols + t] += live ? (double)X[i * ldx + j] : 0.0;
            if (counter) kcnt[k] += 1u;
        }
    }
    __syncthreads();
    if (live)
        for (int k = 0; k < K; ++k) psum[(r * K + k) * (int64_t)p + j] = ksum[k * cols + t];
    if (counter)
        for (int k = 0; k < K; ++k) pcnt[r * K + k] = kcnt[k];
}

// Centers: fixed-order FP64 sum over the row ranges, divided by the count.
__global__ __launch_bounds__(256) void k_km2_update(const double* __restrict__ psum,
                                                    const uint32_t* __restrict__ pcnt, int64_t nranges, int K, int p,
                                                    const double* __restrict__ mu_hat, double* __restrict__ mu_out)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)K * p) return;
    const int k = (int)(e / p);
    double s = 0.0;
    uint64_t c = 0;
#pragma unroll 8
    for (int64_t r = 0; r < nranges; ++r) {
        s += psum[r * (int64_t)K * p + e];
        c += pcnt[r * K + k];
    }
    mu_out[e] = c > 0 ? s / (double)c : mu_hat[e];
}

struct Km2Plan {
    int cols, ncb;
    int64_t rows_per, nranges;
    size_t ct_bytes, cmax_bytes, psum_bytes, pcnt_bytes;
};

static Km2Plan km2_plan(int prec, int p, int64_t n, int K, const DeviceInfo& dev)
{
    Km2Plan k;
    int cols = 256;
    while (cols > 16 && (size_t)cols * K * 8 > (size_t)kK2SumLds) cols >>= 1;
    if (cols > p) cols = p < 16 ? 16 : p;
    k.cols = cols;
    k.ncb = (p + cols - 1) / cols;
    const int64_t want = (int64_t)dev.cus * 8;  // workgroups in flight
    int64_t nr = (want + k.ncb - 1) / k.ncb;
    const int64_t maxr = (n + 255) / 256;  // at least 256 rows per range
    if (nr > maxr) nr = maxr;
    if (nr < 1) nr = 1;
    k.rows_per = (n + nr - 1) / nr;
    if (k.rows_per < 1) k.rows_per = 1;
    k.nranges = (n + k.rows_per - 1) / k.rows_per;
    if (k.nranges < 1) k.nranges = 1;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    k.ct_bytes = prec == 0 ? 0 : up((size_t)K * p * 4);
    k.cmax_bytes = 256;
    k.psum_bytes = up((size_t)k.nranges * K * p * 8);
    k.pcnt_bytes = up((size_t)k.nranges * K * 4);
    return k;
}

size_t kmeans2_workspace(int prec, int p, int64_t n, int K, const DeviceInfo& dev)
{
    const Km2Plan k = km2_plan(prec, p, n, K, dev);
    return k.ct_bytes + k.cmax_bytes + k.psum_bytes + k.pcnt_bytes;
}

bool kmeans2_supported(int K)
{
    return (size_t)16 * K * 8 <= (size_t)kK2SumLds;  // at least 16 columns of cluster sums in LDS
}

hipError_t launch_kmeans_2pass(int prec, int p, const void* X, int64_t n, int64_t ldx, int K, const int32_t* c_hat,
                               const double* mu_hat, double* mu_out, int32_t* c_out, void* ws, size_t ws_bytes,
                               const DeviceInfo& dev, hipStream_t s)
{
    (void)ws_bytes;
    const Km2Plan k = km2_plan(prec, p, n, K, dev);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    float* ct = prec == 0 ? nullptr : reinterpret_cast<float*>(w);
    w += k.ct_bytes;
    uint32_t* cmax = reinterpret_cast<uint32_t*>(w);
    w += k.cmax_bytes;
    double* psum = reinterpret_cast<double*>(w);
    w += k.psum_bytes;
    uint32_t* pcnt = reinterpret_cast<uint32_t*>(w);
    const int64_t KP = (int64_t)K * p;
    {
        ProfScope ps_("km2_prep", s);
        hipLaunchKernelGGL(k_km2_prep, dim3(1), dim3(1024), 0, s, mu_hat, KP, ct, cmax);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        ProfScope ps_("km2_assign", s);
        int64_t grid = (n + 15) / 16;
        if (grid > (int64_t)dev.cus * 8) grid = (int64_t)dev.cus * 8;
        const size_t ce = prec == 0 ? 8 : 4;
        const size_t clds = (size_t)KP * ce;
        const bool lds = clds <= (size_t)kK2CenterLds;
        static bool attr = false;
        if (!attr) {
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_km2_assign<double, true>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, kK2CenterLds);
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_km2_assign<float, true>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, kK2CenterLds);
            attr = true;
        }
        if (prec == 0) {
            const double* Xd = reinterpret_cast<const double*>(X);
            if (lds)
                hipLaunchKernelGGL((k_km2_assign<double, true>), dim3((unsigned)grid), dim3(kK2AssignThreads), clds,
                                   s, Xd, n, ldx, p, K, mu_hat, mu_hat, cmax, c_out);
            else
                hipLaunchKernelGGL((k_km2_assign<double, false>), dim3((unsigned)grid), dim3(kK2AssignThreads), 0, s,
                                   Xd, n, ldx, p, K, mu_hat, mu_hat, cmax, c_out);
        } else {
            const float* Xf = reinterpret_cast<const float*>(X);
            if (lds)
                hipLaunchKernelGGL((k_km2_assign<float, true>), dim3((unsigned)grid), dim3(kK2AssignThreads), clds, s,
                                   Xf, n, ldx, p, K, ct, mu_hat, cmax, c_out);
            else
                hipLaunchKernelGGL((k_km2_assign<float, false>), dim3((unsigned)grid), dim3(kK2AssignThreads), 0, s,
                                   Xf, n, ldx, p, K, ct, mu_hat, cmax, c_out);
        }
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        ProfScope ps_("km2_sums", s);
        const size_t lds = (size_t)K * k.cols * 8 + (size_t)K * 4;
        static bool attr = false;
        if (!attr) {
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_km2_sums<double>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, kK2SumLds + 1024 * 4);
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_km2_sums<float>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, kK2SumLds + 1024 * 4);
            attr = true;
        }
        const dim3 grid((unsigned)k.nranges, (unsigned)k.ncb);
        if (prec == 0)
            hipLaunchKernelGGL(k_km2_sums<double>, grid, dim3(k.cols), lds, s, reinterpret_cast<const double*>(X),
                               n, ldx, p, K, c_hat, k.rows_per, k.cols, psum, pcnt);
        else
            hipLaunchKernelGGL(k_km2_sums<float>, grid, dim3(k.cols), lds, s, reinterpret_cast<const float*>(X), n,
                               ldx, p, K, c_hat, k.rows_per, k.cols, psum, pcnt);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        ProfScope ps_("km2_update", s);
        hipLaunchKernelGGL(k_km2_update, dim3((unsigned)((KP + 255) / 256)), dim3(256), 0, s, psum, pcnt, k.nranges,
                           K, p, mu_hat, mu_out);
    }
    return hipGetLastError();
}

}  // namespace pds
