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
//   update  fixed-order FP64 sum of the range partials (eight interleaved
//           partial sums added in lane order), division by the count
// Rows are read twice (assign, sums): the second read replaces FP64 atomics.
// For K <= 16 both passes keep the next rows' loads in flight while the
// current ones are used (pipelined assignment; sums in registers).
// Rows whose one-pass cluster lies outside [0, K) take no part in the centers.
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

constexpr int kK2Window = 16;          // clusters per assignment window
constexpr int kK2SumLds = 131072;      // LDS bytes of the per-column cluster sums (the K counts come on top)
constexpr int kK2AssignThreads = 256;  // sixteen rows at a time per workgroup
constexpr int kK2CenterLds = 65536;    // centers in LDS up to this size (else read from memory)
constexpr int kK2Assign16Threads = 512;  // K <= 16: 32 rows per workgroup share one LDS copy of the centers

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

// The same assignment for K <= 16 (one cluster window), software-pipelined,
// 512 threads per workgroup (the LDS copy of the centers serves twice as many
// rows):
// while a lane's sixteen values of one 256-coordinate block are used, the
// next block's loads (or the next row's first block) are already in flight,
// so a row group never waits on memory between blocks.  Same arithmetic and
// order as above.
template <typename T, bool LDS, int NQ>
__global__ __launch_bounds__(kK2Assign16Threads) void k_km2_assign16(const T* __restrict__ X, int64_t n, int64_t ldx,
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
        for (int64_t e = threadIdx.x; e < (int64_t)K * p; e += kK2Assign16Threads) l[e] = ct[e];
        __syncthreads();
        cs = l;
    }
    const int sl = threadIdx.x & 15;
    constexpr int kRows = kK2Assign16Threads / 16;
    const int64_t nr = (int64_t)gridDim.x * kRows;
    const T cmax = (T)__uint_as_float(*cmax_bits);
    const T u = sizeof(T) == 4 ? (T)5.9604645e-8 : (T)1.1102230246251565e-16;
    const int nb = (p + 255) / 256;
    T cur[16], nxt[16];
    auto load = [&](T (&buf)[16], int64_t row, int blk) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int j = blk * 256 + sl + 16 * q;
            buf[q] = (row < n && j < p) ? X[row * ldx + j] : (T)0;
        }
    };
    int64_t i = (int64_t)blockIdx.x * kRows + (threadIdx.x >> 4);
    load(cur, i, 0);
    for (; i < n; i += nr) {
        // NQ >= K cluster slots; slots past K repeat center K - 1 (their
        // distances are computed and dropped), so no multiply-add is predicated
        T d[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) d[q] = 0;
        T sx = 0;
        for (int blk = 0; blk < nb; ++blk) {
            if (blk + 1 < nb)
                load(nxt, i, blk + 1);
            else
                load(nxt, i + nr, 0);
#pragma unroll
            for (int q2 = 0; q2 < 16; ++q2) {
                const int j = blk * 256 + sl + 16 * q2;
                if (j < p) {
                    const T v = cur[q2];
                    sx = fma(v, v, sx);
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        const int qc = q < K ? q : K - 1;
                        const T diff = v - (T)cs[(int64_t)qc * p + j];
                        d[q] = fma(diff, diff, d[q]);
                    }
                }
            }
#pragma unroll
            for (int q2 = 0; q2 < 16; ++q2) cur[q2] = nxt[q2];
        }
        T best = (T)INFINITY, second = (T)INFINITY;
        int bestk = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (q < K) {
                T dq = d[q];
#pragma unroll
                for (int off = 8; off > 0; off >>= 1) dq += __shfl_xor(dq, off, 16);
                if (dq < best) {
                    second = best;
                    best = dq;
                    bestk = q;
                } else if (dq < second) {
                    second = dq;
                }
            }
        }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) sx += __shfl_xor(sx, off, 16);
        bool flag = false;
        if (K > 1) {
            const T pf = (T)p;
            const T bound = (T)2 * u * ((T)16 * (sx + pf * cmax * cmax) + (T)1.01 * pf * (best + second));
            flag = !(second - best > bound);
        }
        if (flag) {
            const T* x = X + i * ldx;
            double bd = INFINITY;
            int bk = 0x7fffffff;
            for (int k = sl; k < K; k += 16) {
                const double* mu = mu_hat + (int64_t)k * p;
                double dd = 0.0;
                // sixteen coordinates' loads issued together, then summed in
                // ascending order (the oracle's)
                int j = 0;
                for (; j + 16 <= p; j += 16) {
                    double xv[16], mv[16];
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        xv[e] = (double)x[j + e];
                        mv[e] = mu[j + e];
                    }
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const double diff = xv[e] - mv[e];
                        dd = fma(diff, diff, dd);
                    }
                }
                for (; j < p; ++j) {
                    const double diff = (double)x[j] - mu[j];
                    dd = fma(diff, diff, dd);
                }
                if (dd < bd) {
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

// Per-range sums with the clusters' FP64 sums in registers (K <= KR <= 16).
// Every lane of the workgroup adds the same row, so the row's cluster is one
// value for the whole wave: a uniform (scalar) branch picks the accumulator
// and each element costs one FP64 add, in the same row order as the LDS form
// below (bit-identical sums).  Sixteen rows' loads are in flight one batch
// ahead.
template <int KR>
__device__ inline void km2_add(double (&acc)[KR], int k, double v)
{
#pragma unroll
    for (int c = 0; c < KR; ++c)
        if (k == c) {
            acc[c] += v;
            return;
        }
}

template <typename T, int KR>
__global__ __launch_bounds__(256) void k_km2_sums_reg(const T* __restrict__ X, int64_t n, int64_t ldx, int p, int K,
                                                      const int32_t* __restrict__ c_hat, int64_t rows_per, int cols,
                                                      double* __restrict__ psum, uint32_t* __restrict__ pcnt)
{
    constexpr int B = 16;
    const int t = threadIdx.x;
    const int64_t r = blockIdx.x;
    const int j = blockIdx.y * cols + t;
    const bool live = j < p;
    const int jj = live ? j : 0;
    const bool counter = blockIdx.y == 0 && t == 0;
    double acc[KR];
    uint32_t cnt[KR];
#pragma unroll
    for (int q = 0; q < KR; ++q) {
        acc[q] = 0.0;
        cnt[q] = 0u;
    }
    const int64_t i0 = r * rows_per;
    const int64_t i1 = i0 + rows_per < n ? i0 + rows_per : n;
    T va[B], vb[B];
    int ka[B], kb[B];
    auto load = [&](int64_t ib, T (&v)[B], int (&k)[B]) {
#pragma unroll
        for (int q = 0; q < B; ++q) {
            const int64_t i = ib + q;
            const bool in = i < i1;
            // one value for the whole wave (scalar register)
            k[q] = __builtin_amdgcn_readfirstlane(in ? c_hat[i] : -1);
            v[q] = (in && live) ? X[i * ldx + jj] : (T)0;
        }
    };
    auto add = [&](const T (&v)[B], const int (&k)[B]) {
#pragma unroll
        for (int q = 0; q < B; ++q) {
            km2_add<KR>(acc, k[q], (double)v[q]);
            if ((unsigned)k[q] < (unsigned)KR) cnt[k[q]] += 1u;
        }
    };
    if (i0 < i1) load(i0, va, ka);
    for (int64_t ib = i0; ib < i1; ib += 2 * B) {
        if (ib + B < i1) load(ib + B, vb, kb);
        add(va, ka);
        if (ib + B >= i1) break;
        if (ib + 2 * B < i1) load(ib + 2 * B, va, ka);
        add(vb, kb);
    }
    if (live)
#pragma unroll
        for (int q = 0; q < KR; ++q)
            if (q < K) psum[(r * K + q) * (int64_t)p + j] = acc[q];
    if (counter)
#pragma unroll
        for (int q = 0; q < KR; ++q)
            if (q < K) pcnt[r * K + q] = cnt[q];
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
// Eight lanes per center entry, lane g summing ranges g, g + 8, g + 16, ... in
// ascending order; the eight partial sums are then added in lane order.
__global__ __launch_bounds__(256) void k_km2_update(const double* __restrict__ psum,
                                                    const uint32_t* __restrict__ pcnt, int64_t nranges, int K, int p,
                                                    const double* __restrict__ mu_hat, double* __restrict__ mu_out)
{
    const int64_t e = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 3;
    const int g = threadIdx.x & 7;
    const bool live = e < (int64_t)K * p;
    const int64_t ee = live ? e : 0;
    const int k = (int)(ee / p);
    double s = 0.0;
    uint64_t c = 0;
#pragma unroll 4
    for (int64_t r = g; r < nranges; r += 8) {
        s += psum[r * (int64_t)K * p + ee];
        c += pcnt[r * K + k];
    }
    // lane-order combination of the eight partials (lanes g = 0..7 of a group)
    double tot = 0.0;
    uint64_t cn = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        tot += __shfl(s, (threadIdx.x & ~7) + q, 64);
        cn += (uint64_t)__shfl((long long)c, (threadIdx.x & ~7) + q, 64);
    }
    if (live && g == 0) mu_out[e] = cn > 0 ? tot / (double)cn : mu_hat[e];
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
        static bool attr = false, attr16 = false;
        if (!attr) {
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_km2_assign<double, true>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, kK2CenterLds);
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_km2_assign<float, true>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, kK2CenterLds);
            attr = true;
        }
        if (!attr16) {
            const void* fs[] = {reinterpret_cast<const void*>(&k_km2_assign16<double, true, 4>),
                                reinterpret_cast<const void*>(&k_km2_assign16<double, true, 8>),
                                reinterpret_cast<const void*>(&k_km2_assign16<double, true, 12>),
                                reinterpret_cast<const void*>(&k_km2_assign16<double, true, 16>),
                                reinterpret_cast<const void*>(&k_km2_assign16<float, true, 4>),
                                reinterpret_cast<const void*>(&k_km2_assign16<float, true, 8>),
                                reinterpret_cast<const void*>(&k_km2_assign16<float, true, 12>),
                                reinterpret_cast<const void*>(&k_km2_assign16<float, true, 16>)};
            for (const void* f : fs) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kK2CenterLds);
            attr16 = true;
        }
        if (K <= kK2Window) {
            const int nq = (K + 3) & ~3;
            int64_t grid16 = (n + kK2Assign16Threads / 16 - 1) / (kK2Assign16Threads / 16);
            if (grid16 > (int64_t)dev.cus * 4) grid16 = (int64_t)dev.cus * 4;
#define PDS_KM2_A16(NQ)                                                                                            \
    if (prec == 0) {                                                                                               \
        const double* Xd = reinterpret_cast<const double*>(X);                                                     \
        if (lds)                                                                                                   \
            hipLaunchKernelGGL((k_km2_assign16<double, true, NQ>), dim3((unsigned)grid16), dim3(kK2Assign16Threads),  \
                               clds, s, Xd, n, ldx, p, K, mu_hat, mu_hat, cmax, c_out);                            \
        else                                                                                                       \
            hipLaunchKernelGGL((k_km2_assign16<double, false, NQ>), dim3((unsigned)grid16), dim3(kK2Assign16Threads), \
                               0, s, Xd, n, ldx, p, K, mu_hat, mu_hat, cmax, c_out);                               \
    } else {                                                                                                       \
        const float* Xf = reinterpret_cast<const float*>(X);                                                       \
        if (lds)                                                                                                   \
            hipLaunchKernelGGL((k_km2_assign16<float, true, NQ>), dim3((unsigned)grid16), dim3(kK2Assign16Threads),   \
                               clds, s, Xf, n, ldx, p, K, ct, mu_hat, cmax, c_out);                                \
        else                                                                                                       \
            hipLaunchKernelGGL((k_km2_assign16<float, false, NQ>), dim3((unsigned)grid16), dim3(kK2Assign16Threads),  \
                               0, s, Xf, n, ldx, p, K, ct, mu_hat, cmax, c_out);                                   \
    }
            if (nq == 4) {
                PDS_KM2_A16(4)
            } else if (nq == 8) {
                PDS_KM2_A16(8)
            } else if (nq == 12) {
                PDS_KM2_A16(12)
            } else {
                PDS_KM2_A16(16)
            }
#undef PDS_KM2_A16
        } else if (prec == 0) {
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
        const double* Xd = reinterpret_cast<const double*>(X);
        const float* Xf = reinterpret_cast<const float*>(X);
#define PDS_KM2_SUMS_REG(KR)                                                                                        \
    if (prec == 0)                                                                                                 \
        hipLaunchKernelGGL((k_km2_sums_reg<double, KR>), grid, dim3(k.cols), 0, s, Xd, n, ldx, p, K, c_hat,        \
                           k.rows_per, k.cols, psum, pcnt);                                                        \
    else                                                                                                           \
        hipLaunchKernelGGL((k_km2_sums_reg<float, KR>), grid, dim3(k.cols), 0, s, Xf, n, ldx, p, K, c_hat,         \
                           k.rows_per, k.cols, psum, pcnt);
        if (K <= 4) {
            PDS_KM2_SUMS_REG(4)
        } else if (K <= 8) {
            PDS_KM2_SUMS_REG(8)
        } else if (K <= 16) {
            PDS_KM2_SUMS_REG(16)
        } else if (prec == 0) {
            hipLaunchKernelGGL(k_km2_sums<double>, grid, dim3(k.cols), lds, s, Xd, n, ldx, p, K, c_hat, k.rows_per,
                               k.cols, psum, pcnt);
        } else {
            hipLaunchKernelGGL(k_km2_sums<float>, grid, dim3(k.cols), lds, s, Xf, n, ldx, p, K, c_hat, k.rows_per,
                               k.cols, psum, pcnt);
        }
#undef PDS_KM2_SUMS_REG
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        ProfScope ps_("km2_update", s);
        hipLaunchKernelGGL(k_km2_update, dim3((unsigned)((KP * 8 + 255) / 256)), dim3(256), 0, s, psum, pcnt,
                           k.nranges, K, p, mu_hat, mu_out);
    }
    return hipGetLastError();
}

}  // namespace pds
