// Sparsified K-means (Sec. VI; Alg. 1) on compressed data, and unmixing.
//
// kmeans_step = one assignment pass and one coordinate-wise mean update:
//   step 1 (eq. assignments): c_i = argmin_k sum_{l in Omega_i} (y_il - mu'_kl)^2,
//          ties to the lowest k; J' = sum_i d(i, c_i) (eq. CK_means).
//   step 2 (eq. mu_update_two): mu'_kl = S_kl / N_kl with S_kl, N_kl the sum and
//          count of kept entries at coordinate l over cluster k; N_kl = 0 keeps
//          the previous value (the coordinate cannot be estimated).
//
// Pass 1 (k_kmeans_assign) reads every compressed sample once: one thread per
// sample, the K center values of a coordinate contiguous in an LDS copy of
// mu'^T (so a kept entry costs one short contiguous LDS read), distances kept in
// registers, then the sample's m entries are added into per-workgroup LDS sums
// and counts of its cluster.  Each workgroup writes its partial sums once.
// Pass 2 (k_kmeans_update) adds the partials of all workgroups in a fixed order
// in FP64 and divides.
//
// FP32 plans: distances are FP32.  A sample whose best and second-best
// distances are closer than a bound on the FP32 rounding error is recomputed in
// FP64 with the same operation order as an FP64 plan (ascending kept
// coordinate, fused multiply-add), so the assignment equals the FP64 argmin.
//
// When K x p is too large for LDS the centers are read from a transposed copy
// in the workspace and the sums go to FP64 global atomics instead.
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

constexpr int kKmThreads = 256;
constexpr int kKmGroup = 16;  // clusters per register group
constexpr size_t kKmLdsMax = 150 * 1024;

template <typename T>
struct SumType {
    using type = float;
};
template <>
struct SumType<double> {
    using type = double;
};

__device__ inline double block_sum_f64(double v, double* red)
{
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0)
        for (int w = 0; w < kKmThreads / 64; ++w) s += red[w];
    return s;
}

__device__ inline float block_max_f32(float v, float* red)
{
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_down(v, off, 64));
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    float s = red[0];
    for (int w = 1; w < kKmThreads / 64; ++w) s = fmaxf(s, red[w]);
    __syncthreads();
    return s;
}

// FP64 distance in the oracle's order (ascending kept coordinate, fma).
template <typename T>
__device__ inline double dist_f64(const T* __restrict__ v, const uint16_t* __restrict__ ix, int m,
                                  const double* __restrict__ c)
{
    double d = 0.0;
    for (int a = 0; a < m; ++a) {
        double diff = (double)v[a] - c[ix[a]];
        d = fma(diff, diff, d);
    }
    return d;
}

// GLOBAL = centers from workspace copy, sums via FP64 global atomics.
template <typename T, bool GLOBAL>
__global__ __launch_bounds__(kKmThreads) void k_kmeans_assign(const T* __restrict__ vals,
                                                              const uint16_t* __restrict__ idx, int64_t n, int m,
                                                              int p, int K, const double* __restrict__ cin,
                                                              const T* __restrict__ cT_global, int64_t per_wg,
                                                              int32_t* __restrict__ assign,
                                                              typename SumType<T>::type* __restrict__ psum,
                                                              uint32_t* __restrict__ pcnt, double* __restrict__ gsum,
                                                              uint32_t* __restrict__ gcnt, double* __restrict__ pobj)
{
    using S = typename SumType<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red_d[kKmThreads / 64];
    __shared__ float red_f[kKmThreads / 64];
    const int tid = threadIdx.x;
    const int64_t KP = (int64_t)K * p;

    T* cT = nullptr;
    S* sums = nullptr;
    uint32_t* cnts = nullptr;
    if constexpr (!GLOBAL) {
        cT = reinterpret_cast<T*>(smem);
        sums = reinterpret_cast<S*>(smem + ((KP * sizeof(T) + 15) & ~(int64_t)15));
        cnts = reinterpret_cast<uint32_t*>(reinterpret_cast<unsigned char*>(sums) + ((KP * sizeof(S) + 15) & ~(int64_t)15));
        for (int64_t e = tid; e < KP; e += kKmThreads) {
            const int64_t k = e / p, l = e - k * p;
            cT[l * K + k] = (T)cin[e];
            sums[e] = (S)0;
            cnts[e] = 0u;
        }
        __syncthreads();
    } else {
        cT = const_cast<T*>(cT_global);
    }

    // largest |center entry| (FP32 rounding bound only)
    float cmax = 0.0f;
    if constexpr (sizeof(T) == 4) {
        for (int64_t e = tid; e < KP; e += kKmThreads) cmax = fmaxf(cmax, fabsf((float)cT[e]));
        cmax = block_max_f32(cmax, red_f);
    }

    const int64_t i0 = (int64_t)blockIdx.x * per_wg;
    int64_t i1 = i0 + per_wg;
    if (i1 > n) i1 = n;
    double obj = 0.0;

    for (int64_t i = i0 + tid; i < i1; i += kKmThreads) {
        const T* v = vals + i * (int64_t)m;
        const uint16_t* ix = idx + i * (int64_t)m;
        T best = (T)INFINITY, second = (T)INFINITY;
        int bestk = 0;
        T sv = (T)0;
        for (int k0 = 0; k0 < K; k0 += kKmGroup) {
            T d[kKmGroup];
#pragma unroll
            for (int q = 0; q < kKmGroup; ++q) d[q] = (T)0;
            const int kn = (K - k0) < kKmGroup ? (K - k0) : kKmGroup;
            for (int a = 0; a < m; ++a) {
                const T x = v[a];
                const T* c = cT + (int64_t)ix[a] * K + k0;
                if (k0 == 0) sv = fma(x, x, sv);
#pragma unroll
                for (int q = 0; q < kKmGroup; ++q) {
                    if (q < kn) {
                        const T diff = x - c[q];
                        d[q] = fma(diff, diff, d[q]);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < kKmGroup; ++q) {
                if (q < kn) {
                    if (d[q] < best) {
                        second = best;
                        best = d[q];
                        bestk = k0 + q;
                    } else if (d[q] < second) {
                        second = d[q];
                    }
                }
            }
        }
        double dsel = (double)best;
        if constexpr (sizeof(T) == 4) {
            // |d32 - d| <= u (8 (sum v^2 + sum mu^2) + 1.01 m d), u = 2^-24, per
            // candidate; two candidates, factor 2 of slack.
            if (K > 1) {
                const float u = 5.9604645e-8f;
                const float mf = (float)m;
                const float bound =
                    2.0f * u * (16.0f * (sv + mf * cmax * cmax) + 1.01f * mf * ((float)best + (float)second));
                if (!((float)second - (float)best > bound)) {
                    double b64 = dist_f64<T>(v, ix, m, cin);
                    int bk = 0;
                    for (int k = 1; k < K; ++k) {
                        double dk = dist_f64<T>(v, ix, m, cin + (int64_t)k * p);
                        if (dk < b64) {
                            b64 = dk;
                            bk = k;
                        }
                    }
                    bestk = bk;
                    dsel = b64;
                }
            }
        }
        assign[i] = bestk;
        obj += dsel;
        if constexpr (!GLOBAL) {
            S* sk = sums + (int64_t)bestk * p;
            uint32_t* ck = cnts + (int64_t)bestk * p;
            for (int a = 0; a < m; ++a) {
                atomicAdd(&sk[ix[a]], (S)v[a]);
                atomicAdd(&ck[ix[a]], 1u);
            }
        } else {
            double* sk = gsum + (int64_t)bestk * p;
            uint32_t* ck = gcnt + (int64_t)bestk * p;
            for (int a = 0; a < m; ++a) {
                atomicAdd(&sk[ix[a]], (double)v[a]);
                atomicAdd(&ck[ix[a]], 1u);
            }
        }
    }

    double tot = block_sum_f64(obj, red_d);
    if (tid == 0) pobj[blockIdx.x] = tot;
    if constexpr (!GLOBAL) {
        __syncthreads();
        S* ps = psum + (int64_t)blockIdx.x * KP;
        uint32_t* pc = pcnt + (int64_t)blockIdx.x * KP;
        for (int64_t e = tid; e < KP; e += kKmThreads) {
            ps[e] = sums[e];
            pc[e] = cnts[e];
        }
    }
}

template <typename S>
__global__ __launch_bounds__(256) void k_kmeans_update(const S* __restrict__ psum, const uint32_t* __restrict__ pcnt,
                                                       int nparts, int64_t KP, const double* __restrict__ cin,
                                                       double* __restrict__ cout, const double* __restrict__ pobj,
                                                       int nobj, double* __restrict__ objective)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g == 0) {
        double o = 0.0;
        for (int w = 0; w < nobj; ++w) o += pobj[w];
        *objective = o;
    }
    if (g >= KP) return;
    double sum = 0.0;
    uint64_t cnt = 0;
    for (int w = 0; w < nparts; ++w) {
        sum += (double)psum[(int64_t)w * KP + g];
        cnt += pcnt[(int64_t)w * KP + g];
    }
    cout[g] = (cnt > 0) ? sum / (double)cnt : cin[g];
}

template <typename T>
__global__ __launch_bounds__(256) void k_kmeans_prep_global(const double* __restrict__ cin, int K, int p,
                                                            T* __restrict__ cT, double* __restrict__ gsum,
                                                            uint32_t* __restrict__ gcnt)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t KP = (int64_t)K * p;
    if (g >= KP) return;
    const int64_t k = g / p, l = g - k * p;
    cT[l * K + k] = (T)cin[g];
    gsum[g] = 0.0;
    gcnt[g] = 0u;
}

// ---------------------------------------------------------------------------
// Workspace layout and launch.
// ---------------------------------------------------------------------------
struct KmPlan {
    bool global;
    int nwg;
    int64_t per_wg;
    size_t lds;
    size_t psum_bytes, pcnt_bytes, pobj_bytes, ct_bytes, gsum_bytes, gcnt_bytes;
};

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

static KmPlan km_plan(int prec, int p, int64_t n, int K, const DeviceInfo& dev)
{
    KmPlan k;
    const size_t te = (prec == 0) ? 8 : 4;  // center / value element
    const size_t se = (prec == 0) ? 8 : 4;  // partial-sum element
    const int64_t KP = (int64_t)K * p;
    const size_t lds = ((KP * te + 15) & ~(size_t)15) + ((KP * se + 15) & ~(size_t)15) + KP * 4;
    k.global = lds > kKmLdsMax;
    k.lds = k.global ? 0 : lds;
    int64_t want = (n + kKmThreads - 1) / kKmThreads;
    int64_t cap = (int64_t)dev.cus * (k.global ? 8 : 1);
    if (!k.global && lds * 2 <= kKmLdsMax) cap = (int64_t)dev.cus * 2;
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    k.nwg = (int)want;
    k.per_wg = (n + k.nwg - 1) / k.nwg;
    k.psum_bytes = k.global ? 0 : al256((size_t)k.nwg * KP * se);
    k.pcnt_bytes = k.global ? 0 : al256((size_t)k.nwg * KP * 4);
    k.pobj_bytes = al256((size_t)k.nwg * 8);
    k.ct_bytes = k.global ? al256(KP * te) : 0;
    k.gsum_bytes = k.global ? al256(KP * 8) : 0;
    k.gcnt_bytes = k.global ? al256(KP * 4) : 0;
    return k;
}

size_t kmeans_workspace(int prec, int p, int m, int64_t n, int K, const DeviceInfo& dev)
{
    (void)m;
    KmPlan k = km_plan(prec, p, n, K, dev);
    return k.psum_bytes + k.pcnt_bytes + k.pobj_bytes + k.ct_bytes + k.gsum_bytes + k.gcnt_bytes;
}

template <typename T>
static hipError_t km_launch(const KmPlan& k, int p, int m, const T* vals, const uint16_t* idx, int64_t n, int K,
                            const double* cin, double* cout, int32_t* assign, double* objective, void* ws,
                            hipStream_t s)
{
    using S = typename SumType<T>::type;
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    S* psum = reinterpret_cast<S*>(w);
    w += k.psum_bytes;
    uint32_t* pcnt = reinterpret_cast<uint32_t*>(w);
    w += k.pcnt_bytes;
    double* pobj = reinterpret_cast<double*>(w);
    w += k.pobj_bytes;
    T* cT = reinterpret_cast<T*>(w);
    w += k.ct_bytes;
    double* gsum = reinterpret_cast<double*>(w);
    w += k.gsum_bytes;
    uint32_t* gcnt = reinterpret_cast<uint32_t*>(w);
    const int64_t KP = (int64_t)K * p;
    if (k.global) {
        {
        ProfScope ps_("kmeans_prep", s);
        hipLaunchKernelGGL(k_kmeans_prep_global<T>, dim3((unsigned)((KP + 255) / 256)), dim3(256), 0, s, cin, K, p,
                           cT, gsum, gcnt);
    }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        {
        ProfScope ps_("kmeans_assign", s);
        hipLaunchKernelGGL((k_kmeans_assign<T, true>), dim3(k.nwg), dim3(kKmThreads), 0, s, vals, idx, n, m, p, K,
                           cin, cT, k.per_wg, assign, psum, pcnt, gsum, gcnt, pobj);
    }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        {
        ProfScope ps_("kmeans_update", s);
        hipLaunchKernelGGL(k_kmeans_update<double>, dim3((unsigned)((KP + 255) / 256)), dim3(256), 0, s, gsum, gcnt, 1,
                           KP, cin, cout, pobj, k.nwg, objective);
    }
        return hipGetLastError();
    }
    static bool attr_set[2] = {false, false};
    if (!attr_set[sizeof(T) == 8]) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_kmeans_assign<T, false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kKmLdsMax);
        attr_set[sizeof(T) == 8] = true;
    }
    {
        ProfScope ps_("kmeans_assign", s);
        hipLaunchKernelGGL((k_kmeans_assign<T, false>), dim3(k.nwg), dim3(kKmThreads), k.lds, s, vals, idx, n, m, p, K,
                       cin, (const T*)nullptr, k.per_wg, assign, psum, pcnt, (double*)nullptr, (uint32_t*)nullptr,
                       pobj);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        ProfScope ps_("kmeans_update", s);
        hipLaunchKernelGGL(k_kmeans_update<S>, dim3((unsigned)((KP + 255) / 256)), dim3(256), 0, s, psum, pcnt, k.nwg, KP,
                       cin, cout, pobj, k.nwg, objective);
    }
    return hipGetLastError();
}

hipError_t launch_kmeans_step(int prec, int p, int m, const void* vals, const uint16_t* idx, int64_t n, int K,
                              const double* cin, double* cout, int32_t* assign, double* objective, void* ws,
                              size_t ws_bytes, const DeviceInfo& dev, hipStream_t s)
{
    (void)ws_bytes;
    KmPlan k = km_plan(prec, p, n, K, dev);
    if (prec == 0)
        return km_launch<double>(k, p, m, reinterpret_cast<const double*>(vals), idx, n, K, cin, cout, assign,
                                 objective, ws, s);
    return km_launch<float>(k, p, m, reinterpret_cast<const float*>(vals), idx, n, K, cin, cout, assign, objective,
                            ws, s);
}

// ---------------------------------------------------------------------------
// Unmixing (eq. mu-mu'): mu_k = (H D)^T mu'_k = D (H mu'_k), FP64.  One
// workgroup per center; the transform runs in LDS, or in place in the output
// row for p beyond the LDS budget.
// ---------------------------------------------------------------------------
constexpr int kUnmixLdsElems = 4096;

__global__ __launch_bounds__(256) void k_unmix(uint64_t seed, int p, const double* __restrict__ cpre,
                                               double* __restrict__ cout)
{
    __shared__ double lbuf[kUnmixLdsElems];
    const int k = blockIdx.x;
    const int tid = threadIdx.x;
    const bool in_lds = p <= kUnmixLdsElems;
    double* buf = in_lds ? lbuf : cout + (int64_t)k * p;
    const double* src = cpre + (int64_t)k * p;
    for (int j = tid; j < p; j += 256) buf[j] = src[j];
    for (int h = 1; h < p; h <<= 1) {
        if (!in_lds) __threadfence();
        __syncthreads();
        if (!in_lds) __threadfence();
        for (int q = tid; q < p / 2; q += 256) {
            int a = (q / h) * 2 * h + (q % h);
            double u = buf[a], v = buf[a + h];
            buf[a] = u + v;
            buf[a + h] = u - v;
        }
    }
    if (!in_lds) __threadfence();
    __syncthreads();
    if (!in_lds) __threadfence();
    const double scale = 1.0 / sqrt((double)p);
    double* dst = cout + (int64_t)k * p;
    for (int j = tid; j < p; j += 256) {
        u64x4 blk = sign_block(seed, (uint64_t)(j >> 8));
        uint64_t w = blk.w[(j >> 6) & 3];
        double sgn = ((w >> (j & 63)) & 1ull) ? -1.0 : 1.0;
        dst[j] = sgn * (buf[j] * scale);
    }
}

hipError_t launch_unmix(uint64_t seed, int p, const double* cpre, int K, double* cout, hipStream_t s)
{
    if (K <= 0) return hipSuccess;
    {
        ProfScope ps_("unmix", s);
        hipLaunchKernelGGL(k_unmix, dim3(K), dim3(256), 0, s, seed, p, cpre, cout);
    }
    return hipGetLastError();
}

}  // namespace pds
