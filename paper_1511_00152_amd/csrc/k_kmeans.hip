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
// in FP64 and divides; the objective is a fixed-order sum of per-sample
// distances (k_kmeans_objective).
//
// FP32 plans: distances are FP32.  A sample whose best and second-best
// distances are closer than a bound on the FP32 rounding error is recomputed in
// FP64 with the same operation order as an FP64 plan (ascending kept
// coordinate, fused multiply-add), so the assignment equals the FP64 argmin;
// those samples are collected in a list and decided by k_kmeans_recheck, one
// wave per sample, and their entries go to FP64 side sums.
//
// When K x p is too large for LDS the centers are read from a transposed copy
// in the workspace and the sums go to global integer atomics instead.
//
// Every sum is fixed point (km_fx_*): each value is rounded once to a multiple
// of 2^-F and added as an integer, so a sum is exact and the same in any order
// of addition, and every result is deterministic.  FP32 values take one 64-bit
// word per sum; FP64 values two (high and low 32-bit parts of v 2^F), which
// keeps their rounding far below FP64's own.
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

constexpr int kKmThreads = 256;        // GLOBAL assignment path and helper kernels
constexpr int kKmLdsThreads = 1024;    // LDS path: many waves share one LDS copy of the centers and sums
constexpr int kKmGroup = 16;  // clusters per register group
constexpr size_t kKmLdsMax = 150 * 1024;

// Fixed-point sums (see the file comment).  ev: |value| < 2^ev over the
// values of the sum; lc: at most 2^lc values go into one sum.  One word:
// F = 62 - ev - lc, |sum| 2^F < 2^62.  Two words: F = 94 - ev - lc,
// v 2^F = hi 2^32 + lo with 0 <= lo <= 2^32, |sum of hi| < 2^62 and the sum
// of lo below 2^(32 + lc).
template <typename T>
constexpr int km_words() { return sizeof(T) == 8 ? 2 : 1; }

__device__ inline int km_ev(uint64_t vmax_bits)  // vmax as FP64 bits
{
    int ev = 0;
    (void)frexp(__longlong_as_double((long long)vmax_bits), &ev);
    return ev;
}

__host__ __device__ inline int km_lc(int64_t count)
{
    int l = 0;
    while (l < 62 && ((int64_t)1 << l) < count) ++l;
    return l;
}

template <typename T>
__device__ inline int km_F(int ev, int lc)
{
    return (sizeof(T) == 8 ? 94 : 62) - ev - lc;
}

__device__ inline void km_fx_add(unsigned long long* s, float v, int F)
{
    atomicAdd(s, (unsigned long long)__double2ll_rn(ldexp((double)v, F)));
}

__device__ inline void km_fx_add(unsigned long long* s, double v, int F)
{
    const double x = ldexp(v, F);
    const double h = floor(ldexp(x, -32));
    const double r = x - ldexp(h, 32);  // exact: the low part of x, in [0, 2^32)
    atomicAdd(&s[0], (unsigned long long)(long long)h);
    atomicAdd(&s[1], (unsigned long long)__double2ll_rn(r));
}

template <int WORDS>
__device__ inline double km_fx_value(const unsigned long long* s, int F)
{
    if constexpr (WORDS == 1)
        return ldexp((double)(long long)s[0], -F);
    else
        return ldexp((double)(long long)s[0], 32 - F) + ldexp((double)(long long)s[1], -F);
}

__device__ inline uint64_t dbits(double v) { return (uint64_t)__double_as_longlong(v); }

template <int NT>
__device__ inline double block_sum_f64(double v, double* red)
{
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0)
        for (int w = 0; w < NT / 64; ++w) s += red[w];
    return s;
}

template <int NT>
__device__ inline float block_max_f32(float v, float* red)
{
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_down(v, off, 64));
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    float s = red[0];
    for (int w = 1; w < NT / 64; ++w) s = fmaxf(s, red[w]);
    __syncthreads();
    return s;
}

// FP64 distance in the oracle's order (ascending kept coordinate, fma).
// Eight entries' loads (values, coordinates, then the center gathers) are
// issued together before their multiply-adds, which keep that order.
template <typename T>
__device__ inline double dist_f64(const T* __restrict__ v, const uint16_t* __restrict__ ix, int m,
                                  const double* __restrict__ c)
{
    double d = 0.0;
    int a = 0;
    for (; a + 8 <= m; a += 8) {
        double xv[8], cv[8];
        int iv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            xv[e] = (double)v[a + e];
            iv[e] = ix[a + e];
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) cv[e] = c[iv[e]];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const double diff = xv[e] - cv[e];
            d = fma(diff, diff, d);
        }
    }
    for (; a < m; ++a) {
        double diff = (double)v[a] - c[ix[a]];
        d = fma(diff, diff, d);
    }
    return d;
}

// GLOBAL = centers from workspace copy, sums via global integer atomics (scale
// from gmax, the largest |value| of the whole call, taken by k_kmeans_vmax).
// Otherwise the sums and counts sit in LDS with this workgroup's own scale
// (its samples' largest |value|, kept in wvmax for the update).
// FP32 plans: a sample whose two best distances are closer than the rounding
// bound is appended to rlist and left to k_kmeans_recheck (its assignment,
// distance and entries are written there), so no wave here runs the serial
// FP64 loop on behalf of one lane.
template <typename T, bool GLOBAL, int NT>
__global__ __launch_bounds__(NT) void k_kmeans_assign(const T* __restrict__ vals,
                                                              const uint16_t* __restrict__ idx, int64_t n, int m,
                                                              int p, int K, const double* __restrict__ cin,
                                                              const T* __restrict__ cT_global, int64_t per_wg,
                                                              int32_t* __restrict__ assign,
                                                              unsigned long long* __restrict__ psum,
                                                              uint32_t* __restrict__ pcnt,
                                                              unsigned long long* __restrict__ gsum,
                                                              uint32_t* __restrict__ gcnt, double* __restrict__ dist,
                                                              int64_t* __restrict__ rlist,
                                                              uint32_t* __restrict__ rcount,
                                                              uint64_t* __restrict__ wvmax,
                                                              unsigned long long* __restrict__ gmax, int reuse)
{
    constexpr int WS = km_words<T>();
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float red_f[NT / 64];
    __shared__ double red_d[NT / 64];
    const int tid = threadIdx.x;
    const int64_t KP = (int64_t)K * p;
    const int64_t i0 = (int64_t)blockIdx.x * per_wg;
    int64_t i1 = i0 + per_wg;
    if (i1 > n) i1 = n;

    T* cT = nullptr;
    unsigned long long* sums = nullptr;
    uint32_t* cnts = nullptr;
    int F = 0;
    if constexpr (!GLOBAL) {
        cT = reinterpret_cast<T*>(smem);
        sums = reinterpret_cast<unsigned long long*>(smem + ((KP * sizeof(T) + 15) & ~(int64_t)15));
        cnts = reinterpret_cast<uint32_t*>(reinterpret_cast<unsigned char*>(sums) + KP * 8 * WS);
        for (int64_t e = tid; e < KP; e += NT) {
            const int64_t k = e / p, l = e - k * p;
            cT[l * K + k] = (T)cin[e];
            cnts[e] = 0u;
        }
        for (int64_t e = tid; e < KP * WS; e += NT) sums[e] = 0ull;
        // this workgroup's scale: the largest |value| of its own samples (or,
        // with reuse, the one an earlier round of the same call recorded)
        double vm = 0.0;
        if (reuse) {
            vm = __longlong_as_double((long long)wvmax[blockIdx.x]);
        } else {
            const T* vb = vals + i0 * (int64_t)m;
            const int64_t cnt = (i1 > i0 ? i1 - i0 : 0) * (int64_t)m;
            for (int64_t e = tid; e < cnt; e += NT) vm = fmax(vm, fabs((double)vb[e]));
            for (int off = 32; off > 0; off >>= 1) vm = fmax(vm, __shfl_down(vm, off, 64));
            if ((tid & 63) == 0) red_d[tid >> 6] = vm;
            __syncthreads();
            vm = red_d[0];
            for (int w = 1; w < NT / 64; ++w) vm = fmax(vm, red_d[w]);
        }
        if (tid == 0) {
            if (!reuse) wvmax[blockIdx.x] = dbits(vm);
            atomicMax(gmax, (unsigned long long)dbits(vm));
        }
        F = km_F<T>(km_ev(dbits(vm)), km_lc(per_wg));
        __syncthreads();
    } else {
        cT = const_cast<T*>(cT_global);
        F = km_F<T>(km_ev((uint64_t)*gmax), km_lc(n));
    }

    // largest |center entry| (FP32 rounding bound only)
    float cmax = 0.0f;
    if constexpr (sizeof(T) == 4) {
        for (int64_t e = tid; e < KP; e += NT) cmax = fmaxf(cmax, fabsf((float)cT[e]));
        cmax = block_max_f32<NT>(cmax, red_f);
    }

    for (int64_t i = i0 + tid; i < i1; i += NT) {
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
        if constexpr (sizeof(T) == 4) {
            // |d32 - d| <= u (8 (sum v^2 + sum mu^2) + 1.01 m d), u = 2^-24, per
            // candidate; two candidates, factor 2 of slack
            if (K > 1) {
                const float u = 5.9604645e-8f;
                const float mf = (float)m;
                const float bound =
                    2.0f * u * (16.0f * (sv + mf * cmax * cmax) + 1.01f * mf * ((float)best + (float)second));
                if (!((float)second - (float)best > bound)) {
                    rlist[atomicAdd(rcount, 1u)] = i;
                    continue;
                }
            }
        }
        assign[i] = bestk;
        dist[i] = (double)best;
        unsigned long long* sk = (GLOBAL ? gsum : sums) + (int64_t)bestk * p * WS;
        uint32_t* ck = (GLOBAL ? gcnt : cnts) + (int64_t)bestk * p;
        for (int a = 0; a < m; ++a) {
            km_fx_add(sk + (int64_t)ix[a] * WS, v[a], F);
            atomicAdd(&ck[ix[a]], 1u);
        }
    }

    if constexpr (!GLOBAL) {
        __syncthreads();
        unsigned long long* ps = psum + (int64_t)blockIdx.x * KP * WS;
        uint32_t* pc = pcnt + (int64_t)blockIdx.x * KP;
        for (int64_t e = tid; e < KP * WS; e += NT) ps[e] = sums[e];
        for (int64_t e = tid; e < KP; e += NT) pc[e] = cnts[e];
    }
}

// gmax = the largest |value| of the call (GLOBAL path, before the assignment).
template <typename T>
__global__ __launch_bounds__(256) void k_kmeans_vmax(const T* __restrict__ vals, int64_t tot,
                                                     unsigned long long* __restrict__ gmax)
{
    __shared__ double red[4];
    double vm = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256)
        vm = fmax(vm, fabs((double)vals[e]));
    for (int off = 32; off > 0; off >>= 1) vm = fmax(vm, __shfl_down(vm, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = vm;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) vm = fmax(vm, red[w]);
        atomicMax(gmax, (unsigned long long)dbits(vm));
    }
}

// Row sum over the 16 lanes of a DPP row (inclusive shift-add; lane 15 of
// the row ends with the total).
__device__ inline float dpp_row_shr(float v, int n)
{
    int r;
    switch (n) {
        case 1: r = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, true); break;
        case 2: r = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, true); break;
        case 4: r = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, true); break;
        default: r = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, true); break;
    }
    return __int_as_float(r);
}

__device__ inline float dpp_row_total(float v)
{
    v += dpp_row_shr(v, 1);
    v += dpp_row_shr(v, 2);
    v += dpp_row_shr(v, 4);
    v += dpp_row_shr(v, 8);
    return v;  // the row total in lane 15 of the row
}


// 4-lane butterfly sum (DPP quad permutations): every lane of the quad ends
// with the same total (a + b and b + a are the same in floating point).
__device__ inline float quad_total(float v)
{
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xf, 0xf, true));  // [1,0,3,2]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xf, 0xf, true));  // [2,3,0,1]
    return v;
}

// One sample of the cooperative assignment (its group of W lanes): distances
// from the entries the lanes hold (x, l: E per lane, entries u W + sl, -1 past
// m; further entries are loaded here when m > E W), the decision, and the
// entries' sums and counts.  W = 16: a DPP row per sample, lane 15 decides
// and broadcasts; W = 4: a quad per sample, every lane has the totals.
template <int W, int E, int NQ4>
__device__ inline void coop_sample(int64_t i, const float (&x0)[E], const int (&l0)[E],
                                   const float* __restrict__ vals, const uint16_t* __restrict__ idx, int m, int p,
                                   int K, int KP4, const float* cT, unsigned long long* sums, uint32_t* cnt2,
                                   int fx, float cmax, int sl, int32_t* __restrict__ assign,
                                   double* __restrict__ dist, int64_t* __restrict__ rlist,
                                   uint32_t* __restrict__ rcount)
{
    constexpr int NQ = 4 * NQ4;  // clusters padded to a multiple of four
    const float* v = vals + i * (int64_t)m;
    const uint16_t* ix = idx + i * (int64_t)m;
    float d[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) d[q] = 0.0f;
    float sv = 0.0f;
    auto add_entry = [&](float xv, int lv) {
        sv = fmaf(xv, xv, sv);
        const float4* c4 = reinterpret_cast<const float4*>(cT + __umul24((unsigned)lv, (unsigned)KP4));
#pragma unroll
        for (int q4 = 0; q4 < NQ4; ++q4) {
            const float4 c = c4[q4];
            const float cc[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float diff = xv - cc[r];
                d[4 * q4 + r] = fmaf(diff, diff, d[4 * q4 + r]);
            }
        }
    };
#pragma unroll
    for (int u = 0; u < E; ++u)
        if (l0[u] >= 0) add_entry(x0[u], l0[u]);
    for (int a = E * W + sl; a < m; a += W) add_entry(v[a], (int)ix[a]);
    float best = INFINITY, second = INFINITY;
    int bestk = 0;
    int flag = 0;
    if constexpr (W == 4) {
        sv = quad_total(sv);
#pragma unroll
        for (int q = 0; q < NQ; ++q) d[q] = quad_total(d[q]);
    } else {
        sv = dpp_row_total(sv);
#pragma unroll
        for (int q = 0; q < NQ; ++q) d[q] = dpp_row_total(d[q]);
    }
    // padding clusters (q >= K) take no part
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const float dq = q < K ? d[q] : INFINITY;
        const bool nb = dq < best;
        second = nb ? best : fminf(second, dq);
        bestk = nb ? q : bestk;
        best = nb ? dq : best;
    }
    if (K > 1) {
        // |d32 - d| <= u (8 (sum v^2 + sum mu^2) + 1.01 m d), u = 2^-24, per
        // candidate; two candidates, factor 2 of slack
        const float u = 5.9604645e-8f;
        const float mf = (float)m;
        const float bound = 2.0f * u * (16.0f * (sv + mf * cmax * cmax) + 1.01f * mf * (best + second));
        flag = !(second - best > bound);
    }
    if constexpr (W == 16) {
        // lane 15 of the row holds the totals
        flag = __shfl(flag, W - 1, W);
        bestk = __shfl(bestk, W - 1, W);
    }
    if (flag) {
        if (sl == W - 1) rlist[atomicAdd(rcount, 1u)] = i;
        return;
    }
    if (sl == W - 1) {
        assign[i] = bestk;
        dist[i] = (double)best;
    }
    const int64_t kb = (int64_t)bestk * p;
    auto add_sum = [&](float xv, int lv) {
        const int64_t e = kb + lv;
        atomicAdd(&sums[e], (unsigned long long)__double2ll_rn(ldexp((double)xv, fx)));
        atomicAdd(&cnt2[e >> 1], 1u << (16 * (int)(e & 1)));
    };
    // the first E W entries from registers, any others from memory
#pragma unroll
    for (int u = 0; u < E; ++u)
        if (l0[u] >= 0) add_sum(x0[u], l0[u]);
    for (int a = E * W + sl; a < m; a += W) add_sum(v[a], (int)ix[a]);
}


// FP32 assignment with coalesced rows: a group of W lanes per sample (a quad
// for m <= 64, a DPP row otherwise), lanes over its kept entries, each lane's
// partial distances to the K <= 32 centers in registers, then a group sum.
// The summation order differs from the sequential one, but its rounding error
// obeys the same bound (every term passes through at most m additions), so the
// near-tie test and the FP64 recheck give the FP64 argmin as before.  Centers
// are transposed in LDS with rows padded to KP4 = ceil4(K) floats and read as
// float4.  Each workgroup takes its own fixed-point scale from its samples'
// largest |value|.
template <int W, int E, int NQ4>
__global__ __launch_bounds__(kKmLdsThreads) void k_kmeans_assign_coop(
    const float* __restrict__ vals, const uint16_t* __restrict__ idx, int64_t n, int m, int p, int K,
    const double* __restrict__ cin, int64_t per_wg, int32_t* __restrict__ assign, int64_t* __restrict__ psum,
    uint32_t* __restrict__ pcnt, uint64_t* __restrict__ wvmax, unsigned long long* __restrict__ gmax,
    double* __restrict__ dist, int64_t* __restrict__ rlist, uint32_t* __restrict__ rcount, int reuse)
{
    constexpr int G = kKmLdsThreads / W;  // groups per workgroup
    constexpr int AHEAD = (E >= 16) ? 1 : 2;  // samples whose first entries are in flight
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float red_f[kKmLdsThreads / 64];
    const int tid = threadIdx.x;
    const int KP4 = (K + 3) & ~3;
    const int64_t KP = (int64_t)K * p;
    // centers transposed (rows padded to 4), 64-bit fixed-point sums and
    // 16-bit counts two to a word: integer LDS atomics run at full rate, the
    // FP32 ones do not; at most 65535 samples per workgroup
    float* cT = reinterpret_cast<float*>(smem);
    unsigned long long* sums = reinterpret_cast<unsigned long long*>(cT + (int64_t)KP4 * p);
    uint32_t* cnt2 = reinterpret_cast<uint32_t*>(sums + KP);
    const int64_t i0 = (int64_t)blockIdx.x * per_wg;
    int64_t i1 = i0 + per_wg;
    if (i1 > n) i1 = n;
    // the fixed-point scale of this workgroup's sums: the largest |value| of
    // its own samples (kept in wvmax for the update; with reuse, the one an
    // earlier round of the same call recorded there)
    float vm = 0.0f;
    if (reuse) {
        vm = (float)__longlong_as_double((long long)wvmax[blockIdx.x]);
    } else {
        const float* vb = vals + i0 * (int64_t)m;
        const int64_t cnt = (i1 > i0 ? i1 - i0 : 0) * (int64_t)m;
#pragma unroll 4
        for (int64_t e = tid; e < cnt; e += kKmLdsThreads) vm = fmaxf(vm, fabsf(vb[e]));
    }
    for (int64_t e = tid; e < (int64_t)KP4 * p; e += kKmLdsThreads) {
        const int64_t l = e / KP4, k = e - l * KP4;
        cT[e] = (k < K) ? (float)cin[k * p + l] : 0.0f;
    }
    for (int64_t e = tid; e < KP; e += kKmLdsThreads) sums[e] = 0ull;
    for (int64_t e = tid; e < (KP + 1) / 2; e += kKmLdsThreads) cnt2[e] = 0u;
    __syncthreads();
    float cmax = 0.0f;
    for (int64_t e = tid; e < (int64_t)KP4 * p; e += kKmLdsThreads) cmax = fmaxf(cmax, fabsf(cT[e]));
    cmax = block_max_f32<kKmLdsThreads>(cmax, red_f);
    vm = block_max_f32<kKmLdsThreads>(vm, red_f);
    if (tid == 0) {
        if (!reuse) wvmax[blockIdx.x] = dbits((double)vm);
        atomicMax(gmax, (unsigned long long)dbits((double)vm));
    }
    const int fx = km_F<float>(km_ev(dbits((double)vm)), km_lc(per_wg));

    const int g = tid / W, sl = tid % W;
    auto load_first = [&](int64_t i, float (&x)[E], int (&l)[E]) {
        const float* v = vals + i * (int64_t)m;
        const uint16_t* ix = idx + i * (int64_t)m;
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int a = u * W + sl;
            x[u] = (a < m) ? v[a] : 0.0f;
            l[u] = (a < m) ? (int)ix[a] : -1;
        }
    };
    float xa[E], xb[E];
    int la[E], lb[E];
    if (i0 + g < i1) load_first(i0 + g, xa, la);
    if (AHEAD == 2 && i0 + g + G < i1) load_first(i0 + g + G, xb, lb);
    for (int64_t i = i0 + g; i < i1; i += G) {
        float x[E];
        int l[E];
#pragma unroll
        for (int u = 0; u < E; ++u) {
            x[u] = xa[u];
            l[u] = la[u];
            if (AHEAD == 2) {
                xa[u] = xb[u];
                la[u] = lb[u];
            }
        }
        if (AHEAD == 2) {
            if (i + 2 * G < i1) load_first(i + 2 * G, xb, lb);
        } else {
            if (i + G < i1) load_first(i + G, xa, la);
        }
        coop_sample<W, E, NQ4>(i, x, l, vals, idx, m, p, K, KP4, cT, sums, cnt2, fx, cmax, sl, assign, dist,
                               rlist, rcount);
    }
    __syncthreads();
    int64_t* ps = psum + (int64_t)blockIdx.x * KP;
    uint32_t* pc = pcnt + (int64_t)blockIdx.x * KP;
    for (int64_t e = tid; e < KP; e += kKmLdsThreads) {
        ps[e] = (int64_t)sums[e];
        pc[e] = (cnt2[e >> 1] >> (16 * (int)(e & 1))) & 0xffffu;
    }
}

// FP64 decision for the flagged samples: one wave per sample, lanes over
// clusters, each distance summed in the oracle's order; ties to the lowest k.
// The sample's entries go to the side sums (gsum_r, gcnt_r), fixed point with
// the call's largest |value| (gmax) and at most n values per sum.
__global__ __launch_bounds__(256) void k_kmeans_recheck(const float* __restrict__ vals,
                                                        const uint16_t* __restrict__ idx, int64_t n, int m, int p,
                                                        int K, const double* __restrict__ cin,
                                                        const int64_t* __restrict__ rlist,
                                                        const uint32_t* __restrict__ rcount,
                                                        int32_t* __restrict__ assign, double* __restrict__ dist,
                                                        unsigned long long* __restrict__ gsum_r,
                                                        uint32_t* __restrict__ gcnt_r,
                                                        const unsigned long long* __restrict__ gmax)
{
    const int lane = threadIdx.x & 63;
    const int F = km_F<float>(km_ev((uint64_t)*gmax), km_lc(n));
    const int64_t nw = (int64_t)gridDim.x * 4;
    const int64_t cnt = *rcount;
    for (int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); e < cnt; e += nw) {
        const int64_t i = rlist[e];
        const float* v = vals + i * (int64_t)m;
        const uint16_t* ix = idx + i * (int64_t)m;
        double bd = INFINITY;
        int bk = 0x7fffffff;
        for (int k = lane; k < K; k += 64) {
            const double dk = dist_f64<float>(v, ix, m, cin + (int64_t)k * p);
            if (dk < bd) {  // k ascends within a lane: ties keep the lower k
                bd = dk;
                bk = k;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double od = __shfl_xor(bd, off, 64);
            const int ok = __shfl_xor(bk, off, 64);
            if (od < bd || (od == bd && ok < bk)) {
                bd = od;
                bk = ok;
            }
        }
        if (lane == 0) {
            assign[i] = bk;
            dist[i] = bd;
        }
        unsigned long long* sk = gsum_r + (int64_t)bk * p;
        uint32_t* ck = gcnt_r + (int64_t)bk * p;
        for (int a = lane; a < m; a += 64) {
            km_fx_add(&sk[ix[a]], v[a], F);
            atomicAdd(&ck[ix[a]], 1u);
        }
    }
}

// objective partial of each assignment workgroup's range, fixed order
__global__ __launch_bounds__(kKmThreads) void k_kmeans_objective(const double* __restrict__ dist, int64_t n,
                                                                 int64_t per_wg, double* __restrict__ pobj)
{
    __shared__ double red[kKmThreads / 64];
    const int64_t i0 = (int64_t)blockIdx.x * per_wg;
    int64_t i1 = i0 + per_wg;
    if (i1 > n) i1 = n;
    double o = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kKmThreads) o += dist[i];
    const double t = block_sum_f64<kKmThreads>(o, red);
    if (threadIdx.x == 0) pobj[blockIdx.x] = t;
}

// Update: a workgroup per 64 center entries; its 16 waves each add every
// 16th partial for the 64 entries (coalesced), then the 16 wave sums are
// combined in a fixed order; the first workgroup also sums the objective.
// Partial w is fixed point with its workgroup's scale (PER_WG: wvmax[w] and at
// most 2^lc_part values per sum) or with the call's (gmax, 2^lc_part); the
// side sums with the call's scale and 2^lc_side.
constexpr int kUpdThreads = 1024;

template <typename T, bool PER_WG>
__global__ __launch_bounds__(kUpdThreads) void k_kmeans_update(const unsigned long long* __restrict__ psum,
                                                               const uint32_t* __restrict__ pcnt, int nparts,
                                                               int64_t KP, const uint64_t* __restrict__ wvmax,
                                                               int lc_part,
                                                               const unsigned long long* __restrict__ gsum_r,
                                                               const uint32_t* __restrict__ gcnt_r,
                                                               const unsigned long long* __restrict__ gmax,
                                                               int lc_side, const double* __restrict__ cin,
                                                               double* __restrict__ cout,
                                                               const double* __restrict__ pobj, int nobj,
                                                               double* __restrict__ objective)
{
    constexpr int WS = km_words<T>();
    __shared__ double rs[kUpdThreads / 64][64];
    __shared__ uint64_t rc[kUpdThreads / 64][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t g = (int64_t)blockIdx.x * 64 + lane;
    const int ev_g = km_ev((uint64_t)*gmax);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double o = 0.0;
        for (int w = 0; w < nobj; ++w) o += pobj[w];
        *objective = o;
    }
    double sum = 0.0;
    uint64_t cnt = 0;
    if (g < KP) {
        // eight partials' loads in flight per thread; the sum keeps partial order
#pragma unroll 8
        for (int w = wv; w < nparts; w += kUpdThreads / 64) {
            const int F = km_F<T>(PER_WG ? km_ev(wvmax[w]) : ev_g, lc_part);
            sum += km_fx_value<WS>(psum + ((int64_t)w * KP + g) * WS, F);
            cnt += pcnt[(int64_t)w * KP + g];
        }
    }
    rs[wv][lane] = sum;
    rc[wv][lane] = cnt;
    __syncthreads();
    if (wv == 0 && g < KP) {
        double t = 0.0;
        uint64_t c = 0;
        for (int w = 0; w < kUpdThreads / 64; ++w) {
            t += rs[w][lane];
            c += rc[w][lane];
        }
        t += km_fx_value<1>(gsum_r + g, km_F<float>(ev_g, lc_side));
        c += gcnt_r[g];
        cout[g] = (c > 0) ? t / (double)c : cin[g];
    }
}

// per call: side sums, counter and gmax cleared; for the GLOBAL path also the
// transposed centers and the global sums
template <typename T>
__global__ __launch_bounds__(256) void k_kmeans_prep(const double* __restrict__ cin, int K, int p, int global,
                                                     T* __restrict__ cT, unsigned long long* __restrict__ gsum,
                                                     uint32_t* __restrict__ gcnt,
                                                     unsigned long long* __restrict__ gsum_r,
                                                     uint32_t* __restrict__ gcnt_r, uint32_t* __restrict__ rcount,
                                                     unsigned long long* __restrict__ gmax)
{
    constexpr int WS = km_words<T>();
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t KP = (int64_t)K * p;
    if (g == 0) {
        *rcount = 0u;
        *gmax = 0ull;
    }
    if (g >= KP) return;
    gsum_r[g] = 0ull;
    gcnt_r[g] = 0u;
    if (global) {
        const int64_t k = g / p, l = g - k * p;
        cT[l * K + k] = (T)cin[g];
        for (int w = 0; w < WS; ++w) gsum[g * WS + w] = 0ull;
        gcnt[g] = 0u;
    }
}

// ---------------------------------------------------------------------------
// Workspace layout and launch.
// ---------------------------------------------------------------------------
struct KmPlan {
    bool global;
    int coop;  // FP32 group-per-sample assignment: lanes per sample (0 = not used)
    int nwg;
    int64_t per_wg;
    size_t lds;
    size_t psum_bytes, pcnt_bytes, pobj_bytes, ct_bytes, gsum_bytes, gcnt_bytes;
    size_t dist_bytes, rlist_bytes, rcount_bytes, gsumr_bytes, gcntr_bytes, vmax_bytes, gmax_bytes;
};

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

static KmPlan km_plan(int prec, int p, int64_t n, int K, const DeviceInfo& dev)
{
    KmPlan k;
    const size_t te = (prec == 0) ? 8 : 4;  // center / value element
    const size_t ws = (prec == 0) ? 2 : 1;  // 64-bit words per fixed-point sum
    const int64_t KP = (int64_t)K * p;
    const size_t lds = ((KP * te + 15) & ~(size_t)15) + (size_t)KP * 8 * ws + KP * 4;
    k.global = lds > kKmLdsMax;
    k.lds = k.global ? 0 : lds;
    // FP32, K <= 32: centers (rows padded to 4), 64-bit fixed-point sums and
    // 16-bit counts in LDS
    const size_t lds_coop = (size_t)((K + 3) & ~3) * p * 4 + (size_t)KP * 8 + (size_t)((KP + 1) / 2) * 4;
    k.coop = 0;
    if (prec != 0 && K <= 32 && lds_coop <= kKmLdsMax) {
        k.coop = 16;
        k.global = false;
        k.lds = lds_coop;
    }
    const int nt = k.global ? kKmThreads : kKmLdsThreads;
    // the cooperative kernel takes a quad of lanes per sample: a workgroup per
    // nt / 4 samples until every CU has one (at n = 70000 that halves the
    // assignment, 64 -> 33 us per round, for about 9 us more in the update,
    // which sums 3.7 times as many partials)
    int64_t want = k.coop ? (n + nt / 4 - 1) / (nt / 4) : (n + nt - 1) / nt;
    int64_t cap = (int64_t)dev.cus * (k.global ? 8 : 1);
    if (!k.global && lds * 2 <= kKmLdsMax) cap = (int64_t)dev.cus * 2;
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    if (k.coop && (n + want - 1) / want > 65535) want = (n + 65534) / 65535;  // 16-bit counts
    k.nwg = (int)want;
    k.per_wg = (n + k.nwg - 1) / k.nwg;
    k.psum_bytes = k.global ? 0 : al256((size_t)k.nwg * KP * 8 * (k.coop ? 1 : ws));
    k.pcnt_bytes = k.global ? 0 : al256((size_t)k.nwg * KP * 4);
    k.pobj_bytes = al256((size_t)k.nwg * 8);
    k.ct_bytes = k.global ? al256(KP * te) : 0;
    k.gsum_bytes = k.global ? al256(KP * 8 * ws) : 0;
    k.gcnt_bytes = k.global ? al256(KP * 4) : 0;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    k.dist_bytes = al256(nn * 8);
    k.rlist_bytes = (prec == 0) ? 0 : al256(nn * 8);
    k.rcount_bytes = 256;
    k.gsumr_bytes = al256(KP * 8);
    k.gcntr_bytes = al256(KP * 4);
    k.vmax_bytes = al256((size_t)k.nwg * 8);  // per-workgroup largest |value| (FP64 bits)
    k.gmax_bytes = 256;                       // the call's largest |value| (FP64 bits)
    return k;
}

size_t kmeans_workspace(int prec, int p, int m, int64_t n, int K, const DeviceInfo& dev)
{
    (void)m;
    KmPlan k = km_plan(prec, p, n, K, dev);
    return k.psum_bytes + k.pcnt_bytes + k.pobj_bytes + k.ct_bytes + k.gsum_bytes + k.gcnt_bytes + k.dist_bytes +
           k.rlist_bytes + k.rcount_bytes + k.gsumr_bytes + k.gcntr_bytes + k.vmax_bytes + k.gmax_bytes;
}

template <typename T>
static hipError_t km_launch(const KmPlan& k, int p, int m, const T* vals, const uint16_t* idx, int64_t n, int K,
                            const double* cin, double* cout, int32_t* assign, double* objective, void* ws,
                            size_t ws_bytes, const DeviceInfo& dev, hipStream_t s, bool reuse)
{
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    unsigned long long* psum = reinterpret_cast<unsigned long long*>(w);
    w += k.psum_bytes;
    uint32_t* pcnt = reinterpret_cast<uint32_t*>(w);
    w += k.pcnt_bytes;
    double* pobj = reinterpret_cast<double*>(w);
    w += k.pobj_bytes;
    T* cT = reinterpret_cast<T*>(w);
    w += k.ct_bytes;
    unsigned long long* gsum = reinterpret_cast<unsigned long long*>(w);
    w += k.gsum_bytes;
    uint32_t* gcnt = reinterpret_cast<uint32_t*>(w);
    w += k.gcnt_bytes;
    double* dist = reinterpret_cast<double*>(w);
    w += k.dist_bytes;
    int64_t* rlist = reinterpret_cast<int64_t*>(w);
    w += k.rlist_bytes;
    uint32_t* rcount = reinterpret_cast<uint32_t*>(w);
    w += k.rcount_bytes;
    unsigned long long* gsum_r = reinterpret_cast<unsigned long long*>(w);
    w += k.gsumr_bytes;
    uint32_t* gcnt_r = reinterpret_cast<uint32_t*>(w);
    w += k.gcntr_bytes;
    uint64_t* wvmax = reinterpret_cast<uint64_t*>(w);
    w += k.vmax_bytes;
    unsigned long long* gmax = reinterpret_cast<unsigned long long*>(w);
    w += k.gmax_bytes;
    // every carved buffer ends inside the caller's workspace (checked on the
    // host, before any launch)
    if ((size_t)(w - reinterpret_cast<unsigned char*>(ws)) > ws_bytes) return hipErrorInvalidValue;
    const int64_t KP = (int64_t)K * p;
    {
        ProfScope ps_("kmeans_prep", s);
        hipLaunchKernelGGL(k_kmeans_prep<T>, dim3((unsigned)((KP + 255) / 256)), dim3(256), 0, s, cin, K, p,
                           k.global ? 1 : 0, cT, gsum, gcnt, gsum_r, gcnt_r, rcount, gmax);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (k.global) {
        {
            ProfScope ps_("kmeans_vmax", s);
            const int64_t tot = n * (int64_t)m;
            int64_t blocks = (tot + 255) / 256;
            if (blocks > (int64_t)dev.cus * 8) blocks = (int64_t)dev.cus * 8;
            hipLaunchKernelGGL(k_kmeans_vmax<T>, dim3((unsigned)blocks), dim3(256), 0, s, vals, tot, gmax);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        ProfScope ps_("kmeans_assign", s);
        hipLaunchKernelGGL((k_kmeans_assign<T, true, kKmThreads>), dim3(k.nwg), dim3(kKmThreads), 0, s, vals, idx, n,
                           m, p, K, cin, cT, k.per_wg, assign, psum, pcnt, gsum, gcnt, dist, rlist, rcount, wvmax,
                           gmax, 0);
    } else {
        if constexpr (sizeof(T) == 4) {
            if (k.coop) {
                static bool coop_attr = false;
                if (!coop_attr) {
                    const void* fns[16] = {
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<16, 4, 1>),
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<16, 4, 2>),
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<16, 4, 3>),
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<16, 4, 4>),
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<16, 4, 5>),
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<16, 4, 6>),
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<16, 4, 7>),
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<16, 4, 8>),
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<4, 16, 1>),
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<4, 16, 2>),
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<4, 16, 3>),
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<4, 16, 4>),
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<4, 16, 5>),
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<4, 16, 6>),
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<4, 16, 7>),
                        reinterpret_cast<const void*>(&k_kmeans_assign_coop<4, 16, 8>)};
                    for (const void* f : fns)
                        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kKmLdsMax);
                    coop_attr = true;
                }
                {
                    ProfScope ps_("kmeans_assign", s);
                    // K <= 32 here: one instance per number of four-cluster groups; a
                    // quad per sample while its entries fit sixteen per lane
#define PDS_KM_COOP(W_, E_, Q)                                                                                 \
    case Q:                                                                                                    \
        hipLaunchKernelGGL((k_kmeans_assign_coop<W_, E_, Q>), dim3(k.nwg), dim3(kKmLdsThreads), k.lds, s, vals, idx, \
                           n, m, p, K, cin, k.per_wg, assign, reinterpret_cast<int64_t*>(psum), pcnt, wvmax, gmax,   \
                           dist, rlist, rcount, reuse ? 1 : 0);                                                \
        break;
                    if (m <= 64) {
                        switch ((K + 3) / 4) {
                            PDS_KM_COOP(4, 16, 1)
                            PDS_KM_COOP(4, 16, 2)
                            PDS_KM_COOP(4, 16, 3)
                            PDS_KM_COOP(4, 16, 4)
                            PDS_KM_COOP(4, 16, 5)
                            PDS_KM_COOP(4, 16, 6)
                            PDS_KM_COOP(4, 16, 7)
                            default: PDS_KM_COOP(4, 16, 8)
                        }
                    } else {
                        switch ((K + 3) / 4) {
                            PDS_KM_COOP(16, 4, 1)
                            PDS_KM_COOP(16, 4, 2)
                            PDS_KM_COOP(16, 4, 3)
                            PDS_KM_COOP(16, 4, 4)
                            PDS_KM_COOP(16, 4, 5)
                            PDS_KM_COOP(16, 4, 6)
                            PDS_KM_COOP(16, 4, 7)
                            default: PDS_KM_COOP(16, 4, 8)
                        }
                    }
#undef PDS_KM_COOP
                }
                goto assigned;
            }
        }
        static bool attr_set[2] = {false, false};
        if (!attr_set[sizeof(T) == 8]) {
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_kmeans_assign<T, false, kKmLdsThreads>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)kKmLdsMax);
            attr_set[sizeof(T) == 8] = true;
        }
        ProfScope ps_("kmeans_assign", s);
        hipLaunchKernelGGL((k_kmeans_assign<T, false, kKmLdsThreads>), dim3(k.nwg), dim3(kKmLdsThreads), k.lds, s,
                           vals, idx, n, m, p, K, cin, (const T*)nullptr, k.per_wg, assign, psum, pcnt,
                           (unsigned long long*)nullptr, (uint32_t*)nullptr, dist, rlist, rcount, wvmax, gmax,
                           reuse ? 1 : 0);
    }
assigned:
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if constexpr (sizeof(T) == 4) {
        ProfScope ps_("kmeans_recheck", s);
        hipLaunchKernelGGL(k_kmeans_recheck, dim3((unsigned)dev.cus * 4), dim3(256), 0, s, vals, idx, n, m, p, K,
                           cin, rlist, rcount, assign, dist, gsum_r, gcnt_r, gmax);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        ProfScope ps_("kmeans_objective", s);
        hipLaunchKernelGGL(k_kmeans_objective, dim3(k.nwg), dim3(kKmThreads), 0, s, dist, n, k.per_wg, pobj);  // fixed order
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        ProfScope ps_("kmeans_update", s);
        const unsigned ublocks = (unsigned)((KP + 63) / 64);
        const int lc_n = km_lc(n), lc_wg = km_lc(k.per_wg);
        if (k.global)
            hipLaunchKernelGGL((k_kmeans_update<T, false>), dim3(ublocks), dim3(kUpdThreads), 0, s, gsum, gcnt, 1, KP,
                               wvmax, lc_n, gsum_r, gcnt_r, gmax, lc_n, cin, cout, pobj, k.nwg, objective);
        else if (sizeof(T) == 4 && k.coop)
            hipLaunchKernelGGL((k_kmeans_update<float, true>), dim3(ublocks), dim3(kUpdThreads), 0, s, psum, pcnt,
                               k.nwg, KP, wvmax, lc_wg, gsum_r, gcnt_r, gmax, lc_n, cin, cout, pobj, k.nwg,
                               objective);
        else
            hipLaunchKernelGGL((k_kmeans_update<T, true>), dim3(ublocks), dim3(kUpdThreads), 0, s, psum, pcnt, k.nwg,
                               KP, wvmax, lc_wg, gsum_r, gcnt_r, gmax, lc_n, cin, cout, pobj, k.nwg, objective);
    }
    return hipGetLastError();
}

hipError_t launch_kmeans_step(int prec, int p, int m, const void* vals, const uint16_t* idx, int64_t n, int K,
                              const double* cin, double* cout, int32_t* assign, double* objective, void* ws,
                              size_t ws_bytes, const DeviceInfo& dev, hipStream_t s, bool reuse_scale)
{
    KmPlan k = km_plan(prec, p, n, K, dev);
    if (prec == 0)
        return km_launch<double>(k, p, m, reinterpret_cast<const double*>(vals), idx, n, K, cin, cout, assign,
                                 objective, ws, ws_bytes, dev, s, reuse_scale);
    return km_launch<float>(k, p, m, reinterpret_cast<const float*>(vals), idx, n, K, cin, cout, assign, objective,
                            ws, ws_bytes, dev, s, reuse_scale);
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
