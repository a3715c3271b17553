// Batched form: many independent data sets (each with its own p, m, K and
// seed) compressed in one persistent launch, then sparsified K-means rounds
// (Sec. VI; Alg. 1) over all sets with three launches per round.
//
// Compression: one wavefront per group of spw consecutive samples of one set.
// The lanes first draw the group's kept sets into LDS bitmaps (Floyd + Lemire
// on Philox words, exactly as the single-plan sampler), then the wave
// transforms the group's rows one at a time (register/LDS Walsh-Hadamard, the
// single-plan fast transform) and emits each row's kept coordinates in
// ascending order straight from its bitmap, writing idx and the gathered
// values together.  Groups are dealt to the persistent workgroups round-robin.
//
// K-means round (three launches):
//   assign  one thread per sample over items of `achunk` samples: FP32
//           distances to the set's centers (a transposed FP32 copy), FP64
//           recheck of near ties as in the single-plan kernel, assignment and
//           per-item objective partial.
//   accum   one workgroup per (set, sample chunk, cluster group): the chunk's
//           samples whose cluster falls in the group add their kept entries
//           into LDS sums and counts (one wave per sample), then the group's
//           K_g x p partial is written out.
//   update  one thread per center entry: fixed-order FP64 sum of the chunk
//           partials, division (zero count keeps the previous value), the
//           FP32 transposed copy and the largest |center| for the next round;
//           the first thread of a set sums its objective partials.
#include "pds_batch.hpp"
#include "pds_device.hpp"
#include "pds_fast.hpp"
#include "pds_internal.hpp"
#include "pds_sample.hpp"

namespace pds {

// index of the set owning item `it`: largest d with prefix[d] <= it
__device__ inline int owner(const int64_t* __restrict__ prefix, int nsets, int64_t it)
{
    int lo = 0, hi = nsets - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= it)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// compression
// ---------------------------------------------------------------------------
template <int L>
__device__ inline void batch_rows(const BatchSet& S, int64_t r0, int nrows, int spw, int words,
                                  const uint32_t* __restrict__ bitmap, const uint32_t* __restrict__ negbits,
                                  float* __restrict__ buf, int lane)
{
    constexpr int E = (1 << L) / 64;
    const int stride = spw + 1;
    const uint64_t negmask = fast_negmask<float, L>(negbits, lane);
    float x[E];
    load_row<float, L>(x, S.X + r0 * S.ldx, lane);
    for (int k = 0; k < nrows; ++k) {
        fast_transform_to_lds<float, L>(x, negmask, buf, lane);
        if (k + 1 < nrows) load_row<float, L>(x, S.X + (r0 + k + 1) * S.ldx, lane);
        uint16_t* ix = S.idx + (r0 + k) * (int64_t)S.m;
        float* v = S.vals + (r0 + k) * (int64_t)S.m;
        emit_sorted(bitmap, stride, k, words, lane, [&](int pos, int c) {
            ix[pos] = (uint16_t)c;
            v[pos] = buf[lds_pad<float>(c)];
        });
    }
}

__global__ __launch_bounds__(64) void k_batch_compress(const BatchSet* __restrict__ sets, int nsets,
                                                       const int64_t* __restrict__ gprefix, int64_t ngroups, int spw,
                                                       int words_max, int pmax)
{
    extern __shared__ __align__(16) uint32_t lds[];
    uint32_t* bitmap = lds;                                     // [words_max][spw + 1]
    uint32_t* negbits = bitmap + words_max * (spw + 1);         // [pmax / 32]
    float* buf = reinterpret_cast<float*>(negbits + pmax / 32);  // lds_pad(pmax - 1) + 1
    const int lane = threadIdx.x;
    const int stride = spw + 1;
    int cur = -1;
    for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const int d = owner(gprefix, nsets, g);
        const BatchSet& S = sets[d];
        const int p = S.p;
        const int words = p >> 5;
        __syncthreads();  // the previous group's reads of bitmap and negbits are done
        if (d != cur) {
            for (int b = lane; b < (p + 255) / 256; b += 64) {
                const u64x4 blk = sign_block(S.seed, (uint64_t)b);
#pragma unroll
                for (int w = 0; w < 8; ++w)
                    if (b * 8 + w < words) negbits[b * 8 + w] = (w & 1) ? (uint32_t)(blk.w[w >> 1] >> 32)
                                                                        : (uint32_t)blk.w[w >> 1];
            }
            cur = d;
        }
        for (int e = lane; e < words * stride; e += 64) bitmap[e] = 0u;
        __syncthreads();
        const int64_t r0 = (g - gprefix[d]) * (int64_t)spw;
        const int64_t left = S.n - r0;
        const int nrows = left < spw ? (int)left : spw;
        if (lane < nrows) floyd_bitmap(S.seed, (uint64_t)(r0 + lane), p, S.m, bitmap, stride, lane);
        __syncthreads();
        switch (S.L) {
            case 7: batch_rows<7>(S, r0, nrows, spw, words, bitmap, negbits, buf, lane); break;
            case 8: batch_rows<8>(S, r0, nrows, spw, words, bitmap, negbits, buf, lane); break;
            case 9: batch_rows<9>(S, r0, nrows, spw, words, bitmap, negbits, buf, lane); break;
            case 10: batch_rows<10>(S, r0, nrows, spw, words, bitmap, negbits, buf, lane); break;
            default: batch_rows<11>(S, r0, nrows, spw, words, bitmap, negbits, buf, lane); break;
        }
    }
}

// ---------------------------------------------------------------------------
// K-means
// ---------------------------------------------------------------------------
constexpr int kBkThreads = 256;
constexpr int kBkGroup = 16;

__device__ inline const double* round_in(const BatchSet& S, int dir) { return dir ? S.c_a : S.c_b; }
__device__ inline double* round_out(const BatchSet& S, int dir) { return dir ? S.c_b : S.c_a; }

// prep: one workgroup per set; FP32 transposed centers, largest |center|, and
// (odd round counts) the second center buffer
__global__ __launch_bounds__(256) void k_batch_prep(const BatchSet* __restrict__ sets, int nsets,
                                                    float* __restrict__ ct, uint32_t* __restrict__ cmax0,
                                                    int copy_to_b)
{
    __shared__ uint32_t red[256];
    const int d = blockIdx.x;
    const BatchSet& S = sets[d];
    const int64_t KP = (int64_t)S.K * S.p;
    float* c = ct + S.ct_off;
    uint32_t mx = 0;
    for (int64_t e = threadIdx.x; e < KP; e += 256) {
        const double v = S.c_a[e];
        const int64_t k = e / S.p, l = e - k * S.p;
        const float f = (float)v;
        c[l * S.K + k] = f;
        mx = max(mx, __float_as_uint(fabsf(f)));
        if (copy_to_b) S.c_b[e] = v;
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) cmax0[d] = red[0];
}

// FP64 distance in the oracle's order (ascending kept coordinate, fma)
__device__ inline double batch_dist_f64(const float* __restrict__ v, const uint16_t* __restrict__ ix, int m,
                                        const double* __restrict__ c)
{
    double dd = 0.0;
    for (int a = 0; a < m; ++a) {
        const double diff = (double)v[a] - c[ix[a]];
        dd = fma(diff, diff, dd);
    }
    return dd;
}

__global__ __launch_bounds__(kBkThreads) void k_batch_assign(const BatchSet* __restrict__ sets, int nsets,
                                                             const int64_t* __restrict__ aprefix, int64_t nitems,
                                                             int achunk, const float* __restrict__ ct,
                                                             const uint32_t* __restrict__ cmax_cur,
                                                             uint32_t* __restrict__ cmax_next, double* __restrict__ pobj,
                                                             int dir)
{
    __shared__ double red[kBkThreads / 64];
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int d = owner(aprefix, nsets, it);
        const BatchSet& S = sets[d];
        const int64_t j = it - aprefix[d];
        if (j == 0 && threadIdx.x == 0) cmax_next[d] = 0u;
        const double* cin = round_in(S, dir);
        const float* cT = ct + S.ct_off;
        const float cmax = __uint_as_float(cmax_cur[d]);
        const int K = S.K, m = S.m;
        const int64_t i = j * achunk + threadIdx.x;
        double obj = 0.0;
        for (int64_t ii = i; ii < S.n && ii < (j + 1) * (int64_t)achunk; ii += kBkThreads) {
            const float* v = S.vals + ii * (int64_t)m;
            const uint16_t* ix = S.idx + ii * (int64_t)m;
            float best = INFINITY, second = INFINITY, sv = 0.0f;
            int bestk = 0;
            for (int k0 = 0; k0 < K; k0 += kBkGroup) {
                float dk[kBkGroup];
#pragma unroll
                for (int q = 0; q < kBkGroup; ++q) dk[q] = 0.0f;
                const int kn = (K - k0) < kBkGroup ? (K - k0) : kBkGroup;
                for (int a = 0; a < m; ++a) {
                    const float x = v[a];
                    const float* c = cT + (int64_t)ix[a] * K + k0;
                    if (k0 == 0) sv = fmaf(x, x, sv);
#pragma unroll
                    for (int q = 0; q < kBkGroup; ++q) {
                        if (q < kn) {
                            const float diff = x - c[q];
                            dk[q] = fmaf(diff, diff, dk[q]);
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < kBkGroup; ++q) {
                    if (q < kn) {
                        if (dk[q] < best) {
                            second = best;
                            best = dk[q];
                            bestk = k0 + q;
                        } else if (dk[q] < second) {
                            second = dk[q];
                        }
                    }
                }
            }
            double dsel = (double)best;
            if (K > 1) {
                // |d32 - d| <= u (8 (sum v^2 + sum mu^2) + 1.01 m d), u = 2^-24,
                // per candidate; two candidates, factor 2 of slack
                const float u = 5.9604645e-8f;
                const float mf = (float)m;
                const float bound = 2.0f * u * (16.0f * (sv + mf * cmax * cmax) + 1.01f * mf * (best + second));
                if (!(second - best > bound)) {
                    double b64 = batch_dist_f64(v, ix, m, cin);
                    int bk = 0;
                    for (int k = 1; k < K; ++k) {
                        const double dk = batch_dist_f64(v, ix, m, cin + (int64_t)k * S.p);
                        if (dk < b64) {
                            b64 = dk;
                            bk = k;
                        }
                    }
                    bestk = bk;
                    dsel = b64;
                }
            }
            S.assign[ii] = bestk;
            obj += dsel;
        }
        // fixed-order workgroup sum of the objective
        for (int off = 32; off > 0; off >>= 1) obj += __shfl_down(obj, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = obj;
        __syncthreads();
        if (threadIdx.x == 0) pobj[S.aitem0 + j] = red[0] + red[1] + red[2] + red[3];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBkThreads) void k_batch_accum(const BatchSet* __restrict__ sets, int nsets,
                                                            const int64_t* __restrict__ cprefix, int64_t nitems,
                                                            float* __restrict__ psum, uint32_t* __restrict__ pcnt)
{
    extern __shared__ __align__(16) unsigned char smem[];
    float* sums = reinterpret_cast<float*>(smem);
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int d = owner(cprefix, nsets, it);
        const BatchSet& S = sets[d];
        const int64_t j = it - cprefix[d];
        const int grp = (int)(j % S.ngk);
        const int64_t chunk = j / S.ngk;
        const int k0 = grp * S.kg;
        const int kg = (S.K - k0) < S.kg ? (S.K - k0) : S.kg;
        const int p = S.p, m = S.m;
        const int ent = kg * p;
        uint32_t* cnts = reinterpret_cast<uint32_t*>(sums + ent);
        __syncthreads();  // the previous item's LDS reads are done
        for (int e = threadIdx.x; e < ent; e += kBkThreads) {
            sums[e] = 0.0f;
            cnts[e] = 0u;
        }
        __syncthreads();
        const int64_t s0 = chunk * S.cchunk;
        int64_t s1 = s0 + S.cchunk;
        if (s1 > S.n) s1 = S.n;
        for (int64_t base = s0 + (int64_t)wv * 64; base < s1; base += kBkThreads) {
            const int64_t mine = base + lane;
            int c = -1;
            if (mine < s1) c = S.assign[mine];
            const bool in = c >= k0 && c < k0 + kg;
            uint64_t mask = __ballot(in);
            while (mask) {
                const int b = __builtin_ctzll(mask);
                mask &= mask - 1ull;
                const int cb = __shfl(c, b, 64);
                const int64_t i = base + b;
                const float* v = S.vals + i * (int64_t)m;
                const uint16_t* ix = S.idx + i * (int64_t)m;
                float* sk = sums + (cb - k0) * p;
                uint32_t* ck = cnts + (cb - k0) * p;
                for (int a = lane; a < m; a += 64) {
                    const int l = ix[a];
                    atomicAdd(&sk[l], v[a]);
                    atomicAdd(&ck[l], 1u);
                }
            }
        }
        __syncthreads();
        const int64_t KP = (int64_t)S.K * p;
        float* ps = psum + S.part_off + chunk * KP + (int64_t)k0 * p;
        uint32_t* pc = pcnt + S.part_off + chunk * KP + (int64_t)k0 * p;
        for (int e = threadIdx.x; e < ent; e += kBkThreads) {
            ps[e] = sums[e];
            pc[e] = cnts[e];
        }
    }
}

__global__ __launch_bounds__(256) void k_batch_update(const BatchSet* __restrict__ sets, int nsets,
                                                      const int64_t* __restrict__ uprefix, int64_t nitems,
                                                      const float* __restrict__ psum, const uint32_t* __restrict__ pcnt,
                                                      float* __restrict__ ct, uint32_t* __restrict__ cmax_next,
                                                      const double* __restrict__ pobj, int dir, int round)
{
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int d = owner(uprefix, nsets, it);
        const BatchSet& S = sets[d];
        const int64_t j = it - uprefix[d];
        const int64_t KP = (int64_t)S.K * S.p;
        const int64_t e = j * 256 + threadIdx.x;
        if (j == 0 && threadIdx.x == 0) {
            double o = 0.0;
            for (int64_t a = 0; a < S.naitems; ++a) o += pobj[S.aitem0 + a];
            S.objective[round] = o;
        }
        if (e >= KP) continue;
        double sum = 0.0;
        uint64_t cnt = 0;
        for (int64_t c = 0; c < S.nacc; ++c) {
            sum += (double)psum[S.part_off + c * KP + e];
            cnt += pcnt[S.part_off + c * KP + e];
        }
        const double* cin = round_in(S, dir);
        const double nv = (cnt > 0) ? sum / (double)cnt : cin[e];
        round_out(S, dir)[e] = nv;
        const int64_t k = e / S.p, l = e - k * S.p;
        const float f = (float)nv;
        ct[S.ct_off + l * S.K + k] = f;
        atomicMax(&cmax_next[d], __float_as_uint(fabsf(f)));
    }
}

// initial centers: center k of a set = its compressed sample k, zero-filled
// (k < n; further centers zero)
__global__ __launch_bounds__(256) void k_batch_init(const BatchSet* __restrict__ sets, int nsets,
                                                    const int64_t* __restrict__ uprefix, int64_t nitems)
{
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int d = owner(uprefix, nsets, it);
        const BatchSet& S = sets[d];
        const int64_t j = it - uprefix[d];
        const int64_t KP = (int64_t)S.K * S.p;
        const int64_t e = j * 256 + threadIdx.x;
        if (e >= KP) continue;
        const int64_t k = e / S.p;
        const int l = (int)(e - k * S.p);
        double v = 0.0;
        if (k < S.n) {
            const uint16_t* ix = S.idx + k * (int64_t)S.m;
            int lo = 0, hi = S.m - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if ((int)ix[mid] < l)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            if ((int)ix[lo] == l) v = (double)S.vals[k * (int64_t)S.m + lo];
        }
        S.c_a[e] = v;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t batch_init_attributes()
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_compress),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_accum),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kBatchAccumLds);
    return e;
}

size_t batch_compress_lds(int spw, int pmax)
{
    const int words = pmax / 32;
    return ((size_t)words * (spw + 1) + pmax / 32) * 4 + (size_t)(lds_pad<float>(pmax - 1) + 1) * 4;
}

hipError_t launch_batch_compress(const BatchSet* sets, int nsets, const int64_t* gprefix, int64_t ngroups, int spw,
                                 int pmax, int64_t grid, hipStream_t s)
{
    if (ngroups <= 0) return hipSuccess;
    const size_t lds = batch_compress_lds(spw, pmax);
    if (grid > ngroups) grid = ngroups;
    ProfScope ps_("batch_compress", s);
    hipLaunchKernelGGL(k_batch_compress, dim3((unsigned)grid), dim3(64), lds, s, sets, nsets, gprefix, ngroups, spw,
                       pmax / 32, pmax);
    return hipGetLastError();
}

int batch_compress_occupancy(int spw, int pmax)
{
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_batch_compress, 64, batch_compress_lds(spw, pmax)) !=
            hipSuccess ||
        b < 1)
        b = 4;
    return b;
}

hipError_t launch_batch_init(const BatchSet* sets, int nsets, const int64_t* uprefix, int64_t nitems, int64_t grid,
                             hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    if (grid > nitems) grid = nitems;
    hipLaunchKernelGGL(k_batch_init, dim3((unsigned)grid), dim3(256), 0, s, sets, nsets, uprefix, nitems);
    return hipGetLastError();
}

hipError_t launch_batch_round_prep(const BatchSet* sets, int nsets, float* ct, uint32_t* cmax0, int copy_to_b,
                                   hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_prep, dim3(nsets), dim3(256), 0, s, sets, nsets, ct, cmax0, copy_to_b);
    return hipGetLastError();
}

hipError_t launch_batch_round(const BatchSet* sets, int nsets, const BatchTables& t, const BatchTuning& tu,
                              int dir, int round, hipStream_t s)
{
    uint32_t* cm_cur = t.cmax + (size_t)(round & 1) * nsets;
    uint32_t* cm_next = t.cmax + (size_t)((round + 1) & 1) * nsets;
    if (t.naitems > 0) {
        int64_t grid = t.naitems < tu.assign_grid ? t.naitems : tu.assign_grid;
        hipLaunchKernelGGL(k_batch_assign, dim3((unsigned)grid), dim3(kBkThreads), 0, s, sets, nsets, t.aprefix,
                           t.naitems, tu.achunk, t.ct, cm_cur, cm_next, t.pobj, dir);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (t.ncitems > 0) {
        int64_t grid = t.ncitems < tu.accum_grid ? t.ncitems : tu.accum_grid;
        hipLaunchKernelGGL(k_batch_accum, dim3((unsigned)grid), dim3(kBkThreads), (size_t)kBatchAccumLds, s, sets,
                           nsets, t.cprefix, t.ncitems, t.psum, t.pcnt);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (t.nuitems > 0) {
        int64_t grid = t.nuitems < tu.update_grid ? t.nuitems : tu.update_grid;
        hipLaunchKernelGGL(k_batch_update, dim3((unsigned)grid), dim3(256), 0, s, sets, nsets, t.uprefix, t.nuitems,
                           t.psum, t.pcnt, t.ct, cm_next, t.pobj, dir, round);
    }
    return hipGetLastError();
}

}  // namespace pds
