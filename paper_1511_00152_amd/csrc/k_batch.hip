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
//   assign  one thread per sample, 1024 samples per workgroup: FP32
//           distances to the set's centers (a transposed FP32 copy staged
//           through LDS by blocks of coordinates), FP64 recheck of near ties
//           as in the single-plan kernel, assignment and objective partial.
//   accum   one workgroup per (set, sample chunk, cluster group): the chunk's
//           samples whose cluster falls in the group add their kept entries
//           into LDS sums and counts (one wave per sample), then the
//           group's K_g x p partial is written out.
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
// CALLER tells the two kernels' instantiations apart: with one caller each,
// the compiler keeps the register allocation it gives a single kernel (shared,
// it inlined into neither and the batched kernel lost a wave per SIMD)
template <int L, int CALLER>
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
        if (spw <= 32) {
            // lane q + 32 evaluates every other Philox block for lane q's sample
            const int q = lane & 31;
            floyd_bitmap_pair(S.seed, (uint64_t)(r0 + q), p, S.m, bitmap, stride, q, lane < 32 && q < nrows);
        } else if (lane < nrows) {
            floyd_bitmap(S.seed, (uint64_t)(r0 + lane), p, S.m, bitmap, stride, lane);
        }
        __syncthreads();
        switch (S.L) {
            case 7: batch_rows<7, 0>(S, r0, nrows, spw, words, bitmap, negbits, buf, lane); break;
            case 8: batch_rows<8, 0>(S, r0, nrows, spw, words, bitmap, negbits, buf, lane); break;
            case 9: batch_rows<9, 0>(S, r0, nrows, spw, words, bitmap, negbits, buf, lane); break;
            case 10: batch_rows<10, 0>(S, r0, nrows, spw, words, bitmap, negbits, buf, lane); break;
            default: batch_rows<11, 0>(S, r0, nrows, spw, words, bitmap, negbits, buf, lane); break;
        }
    }
}

// Single-plan compression with the sampler fused in (FP32 values, p in
// [512, 2048], 16-byte aligned rows): the group loop above for one data set,
// the kept sets drawn for global sample indices i0 + r, so that idx is written
// once, straight from the bitmaps, and never read back.
__global__ __launch_bounds__(64) void k_compress_fused(uint64_t seed, int p, int m, int L, const float* __restrict__ X,
                                                       int64_t n, int64_t ldx, uint64_t i0, float* __restrict__ vals,
                                                       uint16_t* __restrict__ idx, int spw, int64_t ngroups)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const int words = p >> 5;
    const int stride = spw + 1;
    uint32_t* bitmap = lds;                                      // [words][spw + 1]
    uint32_t* negbits = bitmap + words * stride;                 // [words]
    float* buf = reinterpret_cast<float*>(negbits + words);      // lds_pad(p - 1) + 1
    const int lane = threadIdx.x;
    for (int b = lane; b < (p + 255) / 256; b += 64) {
        const u64x4 blk = sign_block(seed, (uint64_t)b);
#pragma unroll
        for (int w = 0; w < 8; ++w)
            if (b * 8 + w < words)
                negbits[b * 8 + w] = (w & 1) ? (uint32_t)(blk.w[w >> 1] >> 32) : (uint32_t)blk.w[w >> 1];
    }
    BatchSet S{};
    S.X = X;
    S.vals = vals;
    S.idx = idx;
    S.n = n;
    S.ldx = ldx;
    S.p = p;
    S.m = m;
    S.L = L;
    S.seed = seed;
    for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        __syncthreads();  // the previous group's reads of the bitmaps are done (and negbits is written)
        for (int e = lane; e < words * stride; e += 64) bitmap[e] = 0u;
        __syncthreads();
        const int64_t r0 = g * (int64_t)spw;
        const int64_t left = n - r0;
        const int nrows = left < spw ? (int)left : spw;
        if (spw <= 32) {
            const int q = lane & 31;
            floyd_bitmap_pair(seed, i0 + (uint64_t)(r0 + q), p, m, bitmap, stride, q, lane < 32 && q < nrows);
        } else if (lane < nrows) {
            floyd_bitmap(seed, i0 + (uint64_t)(r0 + lane), p, m, bitmap, stride, lane);
        }
        __syncthreads();
        switch (L) {
            case 8: batch_rows<8, 1>(S, r0, nrows, spw, words, bitmap, negbits, buf, lane); break;
            case 9: batch_rows<9, 1>(S, r0, nrows, spw, words, bitmap, negbits, buf, lane); break;
            case 10: batch_rows<10, 1>(S, r0, nrows, spw, words, bitmap, negbits, buf, lane); break;
            default: batch_rows<11, 1>(S, r0, nrows, spw, words, bitmap, negbits, buf, lane); break;
        }
    }
}

// samples per group of the fused single-plan compression (n = 2^20, FP32: at
// p = 512 / 1024 / 2048, 0.62 / 1.05 / 2.21 ms with 32, 0.62 / 1.05 / 2.44 with
// 64, against 0.68 / 1.25 / 2.37 for the separate sampler and transform; at
// p = 256 the separate launches stay ahead, 0.44 against 0.45)
constexpr int kFusedSpw = 32;

bool compress_fused_ok(int prec, int p, const void* X, int64_t ldx)
{
    return prec != 0 && p >= 512 && p <= 2048 && (p & (p - 1)) == 0 && ((uintptr_t)X % 16 == 0) &&
           ((ldx * 4) % 16 == 0);
}

hipError_t launch_compress_fused(uint64_t seed, int p, int m, const float* X, int64_t n, int64_t ldx, uint64_t i0,
                                 float* vals, uint16_t* idx, const DeviceInfo& dev, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int spw = kFusedSpw;
    const int words = p / 32;
    const size_t lds = ((size_t)words * (spw + 1) + words) * 4 + (size_t)(lds_pad<float>(p - 1) + 1) * 4;
    static int per_cu[12] = {0};
    int L = 0;
    while ((1 << L) < p) ++L;
    if (per_cu[L] == 0) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_compress_fused, 64, lds) != hipSuccess || b < 1) b = 4;
        per_cu[L] = b;
    }
    const int64_t ngroups = (n + spw - 1) / spw;
    int64_t grid = (int64_t)dev.cus * per_cu[L];
    if (grid > ngroups) grid = ngroups;
    ProfScope ps_("compress", s);
    hipLaunchKernelGGL(k_compress_fused, dim3((unsigned)grid), dim3(64), lds, s, seed, p, m, L, X, n, ldx, i0, vals,
                       idx, spw, ngroups);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K-means
// ---------------------------------------------------------------------------
constexpr int kBkThreads = 256;   // update
constexpr int kBaThreads = 512;   // assign: one sample per thread
constexpr int kBaLdsFloats = 32768;  // 128 KB: one assignment workgroup per CU
constexpr int kBcThreads = 1024;  // accumulate: one sample per thread

__device__ inline const double* round_in(const BatchSet& S, int dir) { return dir ? S.c_a : S.c_b; }
__device__ inline double* round_out(const BatchSet& S, int dir) { return dir ? S.c_b : S.c_a; }

// Tiles of 64 samples: entries a = 8 c + u of lane (sample) r of tile t sit at
// ((t mp/8 + c) 64 + r) 8 + u, mp = m rounded up to a multiple of 8, so one
// thread per sample fetches eight entries with one 16-byte load of
// coordinates and two of values, and a wave's loads are contiguous.  Entries
// past m and lanes past n hold coordinate 0, value 0 (never used).
__device__ inline int64_t tile_base(const BatchSet& S, int64_t t)
{
    return S.tile_off + t * (int64_t)((S.m + 7) & ~7) * 64;
}

__global__ __launch_bounds__(256) void k_batch_tile(const BatchSet* __restrict__ sets, int nsets,
                                                    const int64_t* __restrict__ tprefix, int64_t ntiles,
                                                    float* __restrict__ vt, uint16_t* __restrict__ it,
                                                    uint32_t* __restrict__ vmax)
{
    __shared__ uint32_t red[256];
    for (int64_t g = blockIdx.x; g < ntiles; g += gridDim.x) {
        const int d = owner(tprefix, nsets, g);
        const BatchSet& S = sets[d];
        const int64_t t = g - tprefix[d];
        const int m = S.m;
        const int mp = (m + 7) & ~7;
        const int64_t r0 = t * 64;
        const float* src_v = S.vals + r0 * (int64_t)m;
        const uint16_t* src_i = S.idx + r0 * (int64_t)m;
        float* dv = vt + tile_base(S, t);
        uint16_t* di = it + tile_base(S, t);
        const int64_t tot = (int64_t)mp * 64;
        uint32_t mx = 0u;  // largest |value| (float bits compare as integers for non-negative floats)
        for (int64_t e = threadIdx.x; e < tot; e += 256) {
            const int u = (int)(e & 7);
            const int r = (int)((e >> 3) & 63);
            const int a = (int)(e >> 9) * 8 + u;
            const bool ok = r0 + r < S.n && a < m;
            const float v = ok ? src_v[(int64_t)r * m + a] : 0.0f;
            dv[e] = v;
            di[e] = ok ? src_i[(int64_t)r * m + a] : (uint16_t)0;
            mx = max(mx, __float_as_uint(fabsf(v)));
        }
        red[threadIdx.x] = mx;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
            __syncthreads();
        }
        if (threadIdx.x == 0) atomicMax(&vmax[d], red[0]);
        __syncthreads();
    }
}

// Fixed-point scale of a set's sums: a chunk sums at most cchunk values of
// magnitude below 2^ev (frexp of the set's largest |value|), so with F =
// 62 - ev - ceil(log2 cchunk) every chunk sum times 2^F stays below 2^62 and
// each value is rounded once, to 2^-F absolute (the sums themselves are then
// exact integers, independent of the order of the additions).
__device__ inline int batch_fx_exp(uint32_t vmax_bits, int64_t cchunk)
{
    int ev = 0;
    (void)frexpf(__uint_as_float(vmax_bits), &ev);
    const int cb = cchunk > 1 ? 64 - __clzll((unsigned long long)(cchunk - 1)) : 0;
    return 62 - ev - cb;
}

// prep: one workgroup per set; FP32 transposed centers, largest |center|, and
// (odd round counts) the second center buffer
__global__ __launch_bounds__(256) void k_batch_prep(const BatchSet* __restrict__ sets, int nsets,
                                                    float* __restrict__ ct, uint32_t* __restrict__ cmax0,
                                                    uint32_t* __restrict__ rcount, uint32_t* __restrict__ vmax,
                                                    int copy_to_b)
{
    __shared__ uint32_t red[256];
    const int d = blockIdx.x;
    if (d == 0 && threadIdx.x == 0) {
        rcount[0] = 0u;
        rcount[1] = 0u;  // the first round's queues
        rcount[2] = 0u;
    }
    if (threadIdx.x == 0) vmax[d] = 0u;  // the tiling that follows takes the set's largest |value|
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

// Assignment of one item (kBaThreads samples, one per thread).  The set's
// FP32 centers are staged through LDS a window of KW clusters at a time, for
// all p coordinates (row l holds the window's centers at coordinate l, its
// 16-byte quads permuted by an XOR with bits of l that the row's own bank
// offset does not use, so the lanes' reads at random rows spread over all
// eight 4-bank groups; unpadded, so the permutation works at every p, where a
// padded row no longer fits from p = 1024); each thread streams its sample's kept
// entries once per window, so every distance accumulates its terms in
// ascending coordinate order exactly as the single-plan kernel does.
template <int KW>
__device__ inline void batch_assign_item(const BatchSet& S, int set, int64_t j, const float* __restrict__ ct,
                                         float cmax, const float* __restrict__ vt, const uint16_t* __restrict__ it,
                                         float* __restrict__ lc, double* __restrict__ dist,
                                         int64_t* __restrict__ rlist, uint32_t* __restrict__ rcount)
{
    const int K = S.K, p = S.p, m = S.m;
    constexpr int NQ = KW / 4;                                  // quads per row
    constexpr int XS = KW == 32 ? 0 : (KW == 16 ? 1 : 2);      // row bits the row offset uses (32 / KW rows per bank sweep)
    const int64_t i = j * kBaThreads + threadIdx.x;
    const bool live = i < S.n;
    // this sample's entries in its tile: chunk c (eight entries) at element tb + 512 c
    const int64_t tl = i >> 6;
    const int64_t tb = tile_base(S, tl) + (i & 63) * 8;
    const uint4* ti = reinterpret_cast<const uint4*>(it + tb);  // 8 coordinates per chunk
    const float4* tv = reinterpret_cast<const float4*>(vt + tb);  // 2 x 4 values per chunk
    const int nch = (m + 7) >> 3;
    const float* cT = ct + S.ct_off;
    float best = INFINITY, second = INFINITY, sv = 0.0f;
    int bestk = 0;
    for (int kc = 0; kc < K; kc += KW) {
        __syncthreads();  // the previous window's reads are done
        for (int e = threadIdx.x; e < p * KW; e += kBaThreads) {
            const int r = e / KW, k = e - r * KW;
            const int pq = (k >> 2) ^ ((r >> XS) & (NQ - 1));
            lc[r * KW + pq * 4 + (k & 3)] = (kc + k < K) ? cT[(int64_t)r * K + kc + k] : 0.0f;
        }
        __syncthreads();
        float d[KW];
#pragma unroll
        for (int q = 0; q < KW; ++q) d[q] = 0.0f;
        if (live) {
            // a ring of four chunks in flight: chunk c + 4 is requested as soon
            // as chunk c has been used
            uint4 I[4];
            float4 A[4], Bv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (r < nch) {
                    I[r] = ti[(int64_t)r * 64];
                    A[r] = tv[(int64_t)r * 128];
                    Bv[r] = tv[(int64_t)r * 128 + 1];
                }
            }
            for (int c0 = 0; c0 < nch; c0 += 4) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = c0 + r;
                    if (c < nch) {
                        const uint32_t iw[4] = {I[r].x, I[r].y, I[r].z, I[r].w};
                        const float xw[8] = {A[r].x, A[r].y, A[r].z, A[r].w, Bv[r].x, Bv[r].y, Bv[r].z, Bv[r].w};
                        if (c + 4 < nch) {
                            // a chunk spans 64 lanes x 8 entries: 64 uint4 of coordinates, 128 float4 of values
                            I[r] = ti[(int64_t)(c + 4) * 64];
                            A[r] = tv[(int64_t)(c + 4) * 128];
                            Bv[r] = tv[(int64_t)(c + 4) * 128 + 1];
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            if (c * 8 + u < m) {
                                const int l = (int)((iw[u >> 1] >> ((u & 1) * 16)) & 0xFFFFu);
                                const float x = xw[u];
                                if (kc == 0) sv = fmaf(x, x, sv);
                                // byte offset of quad q of row l: (l NQ + ((l >> XS) mod NQ)) 16 XOR 16 q
                                const uint32_t rb = (uint32_t)(l * NQ + ((l >> XS) & (NQ - 1))) << 4;
                                const unsigned char* lcb = reinterpret_cast<const unsigned char*>(lc);
#pragma unroll
                                for (int q4 = 0; q4 < NQ; ++q4) {
                                    const float4 c = *reinterpret_cast<const float4*>(lcb + (rb ^ ((uint32_t)q4 << 4)));
                                    const float cc[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
                                    for (int r = 0; r < 4; ++r) {
                                        const float diff = x - cc[r];
                                        d[4 * q4 + r] = fmaf(diff, diff, d[4 * q4 + r]);
                                    }
                                }
                            }
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < KW; ++q) {
            if (kc + q < K) {
                if (d[q] < best) {
                    second = best;
                    best = d[q];
                    bestk = kc + q;
                } else if (d[q] < second) {
                    second = d[q];
                }
            }
        }
    }
    if (!live) return;
    S.assign[i] = bestk;
    dist[S.dist_off + i] = (double)best;
    if (K > 1) {
        // |d32 - d| <= u (8 (sum v^2 + sum mu^2) + 1.01 m d), u = 2^-24, per
        // candidate; two candidates, factor 2 of slack.  Closer calls are
        // decided in FP64 by k_batch_recheck.
        const float u = 5.9604645e-8f;
        const float mf = (float)m;
        const float bound = 2.0f * u * (16.0f * (sv + mf * cmax * cmax) + 1.01f * mf * (best + second));
        if (!(second - best > bound)) {
            const uint32_t slot = atomicAdd(rcount, 1u);
            rlist[slot] = ((int64_t)set << 40) | i;
        }
    }
}

// Work queues of the persistent assignment and accumulation launches: the
// workgroup takes the next item from a counter (items differ in cost by two
// orders of magnitude across sets, so a fixed round-robin leaves CUs idle).
// Counter words: rcount[0] recheck list length, rcount[1] assignment queue,
// rcount[2] accumulation queue; prep clears both, then each queue is cleared
// by a launch that runs after its last use and before its next (the
// assignment clears the accumulation queue, the update the assignment
// queue).
__device__ inline int64_t next_item(uint32_t* queue, int64_t* shared_item)
{
    __syncthreads();  // every thread has read the previous item
    if (threadIdx.x == 0) *shared_item = (int64_t)atomicAdd(queue, 1u);
    __syncthreads();
    return *shared_item;
}

__global__ __launch_bounds__(kBaThreads) void k_batch_assign(const BatchSet* __restrict__ sets, int nsets,
                                                             const int64_t* __restrict__ aprefix, int64_t nitems,
                                                             const float* __restrict__ ct,
                                                             const float* __restrict__ vtile,
                                                             const uint16_t* __restrict__ itile,
                                                             const uint32_t* __restrict__ cmax_cur,
                                                             uint32_t* __restrict__ cmax_next,
                                                             double* __restrict__ dist, int64_t* __restrict__ rlist,
                                                             uint32_t* __restrict__ rcount)
{
    extern __shared__ __align__(16) float lc[];  // kBaLdsFloats
    __shared__ int64_t item;
    if (blockIdx.x == 0 && threadIdx.x == 0) rcount[2] = 0u;  // the accumulation queue, for the launch after
    for (int64_t it = next_item(rcount + 1, &item); it < nitems; it = next_item(rcount + 1, &item)) {
        const int d = owner(aprefix, nsets, it);
        const BatchSet& S = sets[d];
        const int64_t j = it - aprefix[d];
        if (j == 0 && threadIdx.x == 0) cmax_next[d] = 0u;
        const float cmax = __uint_as_float(cmax_cur[d]);
        // cluster window of 8 / 16 / 32 (all p coordinates must fit in LDS):
        // per kept entry a pass reads 4 KW bytes of centers and about 24 bytes'
        // worth of sample data and bookkeeping, so take the fewest of
        // ceil(K / KW) (4 KW + 24) (K = 40: three windows of 16, not two of 32)
        int kw = 8;
        int best_cost = ((S.K + 7) / 8) * (4 * 8 + 24);
        for (int w = 16; w <= 32; w <<= 1) {
            if (S.p * w > kBaLdsFloats) break;
            const int cost = ((S.K + w - 1) / w) * (4 * w + 24);
            if (cost <= best_cost) {
                best_cost = cost;
                kw = w;
            }
        }
        switch (kw) {
            case 8: batch_assign_item<8>(S, d, j, ct, cmax, vtile, itile, lc, dist, rlist, rcount); break;
            case 16: batch_assign_item<16>(S, d, j, ct, cmax, vtile, itile, lc, dist, rlist, rcount); break;
            default: batch_assign_item<32>(S, d, j, ct, cmax, vtile, itile, lc, dist, rlist, rcount); break;
        }
    }
}

// FP64 decision for the samples the assignment flagged: one wave per sample,
// lanes over clusters; each lane sums its distance in the oracle's order
// (ascending kept coordinate, fma), ties go to the lowest k.
__global__ __launch_bounds__(256) void k_batch_recheck(const BatchSet* __restrict__ sets,
                                                       const int64_t* __restrict__ rlist,
                                                       const uint32_t* __restrict__ rcount,
                                                       double* __restrict__ dist, int dir)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * 4;
    const int64_t cnt = *rcount;
    for (int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); e < cnt; e += nw) {
        const int64_t code = rlist[e];
        const int d = (int)(code >> 40);
        const int64_t i = code & (((int64_t)1 << 40) - 1);
        const BatchSet& S = sets[d];
        const int m = S.m, p = S.p;
        const float* v = S.vals + i * (int64_t)m;
        const uint16_t* ix = S.idx + i * (int64_t)m;
        const double* cin = round_in(S, dir);
        double bd = INFINITY;
        int bk = 0x7fffffff;
        for (int k = lane; k < S.K; k += 64) {
            const double dk = batch_dist_f64(v, ix, m, cin + (int64_t)k * p);
            if (dk < bd) {  // k ascends within a lane, so ties keep the lower k
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
            S.assign[i] = bk;
            dist[S.dist_off + i] = bd;
        }
    }
}

constexpr int kAccSeg = 4096;  // samples listed at a time by k_batch_accum

__global__ __launch_bounds__(kBcThreads) void k_batch_accum(const BatchSet* __restrict__ sets, int nsets,
                                                            const int64_t* __restrict__ cprefix, int64_t nitems,
                                                            int64_t* __restrict__ psum, uint32_t* __restrict__ pcnt,
                                                            const uint32_t* __restrict__ vmax,
                                                            const double* __restrict__ dist,
                                                            double* __restrict__ pobj, uint32_t* __restrict__ qcount)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kBcThreads / 64];
    // 64-bit fixed-point sums: integer LDS atomics run at full rate, the FP32
    // ones do not
    unsigned long long* sums = reinterpret_cast<unsigned long long*>(smem);
    uint16_t* list = reinterpret_cast<uint16_t*>(smem + kBatchAccumLds);  // kAccSeg sample offsets
    __shared__ uint32_t lcount[1];
    __shared__ int64_t item;
    for (int64_t it = next_item(qcount + 2, &item); it < nitems; it = next_item(qcount + 2, &item)) {
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
        const int fx = batch_fx_exp(vmax[d], S.cchunk);
        __syncthreads();  // the previous item's LDS reads are done
        for (int e = threadIdx.x; e < ent; e += kBcThreads) {
            sums[e] = 0ull;
            cnts[e] = 0u;
        }
        __syncthreads();
        const int64_t s0 = chunk * S.cchunk;
        int64_t s1 = s0 + S.cchunk;
        if (s1 > S.n) s1 = S.n;
        if (grp == 0) {
            // the chunk's objective, in a fixed order
            double o = 0.0;
            for (int64_t i = s0 + threadIdx.x; i < s1; i += kBcThreads) o += dist[S.dist_off + i];
            for (int off = 32; off > 0; off >>= 1) o += __shfl_down(o, off, 64);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = o;
            __syncthreads();
            if (threadIdx.x == 0) {
                double t = 0.0;
                for (int w = 0; w < kBcThreads / 64; ++w) t += red[w];
                pobj[S.pchunk0 + chunk] = t;
            }
        }
        // The chunk's samples of this cluster group are listed (LDS slot
        // counter, any order), kAccSeg at a time; then the threads walk the
        // listed samples' entries as one flat range (consecutive threads on
        // consecutive entries of a sample: coalesced, and many loads in
        // flight per thread), adding each to its cluster's sums and counts.
        // Integer additions: the order does not change the result.
        for (int64_t g0 = s0; g0 < s1; g0 += kAccSeg) {
            if (threadIdx.x == 0) *lcount = 0u;
            __syncthreads();
            for (int64_t i = g0 + threadIdx.x; i < s1 && i < g0 + kAccSeg; i += kBcThreads) {
                const int c = S.assign[i];
                if (c >= k0 && c < k0 + kg) list[atomicAdd(lcount, 1u)] = (uint16_t)(i - g0);
            }
            __syncthreads();
            const int cnt = (int)*lcount;
            const int tot = cnt * m;
            const float inv_m = 1.0f / (float)m;
#pragma unroll 4
            for (int f = threadIdx.x; f < tot; f += kBcThreads) {
                int r = (int)((float)f * inv_m);
                while (r * m > f) --r;
                while ((r + 1) * m <= f) ++r;
                const int64_t i = g0 + list[r];
                const int64_t e = i * (int64_t)m + (f - r * m);
                const int cb = S.assign[i] - k0;
                const int l = (int)S.idx[e];
                const float x = S.vals[e];
                const long long q = __double2ll_rn(ldexp((double)x, fx));
                atomicAdd(&sums[cb * p + l], (unsigned long long)q);
                atomicAdd(&cnts[cb * p + l], 1u);
            }
            __syncthreads();  // the list is rebuilt for the next segment
        }
        __syncthreads();
        const int64_t KP = (int64_t)S.K * p;
        int64_t* ps = psum + S.part_off + chunk * KP + (int64_t)k0 * p;
        uint32_t* pc = pcnt + S.part_off + chunk * KP + (int64_t)k0 * p;
        for (int e = threadIdx.x; e < ent; e += kBcThreads) {
            ps[e] = (int64_t)sums[e];
            pc[e] = cnts[e];
        }
    }
}

__global__ __launch_bounds__(256) void k_batch_update(const BatchSet* __restrict__ sets, int nsets,
                                                      const int64_t* __restrict__ uprefix, int64_t nitems,
                                                      const int64_t* __restrict__ psum, const uint32_t* __restrict__ pcnt,
                                                      const uint32_t* __restrict__ vmax,
                                                      float* __restrict__ ct, uint32_t* __restrict__ cmax_next,
                                                      const double* __restrict__ pobj, uint32_t* __restrict__ rcount,
                                                      int dir, int round)
{
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int d = owner(uprefix, nsets, it);
        const BatchSet& S = sets[d];
        const int64_t j = it - uprefix[d];
        const int64_t KP = (int64_t)S.K * S.p;
        const int64_t e = j * 256 + threadIdx.x;
        if (j == 0 && threadIdx.x == 0) {
            double o = 0.0;
            for (int64_t a = 0; a < S.nacc; ++a) o += pobj[S.pchunk0 + a];
            S.objective[round] = o;
        }
        if (it == 0 && threadIdx.x == 0) {
            rcount[0] = 0u;  // for the next round: the recheck list and the assignment queue
            rcount[1] = 0u;
        }
        if (e >= KP) continue;
        double sum = 0.0;
        uint64_t cnt = 0;
        // eight chunks' loads in flight; the sum keeps chunk order
#pragma unroll 8
        for (int64_t c = 0; c < S.nacc; ++c) {
            sum += (double)psum[S.part_off + c * KP + e];
            cnt += pcnt[S.part_off + c * KP + e];
        }
        sum = ldexp(sum, -batch_fx_exp(vmax[d], S.cchunk));
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
                                hipFuncAttributeMaxDynamicSharedMemorySize, kBatchAccumLds + kAccSeg * 2);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_assign),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kBaLdsFloats * 4);
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

hipError_t launch_batch_tile(const BatchSet* sets, int nsets, const BatchTables& t, int64_t grid, hipStream_t s)
{
    if (t.ntiles <= 0) return hipSuccess;
    if (grid > t.ntiles) grid = t.ntiles;
    hipLaunchKernelGGL(k_batch_tile, dim3((unsigned)grid), dim3(256), 0, s, sets, nsets, t.tprefix, t.ntiles, t.vt,
                       t.it, t.vmax);
    return hipGetLastError();
}

hipError_t launch_batch_round_prep(const BatchSet* sets, int nsets, const BatchTables& t, int copy_to_b,
                                   hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_prep, dim3(nsets), dim3(256), 0, s, sets, nsets, t.ct, t.cmax, t.rcount, t.vmax,
                       copy_to_b);
    return hipGetLastError();
}

hipError_t launch_batch_round(const BatchSet* sets, int nsets, const BatchTables& t, const BatchTuning& tu,
                              int dir, int round, hipStream_t s)
{
    uint32_t* cm_cur = t.cmax + (size_t)(round & 1) * nsets;
    uint32_t* cm_next = t.cmax + (size_t)((round + 1) & 1) * nsets;
    if (t.naitems > 0) {
        int64_t grid = t.naitems < tu.assign_grid ? t.naitems : tu.assign_grid;
        hipLaunchKernelGGL(k_batch_assign, dim3((unsigned)grid), dim3(kBaThreads), (size_t)kBaLdsFloats * 4, s, sets,
                           nsets, t.aprefix, t.naitems, t.ct, t.vt, t.it, cm_cur, cm_next, t.dist, t.rlist, t.rcount);
        hipLaunchKernelGGL(k_batch_recheck, dim3((unsigned)t.recheck_grid), dim3(256), 0, s, sets, t.rlist, t.rcount,
                           t.dist, dir);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (t.ncitems > 0) {
        int64_t grid = t.ncitems < tu.accum_grid ? t.ncitems : tu.accum_grid;
        hipLaunchKernelGGL(k_batch_accum, dim3((unsigned)grid), dim3(kBcThreads), (size_t)(kBatchAccumLds + kAccSeg * 2), s, sets,
                           nsets, t.cprefix, t.ncitems, t.psum, t.pcnt, t.vmax, t.dist, t.pobj, t.rcount);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (t.nuitems > 0) {
        int64_t grid = t.nuitems < tu.update_grid ? t.nuitems : tu.update_grid;
        hipLaunchKernelGGL(k_batch_update, dim3((unsigned)grid), dim3(256), 0, s, sets, nsets, t.uprefix, t.nuitems,
                           t.psum, t.pcnt, t.vmax, t.ct, cm_next, t.pobj, t.rcount, dir, round);
    }
    return hipGetLastError();
}

}  // namespace pds
