// Covariance estimator of Sec. V on compressed data.
//
//   acc += sum_i w_i w_i^T          (Gram of the zero-filled compressed samples)
//   C_n  = p(p-1)/(m(m-1)) acc/n  with the diagonal scaled by p/(m n) instead,
//          which is C_emp_hat - (p-m)/(p-1) diag(C_emp_hat) written out.
//
// The Gram is a contraction over samples: G = W^T W with W the n x p
// zero-filled compressed matrix.  It runs as dense output tiles on the matrix
// cores: each workgroup owns one upper-triangle tile (rows A, cols B) and one
// range of samples; per chunk of S samples it scatters the chunk's entries that
// fall in A and B into zeroed coordinate-major LDS tiles (sample index
// contiguous, the K dimension of the MFMA), runs the MFMA K-loop, and clears
// the scattered slots again.  Per-sample offsets of each 256-coordinate block
// inside the sorted index row (computed once per call) let a workgroup read
// only the entries of its two blocks.
//
// Precision variants (all accumulate a sample range in FP32 on the matrix
// cores; ranges are summed in FP64 in a fixed order):
//   F32      : v_mfma_f32_32x32x2_f32 on the FP32 values.
//   BF16x3   : each value v = hi + lo (hi = bf16(v), lo = bf16(v - hi)); the
//              products hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16.
//   F64      : FP64 fused multiply-adds on the vector ALUs (64 x 64 tiles).
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kTileMfma = 256;   // output tile edge (MFMA variants)
constexpr int kTileF64 = 64;     // output tile edge (FP64 variant)
constexpr int kChunk = 32;       // samples per LDS chunk
constexpr int kBfStride = kChunk + 8;   // bf16 elements per LDS tile row (80 B: conflict-free 16 B reads)
constexpr int kF32Stride = kChunk + 1;  // floats per LDS tile row (odd: conflict-free column reads)
constexpr int kF64Stride = kChunk + 1;
constexpr int64_t kMaxSamplesPerSplit = 16384;  // FP32 accumulation length before the FP64 sum

// ---------------------------------------------------------------------------
// Block offsets: off[i][b] = number of kept indices of sample i below b * tw
// (b = 0..nb), found by binary search in the ascending index row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_block_offsets(const uint16_t* __restrict__ idx, int64_t n, int m, int tw,
                                                       int nb, uint32_t* __restrict__ off)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= n * (int64_t)(nb + 1)) return;
    const int64_t i = g / (nb + 1);
    const int b = (int)(g - i * (nb + 1));
    const uint16_t* row = idx + i * (int64_t)m;
    const uint32_t key = (uint32_t)b * (uint32_t)tw;
    int lo = 0, hi = m;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((uint32_t)row[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    off[g] = (uint32_t)lo;
}

// Decodes upper-triangle tile t (row-major over ta <= tb) of an nb x nb grid.
__device__ inline void decode_tile(int t, int nb, int& ta, int& tb)
{
    int a = 0;
    while (t >= nb - a) {
        t -= nb - a;
        ++a;
    }
    ta = a;
    tb = a + t;
}

// XCD-aware work-item order: the hardware deals workgroups round-robin to the
// 8 XCDs; item = (b mod 8) * per + b / 8 gives each XCD a contiguous run of
// items, and items are split-major, so the workgroups resident on one XCD walk
// the same samples together and share them in that XCD's L2.
__device__ inline int64_t xcd_item(int64_t b, int64_t total)
{
    const int64_t per = (total + 7) / 8;
    return (b % 8) * per + b / 8;
}

__device__ inline unsigned short bf16_bits_rn(float v)
{
    __bf16 h = (__bf16)v;
    return __builtin_bit_cast(unsigned short, h);
}
__device__ inline float bf16_bits_to_float(unsigned short b) { return __uint_as_float(((uint32_t)b) << 16); }

// ---------------------------------------------------------------------------
// MFMA Gram tile kernel.
// ---------------------------------------------------------------------------
template <bool SPLIT>
struct MfmaLds;

template <>
struct MfmaLds<true> {
    unsigned short ahi[kTileMfma * kBfStride];
    unsigned short alo[kTileMfma * kBfStride];
    unsigned short bhi[kTileMfma * kBfStride];
    unsigned short blo[kTileMfma * kBfStride];
};
template <>
struct MfmaLds<false> {
    float a[kTileMfma * kF32Stride];
    float b[kTileMfma * kF32Stride];
};

template <bool SPLIT>
__device__ inline void scatter_entry(MfmaLds<SPLIT>& L, bool to_b, int coord, int s, float v)
{
    if constexpr (SPLIT) {
        unsigned short h = bf16_bits_rn(v);
        unsigned short l = bf16_bits_rn(v - bf16_bits_to_float(h));
        unsigned short* hi = to_b ? L.bhi : L.ahi;
        unsigned short* lo = to_b ? L.blo : L.alo;
        hi[coord * kBfStride + s] = h;
        lo[coord * kBfStride + s] = l;
    } else {
        float* d = to_b ? L.b : L.a;
        d[coord * kF32Stride + s] = v;
    }
}

// Scatters (or clears, when clear=true) the chunk's entries of block A (and B
// when not a diagonal tile).  8 threads per sample, strided over its entries.
template <bool SPLIT>
__device__ inline void scatter_chunk(MfmaLds<SPLIT>& L, bool clear, const float* __restrict__ vals,
                                     const uint16_t* __restrict__ idx, const uint32_t* __restrict__ off, int m,
                                     int nb, int64_t n, int64_t s0, int ta, int tb, int tw)
{
    const int t = threadIdx.x;
    const int s = t >> 3;
    const int sub = t & 7;
    const int64_t i = s0 + s;
    if (i >= n) return;
    const uint32_t* o = off + i * (nb + 1);
    const float* v = vals + i * (int64_t)m;
    const uint16_t* ix = idx + i * (int64_t)m;
    {
        const int a0 = ta * tw;
        const uint32_t e0 = o[ta], e1 = o[ta + 1];
        for (uint32_t e = e0 + sub; e < e1; e += 8) scatter_entry<SPLIT>(L, false, (int)ix[e] - a0, s, clear ? 0.0f : v[e]);
    }
    if (ta != tb) {
        const int b0 = tb * tw;
        const uint32_t e0 = o[tb], e1 = o[tb + 1];
        for (uint32_t e = e0 + sub; e < e1; e += 8) scatter_entry<SPLIT>(L, true, (int)ix[e] - b0, s, clear ? 0.0f : v[e]);
    }
}

template <bool SPLIT>
__global__ __launch_bounds__(256) void k_gram_mfma(const float* __restrict__ vals, const uint16_t* __restrict__ idx,
                                                   const uint32_t* __restrict__ off, int m, int nb, int tw,
                                                   int64_t n, int ntiles, int nsplit, int64_t split_len,
                                                   float* __restrict__ part)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    MfmaLds<SPLIT>& L = *reinterpret_cast<MfmaLds<SPLIT>*>(smem_raw);

    const int64_t total = (int64_t)ntiles * nsplit;
    const int64_t item = xcd_item(blockIdx.x, total);
    if (item >= total) return;
    const int split = (int)(item / ntiles);
    const int tile = (int)(item % ntiles);
    int ta, tb;
    decode_tile(tile, nb, ta, tb);
    const bool diag = (ta == tb);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;

    // zero the LDS tiles once
    {
        uint4* z = reinterpret_cast<uint4*>(smem_raw);
        const int nz = (int)(sizeof(MfmaLds<SPLIT>) / 16);
        for (int e = tid; e < nz; e += 256) z[e] = make_uint4(0, 0, 0, 0);
    }

    f32x16 acc[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[rb][cb][r] = 0.0f;

    const int64_t sbeg = (int64_t)split * split_len;
    int64_t send = sbeg + split_len;
    if (send > n) send = n;

    for (int64_t s0 = sbeg; s0 < send; s0 += kChunk) {
        __syncthreads();
        scatter_chunk<SPLIT>(L, false, vals, idx, off, m, nb, n, s0, ta, tb, tw);
        __syncthreads();
        if constexpr (SPLIT) {
            const unsigned short* bh = diag ? L.ahi : L.bhi;
            const unsigned short* bl = diag ? L.alo : L.blo;
#pragma unroll
            for (int kk = 0; kk < kChunk; kk += 16) {
                const int koff = kk + 8 * (lane >> 5);
                bf16x8 ah[4], al[4], bhv[4], blv[4];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const int row = wr * 128 + rb * 32 + (lane & 31);
                    ah[rb] = *reinterpret_cast<const bf16x8*>(&L.ahi[row * kBfStride + koff]);
                    al[rb] = *reinterpret_cast<const bf16x8*>(&L.alo[row * kBfStride + koff]);
                }
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    const int col = wc * 128 + cb * 32 + (lane & 31);
                    bhv[cb] = *reinterpret_cast<const bf16x8*>(&bh[col * kBfStride + koff]);
                    blv[cb] = *reinterpret_cast<const bf16x8*>(&bl[col * kBfStride + koff]);
                }
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb) {
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[rb], bhv[cb], acc[rb][cb], 0, 0, 0);
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[rb], blv[cb], acc[rb][cb], 0, 0, 0);
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[rb], bhv[cb], acc[rb][cb], 0, 0, 0);
                    }
            }
        } else {
            const float* bsrc = diag ? L.a : L.b;
#pragma unroll 4
            for (int kk = 0; kk < kChunk; kk += 2) {
                const int k = kk + (lane >> 5);
                float av[4], bv[4];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) av[rb] = L.a[(wr * 128 + rb * 32 + (lane & 31)) * kF32Stride + k];
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) bv[cb] = bsrc[(wc * 128 + cb * 32 + (lane & 31)) * kF32Stride + k];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[rb], bv[cb], acc[rb][cb], 0, 0, 0);
            }
        }
        __syncthreads();
        scatter_chunk<SPLIT>(L, true, vals, idx, off, m, nb, n, s0, ta, tb, tw);
    }

    // write this range's FP32 tile: part[split][tile][i][j], i, j < tw
    float* out = part + ((int64_t)split * ntiles + tile) * (int64_t)tw * tw;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = wr * 128 + rb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int j = wc * 128 + cb * 32 + (lane & 31);
                if (i < tw && j < tw) out[(int64_t)i * tw + j] = acc[rb][cb][r];
            }
}

// ---------------------------------------------------------------------------
// FP64 Gram tile kernel (vector ALUs): 64 x 64 tiles, 4 x 4 outputs per thread.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gram_f64(const double* __restrict__ vals, const uint16_t* __restrict__ idx,
                                                  const uint32_t* __restrict__ off, int m, int nb, int tw, int64_t n,
                                                  int ntiles, int nsplit, int64_t split_len, double* __restrict__ part)
{
    __shared__ double A[kTileF64 * kF64Stride];
    __shared__ double B[kTileF64 * kF64Stride];
    const int64_t total = (int64_t)ntiles * nsplit;
    const int64_t item = xcd_item(blockIdx.x, total);
    if (item >= total) return;
    const int split = (int)(item / ntiles);
    const int tile = (int)(item % ntiles);
    int ta, tb;
    decode_tile(tile, nb, ta, tb);
    const bool diag = (ta == tb);
    const int tid = threadIdx.x;
    for (int e = tid; e < kTileF64 * kF64Stride; e += 256) {
        A[e] = 0.0;
        B[e] = 0.0;
    }
    const int ty = tid >> 4, tx = tid & 15;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;

    const int64_t sbeg = (int64_t)split * split_len;
    int64_t send = sbeg + split_len;
    if (send > n) send = n;
    const int s = tid >> 3, sub = tid & 7;
    for (int64_t s0 = sbeg; s0 < send; s0 += kChunk) {
        __syncthreads();
        const int64_t i = s0 + s;
        if (i < n) {
            const uint32_t* o = off + i * (nb + 1);
            const double* v = vals + i * (int64_t)m;
            const uint16_t* ix = idx + i * (int64_t)m;
            for (uint32_t e = o[ta] + sub; e < o[ta + 1]; e += 8) A[((int)ix[e] - ta * tw) * kF64Stride + s] = v[e];
            if (!diag)
                for (uint32_t e = o[tb] + sub; e < o[tb + 1]; e += 8) B[((int)ix[e] - tb * tw) * kF64Stride + s] = v[e];
        }
        __syncthreads();
        const double* Bs = diag ? A : B;
#pragma unroll 2
        for (int k = 0; k < kChunk; ++k) {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = A[(ty * 4 + a) * kF64Stride + k];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Bs[(tx * 4 + b) * kF64Stride + k];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
        }
        __syncthreads();
        if (i < n) {
            const uint32_t* o = off + i * (nb + 1);
            const uint16_t* ix = idx + i * (int64_t)m;
            for (uint32_t e = o[ta] + sub; e < o[ta + 1]; e += 8) A[((int)ix[e] - ta * tw) * kF64Stride + s] = 0.0;
            if (!diag)
                for (uint32_t e = o[tb] + sub; e < o[tb + 1]; e += 8) B[((int)ix[e] - tb * tw) * kF64Stride + s] = 0.0;
        }
    }
    double* out = part + ((int64_t)split * ntiles + tile) * (int64_t)tw * tw;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ty * 4 + a, j = tx * 4 + b;
            if (i < tw && j < tw) out[(int64_t)i * tw + j] = acc[a][b];
        }
}

// ---------------------------------------------------------------------------
// Split reduction (fixed order, FP64) into the caller's accumulator, and the
// finalize: scaling and mirroring of the upper tiles into a full matrix.
// ---------------------------------------------------------------------------
template <typename PT>
__global__ __launch_bounds__(256) void k_gram_reduce(const PT* __restrict__ part, int nsplit, int ntiles, int nb,
                                                     int tw, int p, double* __restrict__ acc)
{
    const int64_t per_tile = (int64_t)tw * tw;
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= per_tile * ntiles) return;
    const int tile = (int)(g / per_tile);
    const int64_t e = g - (int64_t)tile * per_tile;
    const int i = (int)(e / tw), j = (int)(e - (int64_t)(e / tw) * tw);
    int ta, tb;
    decode_tile(tile, nb, ta, tb);
    double sum = 0.0;
    for (int s = 0; s < nsplit; ++s) sum += (double)part[((int64_t)s * ntiles + tile) * per_tile + e];
    acc[(int64_t)(ta * tw + i) * p + (tb * tw + j)] += sum;
}

__global__ __launch_bounds__(256) void k_cov_finalize(const double* __restrict__ acc, int p, double sdiag,
                                                      double soff, double* __restrict__ C)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)p * p) return;
    const int j = (int)(g / p), k = (int)(g - (int64_t)(g / p) * p);
    // (min, max) lies in an upper tile; reading it for both (j, k) and (k, j)
    // makes the result exactly symmetric
    const int r = j < k ? j : k, c = j < k ? k : j;
    const double v = acc[(int64_t)r * p + c];
    C[g] = (j == k) ? sdiag * v : soff * v;
}

// ---------------------------------------------------------------------------
// Host side: tiling plan and launches.
// ---------------------------------------------------------------------------
struct GramPlan {
    int tw, nb, ntiles, nsplit;
    int64_t split_len;
    size_t off_bytes, part_bytes;
};

static GramPlan gram_plan(int prec, int p, int64_t n, const DeviceInfo& dev)
{
    GramPlan g;
    const int edge = (prec == 0) ? kTileF64 : kTileMfma;
    g.tw = p < edge ? p : edge;
    g.nb = p / g.tw;
    g.ntiles = g.nb * (g.nb + 1) / 2;
    const int64_t nchunks = (n + kChunk - 1) / kChunk;
    int64_t ns = (prec == 0) ? 1 : (n + kMaxSamplesPerSplit - 1) / kMaxSamplesPerSplit;
    const int64_t want = ((int64_t)dev.cus * 2 + g.ntiles - 1) / g.ntiles;  // enough workgroups to fill the chip
    if (ns < want) ns = want;
    if (ns > nchunks) ns = nchunks;
    if (ns < 1) ns = 1;
    const int64_t chunks_per = (nchunks + ns - 1) / ns;
    g.split_len = chunks_per * kChunk;
    g.nsplit = (int)((n + g.split_len - 1) / g.split_len);
    if (g.nsplit < 1) g.nsplit = 1;
    g.off_bytes = (((size_t)(n > 0 ? n : 0) * (g.nb + 1) * 4) + 255) & ~(size_t)255;
    const size_t pe = (prec == 0) ? sizeof(double) : sizeof(float);
    g.part_bytes = (size_t)g.nsplit * g.ntiles * (size_t)g.tw * g.tw * pe;
    return g;
}

size_t covariance_workspace(int prec, int p, int m, int64_t n, const DeviceInfo& dev)
{
    (void)m;
    if (n <= 0) return 0;
    GramPlan g = gram_plan(prec, p, n, dev);
    return g.off_bytes + g.part_bytes;
}

hipError_t launch_covariance_accumulate(int prec, int p, int m, const void* vals, const uint16_t* idx, int64_t n,
                                        double* acc, void* ws, size_t ws_bytes, const DeviceInfo& dev,
                                        hipStream_t s)
{
    (void)ws_bytes;
    if (n <= 0) return hipSuccess;
    GramPlan g = gram_plan(prec, p, n, dev);
    uint32_t* off = reinterpret_cast<uint32_t*>(ws);
    void* part = reinterpret_cast<unsigned char*>(ws) + g.off_bytes;
    {
        const int64_t threads = n * (int64_t)(g.nb + 1);
        hipLaunchKernelGGL(k_block_offsets, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, idx, n, m, g.tw,
                           g.nb, off);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t total = (int64_t)g.ntiles * g.nsplit;
    const int64_t grid = ((total + 7) / 8) * 8;
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram_mfma<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(MfmaLds<true>));
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram_mfma<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(MfmaLds<false>));
        attr_set = true;
    }
    if (prec == 0) {
        hipLaunchKernelGGL(k_gram_f64, dim3((unsigned)grid), dim3(256), 0, s, reinterpret_cast<const double*>(vals),
                           idx, off, m, g.nb, g.tw, n, g.ntiles, g.nsplit, g.split_len, reinterpret_cast<double*>(part));
    } else if (prec == 2) {
        hipLaunchKernelGGL(k_gram_mfma<true>, dim3((unsigned)grid), dim3(256), sizeof(MfmaLds<true>), s,
                           reinterpret_cast<const float*>(vals), idx, off, m, g.nb, g.tw, n, g.ntiles, g.nsplit,
                           g.split_len, reinterpret_cast<float*>(part));
    } else {
        hipLaunchKernelGGL(k_gram_mfma<false>, dim3((unsigned)grid), dim3(256), sizeof(MfmaLds<false>), s,
                           reinterpret_cast<const float*>(vals), idx, off, m, g.nb, g.tw, n, g.ntiles, g.nsplit,
                           g.split_len, reinterpret_cast<float*>(part));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nred = (int64_t)g.ntiles * g.tw * g.tw;
    if (prec == 0)
        hipLaunchKernelGGL(k_gram_reduce<double>, dim3((unsigned)((nred + 255) / 256)), dim3(256), 0, s,
                           reinterpret_cast<const double*>(part), g.nsplit, g.ntiles, g.nb, g.tw, p, acc);
    else
        hipLaunchKernelGGL(k_gram_reduce<float>, dim3((unsigned)((nred + 255) / 256)), dim3(256), 0, s,
                           reinterpret_cast<const float*>(part), g.nsplit, g.ntiles, g.nb, g.tw, p, acc);
    return hipGetLastError();
}

hipError_t launch_covariance_finalize(int prec, int p, int m, int64_t n_total, const double* acc, double* C,
                                      hipStream_t s)
{
    (void)prec;
    const double sdiag = (double)p / ((double)m * (double)n_total);
    const double soff = ((double)p * (double)(p - 1)) / ((double)m * (double)(m - 1) * (double)n_total);
    const int64_t tot = (int64_t)p * p;
    hipLaunchKernelGGL(k_cov_finalize, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, acc, p, sdiag, soff,
                       C);
    return hipGetLastError();
}

}  // namespace pds
