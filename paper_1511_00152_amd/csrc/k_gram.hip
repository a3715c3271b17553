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
// MFMA Gram tile kernel.  A workgroup owns a TR x TC output tile (rows from a
// 256-coordinate block, columns from a 128-coordinate block) and one sample
// range.  Two workgroups fit on a CU (62 KB LDS, 128 accumulator registers
// per wave), so one workgroup's scatter and barriers overlap the other's
// matrix-core work.  Each wave computes a 128 x 64 sub-tile as 4 x 2 blocks of
// 32 x 32.  When the column block lies inside the row block ("inner" tiles,
// those holding the diagonal) the column operand is read from the row tiles.
// ---------------------------------------------------------------------------
constexpr int kTR = 256;  // tile rows (MFMA variants)
constexpr int kTC = 128;  // tile columns (MFMA variants)

template <bool SPLIT>
struct MfmaLds;

template <>
struct MfmaLds<true> {
    unsigned short ahi[kTR * kBfStride];
    unsigned short alo[kTR * kBfStride];
    unsigned short bhi[kTC * kBfStride];
    unsigned short blo[kTC * kBfStride];
    double diag[kTC];  // exact sum of squares per column coordinate (inner tiles)
};
template <>
struct MfmaLds<false> {
    float a[kTR * kF32Stride];
    float b[kTC * kF32Stride];
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

// Tile geometry shared by the host plan and the kernels.
struct TileGeom {
    int p, tr, tc, ratio, nbr, nbc, ntiles;
};

__host__ __device__ inline TileGeom make_geom(int p, int tr_max, int tc_max)
{
    TileGeom g;
    g.p = p;
    g.tr = p < tr_max ? p : tr_max;
    g.tc = p < tc_max ? p : tc_max;
    g.ratio = g.tr / g.tc;
    g.nbr = p / g.tr;
    g.nbc = p / g.tc;
    g.ntiles = 0;
    for (int a = 0; a < g.nbr; ++a) g.ntiles += g.nbc - a * g.ratio;
    return g;
}

// Tile t (row-major over row block a, column blocks b >= a * ratio).
__device__ inline void decode_rect_tile(int t, const TileGeom& g, int& a, int& b)
{
    int r = 0;
    while (t >= g.nbc - r * g.ratio) {
        t -= g.nbc - r * g.ratio;
        ++r;
    }
    a = r;
    b = r * g.ratio + t;
}

// Per-thread share of one chunk: thread t serves sample slot s = t / 8 and
// entries e0 + (t % 8) + 8 k of the row block (k < KA) and of the column block
// (k < KB).  The host picks KA, KB so that a sample rarely has more entries in
// a block; the rare extra entries are read and scattered directly.
struct ChunkOffsets {
    uint32_t a0, a1, b0, b1;
    bool ok;  // the sample belongs to this range (else the offsets are not used)
};

template <int KA, int KB>
struct ChunkEntries {
    uint16_t ia[KA], ib[KB];
    float va[KA], vb[KB];
    uint32_t valid;  // bit k: row entry k, bit 16 + k: column entry k
};

// The load address is always a valid row, so no branch guards it.
__device__ inline ChunkOffsets load_offsets(const uint32_t* __restrict__ off, int nbo, int64_t send, int64_t i,
                                            int64_t i_safe, int oa0, int oa1, int ob0)
{
    const uint32_t* r = off + (i < send ? i : i_safe) * (nbo + 1);
    ChunkOffsets o;
    o.a0 = r[oa0];
    o.a1 = r[oa1];
    o.b0 = r[ob0];
    o.b1 = r[ob0 + 1];
    o.ok = i < send;
    return o;
}

// Raw loaded words; the arithmetic on them waits until the scatter so that
// the loads stay in flight while the matrix cores run.
template <int KA, int KB>
__device__ inline ChunkEntries<KA, KB> load_entries(const float* __restrict__ vals, const uint16_t* __restrict__ idx,
                                                    int m, int64_t send, int64_t i, int64_t i_safe,
                                                    const ChunkOffsets& o, int sub, bool inner)
{
    ChunkEntries<KA, KB> c;
    const int64_t row = (i < send ? i : i_safe) * (int64_t)m;
    const float* v = vals + row;
    const uint16_t* ix = idx + row;
    c.valid = 0;
#pragma unroll
    for (int k = 0; k < KA; ++k) {
        const uint32_t e = o.a0 + sub + 8 * k;
        const uint32_t se = e < (uint32_t)m ? e : (uint32_t)(m - 1);
        c.ia[k] = ix[se];
        c.va[k] = v[se];
        c.valid |= (uint32_t)(o.ok && e < o.a1) << k;
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const uint32_t e = o.b0 + sub + 8 * k;
        const uint32_t se = e < (uint32_t)m ? e : (uint32_t)(m - 1);
        c.ib[k] = ix[se];
        c.vb[k] = v[se];
        c.valid |= (uint32_t)(o.ok && !inner && e < o.b1) << (16 + k);
    }
    return c;
}

// The split products hi*hi + hi*lo + lo*hi drop lo*lo, which biases every
// diagonal entry low by the mean of lo^2 (about 2.5e-6 relative); inner tiles
// therefore also sum the squares v*v of their column block's entries exactly
// in FP64 and those sums replace the matrix-core diagonal.
template <bool SPLIT>
__device__ inline void add_square(MfmaLds<SPLIT>& L, int coord_a, int boff, int tc, float v)
{
    if constexpr (SPLIT) {
        const int c = coord_a - boff;
        if (c >= 0 && c < tc) atomicAdd(&L.diag[c], (double)v * (double)v);
    }
}

template <bool SPLIT, int KA, int KB>
__device__ inline void put_entries(MfmaLds<SPLIT>& L, const ChunkEntries<KA, KB>& c, int s, bool clear, bool inner,
                                   int a_base, int b_base, int boff, int tc)
{
#pragma unroll
    for (int k = 0; k < KA; ++k) {
        if ((c.valid >> k) & 1u) {
            const int coord = (int)c.ia[k] - a_base;
            scatter_entry<SPLIT>(L, false, coord, s, clear ? 0.0f : c.va[k]);
            if (inner && !clear) add_square<SPLIT>(L, coord, boff, tc, c.va[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k)
        if ((c.valid >> (16 + k)) & 1u) scatter_entry<SPLIT>(L, true, (int)c.ib[k] - b_base, s, clear ? 0.0f : c.vb[k]);
}

// entries past the register share of a sample (rare): direct loads
template <bool SPLIT>
__device__ inline void put_overflow(MfmaLds<SPLIT>& L, const float* __restrict__ vals, const uint16_t* __restrict__ idx,
                                    int m, int64_t i, const ChunkOffsets& o, int s, int sub, int a_base, int b_base,
                                    bool inner, int boff, int tc, int ka, int kb, bool clear)
{
    if (!o.ok) return;
    const float* v = vals + i * (int64_t)m;
    const uint16_t* ix = idx + i * (int64_t)m;
    for (uint32_t e = o.a0 + 8 * ka + sub; e < o.a1; e += 8) {
        const int coord = (int)ix[e] - a_base;
        scatter_entry<SPLIT>(L, false, coord, s, clear ? 0.0f : v[e]);
        if (inner && !clear) add_square<SPLIT>(L, coord, boff, tc, v[e]);
    }
    if (!inner)
        for (uint32_t e = o.b0 + 8 * kb + sub; e < o.b1; e += 8)
            scatter_entry<SPLIT>(L, true, (int)ix[e] - b_base, s, clear ? 0.0f : v[e]);
}

template <bool SPLIT, int KA, int KB>
__global__ __launch_bounds__(256, 2) void k_gram_mfma(const float* __restrict__ vals, const uint16_t* __restrict__ idx,
                                                      const uint32_t* __restrict__ off, int m, TileGeom g, int64_t n,
                                                      int nsplit, int64_t split_len, float* __restrict__ part,
                                                      double* __restrict__ pdiag)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    MfmaLds<SPLIT>& L = *reinterpret_cast<MfmaLds<SPLIT>*>(smem_raw);

    const int64_t total = (int64_t)g.ntiles * nsplit;
    const int64_t item = xcd_item(blockIdx.x, total);
    if (item >= total) return;
    const int split = (int)(item / g.ntiles);
    const int tile = (int)(item % g.ntiles);
    int ta, tb;
    decode_rect_tile(tile, g, ta, tb);
    const int a_base = ta * g.tr, b_base = tb * g.tc;
    const bool inner = tb < (ta + 1) * g.ratio;  // column block inside the row block
    const int boff = b_base - a_base;            // row of the column block inside the row tile (inner)
    const int nbo = g.nbc;                       // offsets are per column block
    const int oa0 = ta * g.ratio, oa1 = (ta + 1) * g.ratio, ob0 = tb;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int s = tid >> 3, sub = tid & 7;

    {
        uint4* z = reinterpret_cast<uint4*>(smem_raw);
        const int nz = (int)(sizeof(MfmaLds<SPLIT>) / 16);
        for (int e = tid; e < nz; e += 256) z[e] = make_uint4(0, 0, 0, 0);
    }

    f32x16 acc[4][2];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[rb][cb][r] = 0.0f;

    const int64_t sbeg = (int64_t)split * split_len;
    int64_t send = sbeg + split_len;
    if (send > n) send = n;
    const int64_t i_safe = sbeg;

    // pipeline: offsets two chunks ahead, entries one chunk ahead
    ChunkOffsets o_cur = load_offsets(off, nbo, send, sbeg + s, i_safe, oa0, oa1, ob0);
    ChunkEntries<KA, KB> e_cur = load_entries<KA, KB>(vals, idx, m, send, sbeg + s, i_safe, o_cur, sub, inner);
    ChunkOffsets o_next = load_offsets(off, nbo, send, sbeg + kChunk + s, i_safe, oa0, oa1, ob0);
    ChunkEntries<KA, KB> e_prev;
    e_prev.valid = 0;
    ChunkOffsets o_prev{0, 0, 0, 0, false};
    int64_t i_prev = send;

    // column operand rows: the column tile, or the row tile at offset boff
    const unsigned short* bh_src = nullptr;
    const unsigned short* bl_src = nullptr;
    const float* bf_src = nullptr;
    int brow0;
    if constexpr (SPLIT) {
        bh_src = inner ? L.ahi : L.bhi;
        bl_src = inner ? L.alo : L.blo;
    } else {
        bf_src = inner ? L.a : L.b;
    }
    brow0 = (inner ? boff : 0) + wc * 64;

    for (int64_t s0 = sbeg; s0 < send; s0 += kChunk) {
        const int64_t i_cur = s0 + s;
        __syncthreads();
        // clear the previous chunk's slots, then scatter this chunk (the
        // writers of a sample slot are one wave, so their LDS writes stay ordered)
        put_entries<SPLIT, KA, KB>(L, e_prev, s, true, inner, a_base, b_base, boff, g.tc);
        put_overflow<SPLIT>(L, vals, idx, m, i_prev, o_prev, s, sub, a_base, b_base, inner, boff, g.tc, KA, KB, true);
        put_entries<SPLIT, KA, KB>(L, e_cur, s, false, inner, a_base, b_base, boff, g.tc);
        put_overflow<SPLIT>(L, vals, idx, m, i_cur, o_cur, s, sub, a_base, b_base, inner, boff, g.tc, KA, KB, false);
        __syncthreads();
        e_prev = e_cur;
        o_prev = o_cur;
        i_prev = i_cur;
        // loads for the next chunks fly while this chunk runs on the matrix cores
        e_cur = load_entries<KA, KB>(vals, idx, m, send, s0 + kChunk + s, i_safe, o_next, sub, inner);
        o_cur = o_next;
        o_next = load_offsets(off, nbo, send, s0 + 2 * kChunk + s, i_safe, oa0, oa1, ob0);
        // keep the scheduler from sinking those loads (or their address math)
        // into the matrix-core block, where their waits would stall it
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (SPLIT) {
#pragma unroll
            for (int kk = 0; kk < kChunk; kk += 16) {
                const int koff = kk + 8 * (lane >> 5);
                bf16x8 ah[4], al[4], bhv[2], blv[2];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const int row = wr * 128 + rb * 32 + (lane & 31);
                    ah[rb] = *reinterpret_cast<const bf16x8*>(&L.ahi[row * kBfStride + koff]);
                    al[rb] = *reinterpret_cast<const bf16x8*>(&L.alo[row * kBfStride + koff]);
                }
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    const int col = brow0 + cb * 32 + (lane & 31);
                    bhv[cb] = *reinterpret_cast<const bf16x8*>(&bh_src[col * kBfStride + koff]);
                    blv[cb] = *reinterpret_cast<const bf16x8*>(&bl_src[col * kBfStride + koff]);
                }
                // product-outer order: consecutive MFMAs write different accumulators
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[rb], bhv[cb], acc[rb][cb], 0, 0, 0);
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[rb], blv[cb], acc[rb][cb], 0, 0, 0);
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[rb], bhv[cb], acc[rb][cb], 0, 0, 0);
            }
        } else {
#pragma unroll 4
            for (int kk = 0; kk < kChunk; kk += 2) {
                const int k = kk + (lane >> 5);
                float av[4], bv[2];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) av[rb] = L.a[(wr * 128 + rb * 32 + (lane & 31)) * kF32Stride + k];
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) bv[cb] = bf_src[(brow0 + cb * 32 + (lane & 31)) * kF32Stride + k];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[rb], bv[cb], acc[rb][cb], 0, 0, 0);
            }
        }
    }

    // write this range's FP32 tile: part[split][tile][i][j], i < tr, j < tc
    float* out = part + ((int64_t)split * g.ntiles + tile) * (int64_t)g.tr * g.tc;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = wr * 128 + rb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int j = wc * 64 + cb * 32 + (lane & 31);
                if (i < g.tr && j < g.tc && !(SPLIT && inner && i == j + boff))
                    out[(int64_t)i * g.tc + j] = acc[rb][cb][r];
            }
    if constexpr (SPLIT) {
        if (inner) {
            __syncthreads();
            double* dout = pdiag + ((int64_t)split * g.ntiles + tile) * g.tc;
            for (int c = tid; c < g.tc; c += 256) {
                dout[c] = L.diag[c];
                out[(int64_t)(c + boff) * g.tc + c] = 0.0f;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 Gram tile kernel (vector ALUs): 64 x 64 tiles, 4 x 4 outputs per thread.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gram_f64(const double* __restrict__ vals, const uint16_t* __restrict__ idx,
                                                  const uint32_t* __restrict__ off, int m, TileGeom g, int64_t n,
                                                  int nsplit, int64_t split_len, double* __restrict__ part)
{
    __shared__ double A[kTileF64 * kF64Stride];
    __shared__ double B[kTileF64 * kF64Stride];
    const int64_t total = (int64_t)g.ntiles * nsplit;
    const int64_t item = xcd_item(blockIdx.x, total);
    if (item >= total) return;
    const int split = (int)(item / g.ntiles);
    const int tile = (int)(item % g.ntiles);
    int ta, tb;
    decode_rect_tile(tile, g, ta, tb);
    const bool diag = (ta == tb);
    const int tw = g.tr;
    const int nb = g.nbc;
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
        if (i < send) {
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
        if (i < send) {
            const uint32_t* o = off + i * (nb + 1);
            const uint16_t* ix = idx + i * (int64_t)m;
            for (uint32_t e = o[ta] + sub; e < o[ta + 1]; e += 8) A[((int)ix[e] - ta * tw) * kF64Stride + s] = 0.0;
            if (!diag)
                for (uint32_t e = o[tb] + sub; e < o[tb + 1]; e += 8) B[((int)ix[e] - tb * tw) * kF64Stride + s] = 0.0;
        }
    }
    double* out = part + ((int64_t)split * g.ntiles + tile) * (int64_t)tw * tw;
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
__global__ __launch_bounds__(256) void k_gram_reduce(const PT* __restrict__ part, const double* __restrict__ pdiag,
                                                     int nsplit, TileGeom g, double* __restrict__ acc)
{
    const int64_t per_tile = (int64_t)g.tr * g.tc;
    const int64_t gi = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gi >= per_tile * g.ntiles) return;
    const int tile = (int)(gi / per_tile);
    const int64_t e = gi - (int64_t)tile * per_tile;
    const int i = (int)(e / g.tc), j = (int)(e - (int64_t)(e / g.tc) * g.tc);
    int ta, tb;
    decode_rect_tile(tile, g, ta, tb);
    double sum = 0.0;
    for (int s = 0; s < nsplit; ++s) sum += (double)part[((int64_t)s * g.ntiles + tile) * per_tile + e];
    const int boff = tb * g.tc - ta * g.tr;
    if (pdiag && tb < (ta + 1) * g.ratio && i == j + boff)
        for (int s = 0; s < nsplit; ++s) sum += pdiag[((int64_t)s * g.ntiles + tile) * g.tc + j];
    acc[(int64_t)(ta * g.tr + i) * g.p + (tb * g.tc + j)] += sum;
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
    TileGeom geom;
    int nsplit, ka, kb;
    int64_t split_len;
    size_t off_bytes, part_bytes, diag_bytes;
};

// Register slots per thread for a block of w coordinates: the kept count of a
// sample in the block is hypergeometric (m draws, w of p marked); 8 slots per
// thread-group step, enough for the mean plus four standard deviations.
static int slots_for(int p, int m, int w)
{
    const double mu = (double)m * w / p;
    const double var = (p > 1) ? (double)m * ((double)w / p) * (1.0 - (double)w / p) * (double)(p - m) / (p - 1) : 0.0;
    int k = (int)((mu + 4.0 * sqrt(var) + 7.999) / 8.0);
    k = (k + 1) & ~1;
    if (k < 2) k = 2;
    if (k > 8) k = 8;
    return k;
}

static GramPlan gram_plan(int prec, int p, int m, int64_t n, const DeviceInfo& dev)
{
    GramPlan g;
    g.geom = (prec == 0) ? make_geom(p, kTileF64, kTileF64) : make_geom(p, kTR, kTC);
    g.ka = slots_for(p, m, g.geom.tr);
    g.kb = slots_for(p, m, g.geom.tc);
    if (g.kb > g.ka) g.kb = g.ka;
    const int64_t nchunks = (n + kChunk - 1) / kChunk;
    int64_t ns = (prec == 0) ? 1 : (n + kMaxSamplesPerSplit - 1) / kMaxSamplesPerSplit;
    const int64_t want = ((int64_t)dev.cus * 4 + g.geom.ntiles - 1) / g.geom.ntiles;  // enough workgroups
    if (ns < want) ns = want;
    if (ns > nchunks) ns = nchunks;
    if (ns < 1) ns = 1;
    const int64_t chunks_per = (nchunks + ns - 1) / ns;
    g.split_len = chunks_per * kChunk;
    g.nsplit = (int)((n + g.split_len - 1) / g.split_len);
    if (g.nsplit < 1) g.nsplit = 1;
    g.off_bytes = (((size_t)(n > 0 ? n : 0) * (g.geom.nbc + 1) * 4) + 255) & ~(size_t)255;
    const size_t pe = (prec == 0) ? sizeof(double) : sizeof(float);
    g.part_bytes = (((size_t)g.nsplit * g.geom.ntiles * (size_t)g.geom.tr * g.geom.tc * pe) + 255) & ~(size_t)255;
    g.diag_bytes = (prec == 2) ? (size_t)g.nsplit * g.geom.ntiles * (size_t)g.geom.tc * sizeof(double) : 0;
    return g;
}

size_t covariance_workspace(int prec, int p, int m, int64_t n, const DeviceInfo& dev)
{
    if (n <= 0) return 0;
    GramPlan g = gram_plan(prec, p, m, n, dev);
    return g.off_bytes + g.part_bytes + g.diag_bytes;
}

template <bool SPLIT, int KA, int KB>
static void launch_mfma_kernel(const GramPlan& g, int64_t grid, const float* vals, const uint16_t* idx,
                               const uint32_t* off, int m, int64_t n, float* part, double* pdiag, hipStream_t s)
{
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram_mfma<SPLIT, KA, KB>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(MfmaLds<SPLIT>));
        attr_set = true;
    }
    {
        ProfScope ps_(SPLIT ? "gram_bf16x3" : "gram_f32", s);
        hipLaunchKernelGGL((k_gram_mfma<SPLIT, KA, KB>), dim3((unsigned)grid), dim3(256), sizeof(MfmaLds<SPLIT>), s,
                           vals, idx, off, m, g.geom, n, g.nsplit, g.split_len, part, pdiag);
    }
}

template <bool SPLIT>
static void dispatch_mfma(const GramPlan& g, int64_t grid, const float* vals, const uint16_t* idx,
                          const uint32_t* off, int m, int64_t n, float* part, double* pdiag, hipStream_t s)
{
#define PDS_GRAM_CASE(A, B)                                                                 \
    if (g.ka == A && g.kb == B) {                                                           \
        launch_mfma_kernel<SPLIT, A, B>(g, grid, vals, idx, off, m, n, part, pdiag, s); \
        return;                                                                             \
    }
    PDS_GRAM_CASE(2, 2)
    PDS_GRAM_CASE(4, 2)
    PDS_GRAM_CASE(4, 4)
    PDS_GRAM_CASE(6, 2)
    PDS_GRAM_CASE(6, 4)
    PDS_GRAM_CASE(6, 6)
    PDS_GRAM_CASE(8, 2)
    PDS_GRAM_CASE(8, 4)
    PDS_GRAM_CASE(8, 6)
    PDS_GRAM_CASE(8, 8)
#undef PDS_GRAM_CASE
}

hipError_t launch_covariance_accumulate(int prec, int p, int m, const void* vals, const uint16_t* idx, int64_t n,
                                        double* acc, void* ws, size_t ws_bytes, const DeviceInfo& dev,
                                        hipStream_t s)
{
    (void)ws_bytes;
    if (n <= 0) return hipSuccess;
    GramPlan g = gram_plan(prec, p, m, n, dev);
    uint32_t* off = reinterpret_cast<uint32_t*>(ws);
    void* part = reinterpret_cast<unsigned char*>(ws) + g.off_bytes;
    double* pdiag = (prec == 2)
                        ? reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(ws) + g.off_bytes + g.part_bytes)
                        : nullptr;
    {
        const int64_t threads = n * (int64_t)(g.geom.nbc + 1);
        ProfScope ps_("block_offsets", s);
        hipLaunchKernelGGL(k_block_offsets, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, idx, n, m,
                           g.geom.tc, g.geom.nbc, off);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t total = (int64_t)g.geom.ntiles * g.nsplit;
    const int64_t grid = ((total + 7) / 8) * 8;
    if (prec == 0) {
        ProfScope ps_("gram_f64", s);
        hipLaunchKernelGGL(k_gram_f64, dim3((unsigned)grid), dim3(256), 0, s, reinterpret_cast<const double*>(vals),
                           idx, off, m, g.geom, n, g.nsplit, g.split_len, reinterpret_cast<double*>(part));
    } else if (prec == 2) {
        dispatch_mfma<true>(g, grid, reinterpret_cast<const float*>(vals), idx, off, m, n,
                            reinterpret_cast<float*>(part), pdiag, s);
    } else {
        dispatch_mfma<false>(g, grid, reinterpret_cast<const float*>(vals), idx, off, m, n,
                             reinterpret_cast<float*>(part), nullptr, s);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nred = (int64_t)g.geom.ntiles * g.geom.tr * g.geom.tc;
    {
        ProfScope ps_("gram_reduce", s);
        if (prec == 0)
            hipLaunchKernelGGL(k_gram_reduce<double>, dim3((unsigned)((nred + 255) / 256)), dim3(256), 0, s,
                               reinterpret_cast<const double*>(part), (const double*)nullptr, g.nsplit, g.geom, acc);
        else
            hipLaunchKernelGGL(k_gram_reduce<float>, dim3((unsigned)((nred + 255) / 256)), dim3(256), 0, s,
                               reinterpret_cast<const float*>(part), pdiag, g.nsplit, g.geom, acc);
    }
    return hipGetLastError();
}

hipError_t launch_covariance_finalize(int prec, int p, int m, int64_t n_total, const double* acc, double* C,
                                      hipStream_t s)
{
    (void)prec;
    const double sdiag = (double)p / ((double)m * (double)n_total);
    const double soff = ((double)p * (double)(p - 1)) / ((double)m * (double)(m - 1) * (double)n_total);
    const int64_t tot = (int64_t)p * p;
    {
        ProfScope ps_("cov_finalize", s);
        hipLaunchKernelGGL(k_cov_finalize, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, acc, p, sdiag, soff,
                       C);
    }
    return hipGetLastError();
}

}  // namespace pds
