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
constexpr int64_t kMaxSamplesPerSplit = 32768;  // FP32 accumulation length before the FP64 sum

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
    double diag[kTC];  // FP64 sum of squares per column coordinate (inner tiles)
    __device__ double* diag_ptr() { return diag; }
};
template <>
struct MfmaLds<false> {
    float a[kTR * kF32Stride];
    float b[kTC * kF32Stride];
    __device__ double* diag_ptr() { return nullptr; }
};

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

// ---------------------------------------------------------------------------
// Chunk packing (matrix-core variants).  Chunk c holds samples 32c .. 32c+31;
// its n_c m entries are rewritten, in the chunk's own 32 m slots, ordered by
// column block (tc coordinates), then sample, then coordinate:
//   P[c][q]  the stored value: bf16 hi | bf16 lo << 16 (split), or the FP32 bits
//   OA[c][q] LDS byte offset of the entry in a row tile: coordinate-in-tile
//            * row bytes + slot * element bytes.  Its offset in a column tile
//            (tc rows) is OA mod (tc * row bytes), taken by the tile kernel.
//   BS[c][b] first q of block b, b = 0 .. nbc (BS[c][nbc] = n_c m)
// A tile's entries of one chunk are then one contiguous run: the tile kernel
// reads them coalesced, balanced over its threads, and scatters each with one
// offset extraction, and the bf16 split is done once per entry instead of once
// per tile.
// ---------------------------------------------------------------------------
__device__ inline uint32_t split_bits(float v)
{
    const unsigned short h = bf16_bits_rn(v);
    const unsigned short l = bf16_bits_rn(v - bf16_bits_to_float(h));
    return (uint32_t)h | ((uint32_t)l << 16);
}

template <int NT>
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* wsum)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t base = 0;
    for (int w = 0; w < wave; ++w) base += wsum[w];
    return base + incl - v;
}

constexpr int kPackStageBytes = 32768;  // chunk index rows staged in LDS up to this size

// STAGE: the chunk's index rows (at most kPackStageBytes, 16-byte aligned
// source) are copied to LDS with 16-byte loads first; otherwise read in place.
// eb: bytes of one sample slot in OA.  The sparse Gram packs with tr = tc,
// rowbytes = 1 and eb = 128, so that OA = (sample << 7) | coordinate-in-block,
// and also takes SS[c][b][s] (start of sample s inside block b's run, uint16)
// and CM[c] (the chunk's largest |value|, FP32 bits); both are skipped when
// NULL.  VREG > 0 (chunks of at most NT VREG entries): each thread's values
// are requested into registers before the index tables are built, so their
// loads fly during the table and scan phases instead of stalling the writes.
// NT threads per chunk: 512 for large chunks, so that more waves per CU keep
// loads and stores in flight while others build their tables.
template <bool STAGE, int VREG, int NT>
__global__ __launch_bounds__(NT) void k_gram_pack(const float* __restrict__ vals, const uint16_t* __restrict__ idx,
                                                   int64_t n, int m, int tr, int tc, int nbc, int rowbytes, int eb,
                                                   int split, uint32_t* __restrict__ P, uint16_t* __restrict__ OA,
                                                   uint32_t* __restrict__ BS, uint16_t* __restrict__ SS,
                                                   uint32_t* __restrict__ CM)
{
    extern __shared__ __align__(16) uint32_t pk_sh[];
    const int nb1 = nbc + 1;
    uint32_t* off = pk_sh;              // [32][nb1]: first entry of block b in the sample's row
    uint32_t* seg = pk_sh + 32 * nb1;   // [nbc][32]: chunk position of segment (b, s) minus off[s][b]
    uint32_t* wsum = seg + 32 * nbc;    // NT / 64 wave totals
    const int64_t c = blockIdx.x;
    const int64_t i0 = c * kChunk;
    const int ns = (int)((n - i0) < kChunk ? (n - i0) : kChunk);
    const int tid = threadIdx.x;
    const int sh_c = __builtin_ctz((unsigned)tc);

    const int tot = ns * m;
    const float inv_m = 1.0f / (float)m;
    const float* cval = vals + i0 * (int64_t)m;
    float pv[VREG > 0 ? VREG : 1];
#pragma unroll
    for (int k = 0; k < VREG; ++k) pv[k] = tid + NT * k < tot ? cval[tid + NT * k] : 0.0f;
    const uint16_t* gidx = idx + i0 * (int64_t)m;
    const uint16_t* cidx = gidx;
    if constexpr (STAGE) {
        uint16_t* sidx = reinterpret_cast<uint16_t*>(wsum + NT / 64);  // 16-byte aligned (byte offset 256 nbc + 128 + NT / 16)
        const int nvec = (tot * 2) / 16;
        const uint4* src = reinterpret_cast<const uint4*>(gidx);
        uint4* dst = reinterpret_cast<uint4*>(sidx);
        for (int v = tid; v < nvec; v += NT) dst[v] = src[v];
        for (int f = nvec * 8 + tid; f < tot; f += NT) sidx[f] = gidx[f];
        cidx = sidx;
        __syncthreads();
    }

    // block starts: block b begins at the first entry whose block number
    // reaches b, which the entry finds by comparing with its predecessor.  The
    // chunk's index rows are one contiguous range, walked flat (entry f of the
    // chunk is entry e = f - s m of sample s) so that loads stay in flight.
    for (int s = ns; s < kChunk; ++s)
        for (int b = tid; b < nb1; b += NT) off[s * nb1 + b] = 0;
#pragma unroll 4
    for (int f = tid; f < tot; f += NT) {
        int s = (int)((float)f * inv_m);
        if (s * m > f) --s;
        if ((s + 1) * m <= f) ++s;
        const int e = f - s * m;
        const int be = (int)cidx[f] >> sh_c;
        const int bp = e > 0 ? ((int)cidx[f - 1] >> sh_c) : -1;
        for (int b = bp + 1; b <= be; ++b) off[s * nb1 + b] = (uint32_t)e;
        if (e == m - 1)
            for (int b = be + 1; b <= nbc; ++b) off[s * nb1 + b] = (uint32_t)m;
    }
    __syncthreads();

    // exclusive scan of the segment sizes in (block, sample) order
    const int Q = nbc * kChunk;
    const int per = (Q + NT - 1) / NT;
    const int q0 = tid * per;
    uint32_t run = 0;
    for (int k = 0; k < per; ++k) {
        const int q = q0 + k;
        if (q < Q) {
            const int b = q >> 5, s = q & 31;
            run += off[s * nb1 + b + 1] - off[s * nb1 + b];
        }
    }
    uint32_t pos = block_exclusive_scan<NT>(run, wsum);
    uint32_t* bs = BS + c * nb1;
    for (int k = 0; k < per; ++k) {
        const int q = q0 + k;
        if (q < Q) {
            const int b = q >> 5, s = q & 31;
            const uint32_t o0 = off[s * nb1 + b];
            if (s == 0) bs[b] = pos;
            seg[q] = pos - o0;  // modular: seg + e is the chunk position of entry e
            pos += off[s * nb1 + b + 1] - o0;
        }
    }
    if (tid == 0) bs[nbc] = (uint32_t)ns * (uint32_t)m;
    __syncthreads();
    if (SS) {
        // start of segment (b, s) relative to block b's run
        uint16_t* ssc = SS + c * (int64_t)Q;
        for (int q = tid; q < Q; q += NT) {
            const int b = q >> 5, s = q & 31;
            const uint32_t st = seg[q] + off[s * nb1 + b];
            const uint32_t s0 = seg[b * kChunk] + off[b];
            ssc[q] = (uint16_t)(st - s0);
        }
    }

    uint32_t* Pc = P + c * (int64_t)kChunk * m;
    uint16_t* OAc = OA + c * (int64_t)kChunk * m;
    uint32_t vmax = 0u;  // largest |value| as FP32 bits: NaN and infinity order above every finite value
    auto put = [&](int f, float v) {
        int s = (int)((float)f * inv_m);
        if (s * m > f) --s;
        if ((s + 1) * m <= f) ++s;
        const uint32_t j = cidx[f];
        const uint32_t q = seg[((int)j >> sh_c) * kChunk + s] + (uint32_t)(f - s * m);
        const uint32_t vb = __float_as_uint(v) & 0x7fffffffu;
        vmax = vb > vmax ? vb : vmax;
        Pc[q] = split ? split_bits(v) : __float_as_uint(v);
        OAc[q] = (uint16_t)((j & (uint32_t)(tr - 1)) * rowbytes + s * eb);
    };
    if constexpr (VREG > 0) {
#pragma unroll
        for (int k = 0; k < VREG; ++k)
            if (tid + NT * k < tot) put(tid + NT * k, pv[k]);
    } else {
#pragma unroll 4
        for (int f = tid; f < tot; f += NT) put(f, cval[f]);
    }
    if (CM) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t t = (uint32_t)__shfl_xor((int)vmax, o, 64);
            vmax = t > vmax ? t : vmax;
        }
        __syncthreads();  // wsum is free again
        if ((tid & 63) == 0) wsum[tid >> 6] = vmax;
        __syncthreads();
        if (tid == 0) {
            uint32_t mx = wsum[0];
            for (int w = 1; w < NT / 64; ++w) mx = wsum[w] > mx ? wsum[w] : mx;
            CM[c] = mx;
        }
    }
}

// A chunk's runs for one tile (workgroup-uniform).
struct ChunkRun {
    uint32_t a0, na;  // row-block run: first q and length
    uint32_t b0, nb;  // column-block run (empty on inner tiles)
};

// The four run bounds of chunk c are loaded by lanes 0..3 as vector loads, so
// that their wait falls at the first use (an iteration later), not at the
// matrix-core block's first LDS wait as a scalar load's would.  Past the range
// (live false) the lanes read chunk c_safe and the runs are emptied at unpack.
__device__ inline int chunk_run_col(int ba0, int ba1, int bb, bool inner, int lane)
{
    const int sel = lane & 3;
    return sel == 0 ? ba0 : sel == 1 ? ba1 : bb + (sel == 3 && !inner ? 1 : 0);
}

__device__ inline uint32_t chunk_run_load(const uint32_t* __restrict__ BS, int nb1, int64_t c, bool live,
                                          int64_t c_safe, int col)
{
    return BS[(live ? c : c_safe) * nb1 + col];
}

__device__ inline ChunkRun chunk_run_unpack(uint32_t v, bool live)
{
    ChunkRun r{0, 0, 0, 0};
    if (live) {
        r.a0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
        r.na = (uint32_t)__builtin_amdgcn_readlane((int)v, 1) - r.a0;
        r.b0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 2);
        r.nb = (uint32_t)__builtin_amdgcn_readlane((int)v, 3) - r.b0;
    }
    return r;
}

// An entry's column-tile offset from its row-tile offset: OA mod tcb, where
// tcb (tc rows) is a multiple of a row and OA < 2 tcb (unsigned wrap-around
// makes the difference the larger operand when OA < tcb).
__device__ inline uint32_t col_offset(uint32_t oa, uint32_t tcb)
{
    const uint32_t d = oa - tcb;
    return d < oa ? d : oa;
}

// Register share of one chunk: thread t holds run entries t + 256 k.
template <int SA, int SB>
struct ChunkRegs {
    uint32_t pa[SA], oa[SA], pb[SB], ob[SB];
};

// Loads for one chunk; lanes past a run's end read entry 0 of the chunk (a
// valid address) and are masked at the scatter.  Byte offsets inside the chunk
// are 32-bit (a chunk holds at most 32 * 65536 entries), so the loads take a
// uniform base and one offset register.
template <int SA, int SB>
__device__ inline void load_chunk(ChunkRegs<SA, SB>& R, const uint32_t* __restrict__ P,
                                  const uint16_t* __restrict__ OA, int64_t cbase, const ChunkRun& r, int tid)
{
    const unsigned char* pc = reinterpret_cast<const unsigned char*>(P + cbase);
    const unsigned char* ac = reinterpret_cast<const unsigned char*>(OA + cbase);
#pragma unroll
    for (int k = 0; k < SA; ++k) {
        const uint32_t j = (uint32_t)(tid + 256 * k);
        const uint32_t q = j < r.na ? r.a0 + j : 0u;
        R.pa[k] = *reinterpret_cast<const uint32_t*>(pc + q * 4u);
        R.oa[k] = *reinterpret_cast<const uint16_t*>(ac + q * 2u);
    }
#pragma unroll
    for (int k = 0; k < SB; ++k) {
        const uint32_t j = (uint32_t)(tid + 256 * k);
        const uint32_t q = j < r.nb ? r.b0 + j : 0u;
        R.pb[k] = *reinterpret_cast<const uint32_t*>(pc + q * 4u);
        R.ob[k] = *reinterpret_cast<const uint16_t*>(ac + q * 2u);  // row-tile offset: folded at the scatter
    }
}

// LO: byte distance from the tile's hi array to its lo array (split variant)
template <bool SPLIT, int LO>
__device__ inline void lds_put(unsigned char* base, uint32_t off, uint32_t pv)
{
    if constexpr (SPLIT) {
        *reinterpret_cast<unsigned short*>(base + off) = (unsigned short)pv;
        *reinterpret_cast<unsigned short*>(base + off + LO) = (unsigned short)(pv >> 16);
    } else {
        *reinterpret_cast<uint32_t*>(base + off) = pv;
    }
}

// The split products hi*hi + hi*lo + lo*hi drop lo*lo, which biases every
// diagonal entry low by the mean of lo^2 (about 2.5e-6 relative); inner tiles
// therefore also sum (hi + lo)^2 of their column block's entries in FP64 and
// those sums replace the matrix-core diagonal (hi + lo is v to 2^-16
// relative, with no systematic bias).
template <bool SPLIT>
__device__ inline void add_square(double* diag, uint32_t oa, uint32_t pv, int boff, int tc)
{
    if constexpr (SPLIT) {
        const int c = (int)(oa / (uint32_t)(kBfStride * 2)) - boff;
        if (c >= 0 && c < tc) {
            const double v = (double)bf16_bits_to_float((unsigned short)pv) +
                             (double)bf16_bits_to_float((unsigned short)(pv >> 16));
            atomicAdd(&diag[c], v * v);
        }
    }
}

template <bool SPLIT>
__device__ inline unsigned char* tile_base(MfmaLds<SPLIT>& L, bool col)
{
    if constexpr (SPLIT)
        return reinterpret_cast<unsigned char*>(col ? L.bhi : L.ahi);
    else
        return reinterpret_cast<unsigned char*>(col ? L.b : L.a);
}

constexpr int kLoA = kTR * kBfStride * 2;
constexpr int kLoB = kTC * kBfStride * 2;

// Scatter (or clear) one chunk's register share, then any run entries past it
// (more than 256 SA or 256 SB in the chunk: a workgroup-uniform branch, direct
// loads four at a time).
template <bool SPLIT, int SA, int SB>
__device__ inline void put_chunk(MfmaLds<SPLIT>& L, double* diag, const ChunkRegs<SA, SB>& R, const ChunkRun& r,
                                 bool clear,
                                 bool inner, int boff, int tc, const uint32_t* __restrict__ P,
                                 const uint16_t* __restrict__ OA, int64_t cbase, uint32_t tcb, int tid)
{
    unsigned char* ta = tile_base<SPLIT>(L, false);
    unsigned char* tb = tile_base<SPLIT>(L, true);
#pragma unroll
    for (int k = 0; k < SA; ++k)
        if ((uint32_t)(tid + 256 * k) < r.na) {
            lds_put<SPLIT, kLoA>(ta, R.oa[k], clear ? 0u : R.pa[k]);
            if (inner && !clear) add_square<SPLIT>(diag, R.oa[k], R.pa[k], boff, tc);
        }
#pragma unroll
    for (int k = 0; k < SB; ++k)
        if ((uint32_t)(tid + 256 * k) < r.nb) lds_put<SPLIT, kLoB>(tb, col_offset(R.ob[k], tcb), clear ? 0u : R.pb[k]);
    const uint32_t* pc = P + cbase;
    const uint16_t* ac = OA + cbase;
    if (r.na > 256u * SA) {
        for (uint32_t j0 = 256u * SA; j0 < r.na; j0 += 1024u) {
            uint32_t pv[4], ov[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t j = j0 + 256u * u + (uint32_t)tid;
                const uint32_t q = j < r.na ? r.a0 + j : 0u;
                ov[u] = ac[q];
                pv[u] = clear ? 0u : pc[q];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (j0 + 256u * u + (uint32_t)tid < r.na) {
                    lds_put<SPLIT, kLoA>(ta, ov[u], pv[u]);
                    if (inner && !clear) add_square<SPLIT>(diag, ov[u], pv[u], boff, tc);
                }
        }
    }
    if (r.nb > 256u * SB) {
        for (uint32_t j0 = 256u * SB; j0 < r.nb; j0 += 1024u) {
            uint32_t pv[4], ov[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t j = j0 + 256u * u + (uint32_t)tid;
                const uint32_t q = j < r.nb ? r.b0 + j : 0u;
                ov[u] = col_offset(ac[q], tcb);
                pv[u] = clear ? 0u : pc[q];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (j0 + 256u * u + (uint32_t)tid < r.nb) lds_put<SPLIT, kLoB>(tb, ov[u], pv[u]);
        }
    }
}

// One half of a chunk's K-loop on the matrix cores for a wave's 128 x 64
// sub-tile (4 x 2 blocks of 32 x 32): K slots 16 half .. 16 half + 15.
template <bool SPLIT>
__device__ inline void mfma_step(const MfmaLds<SPLIT>& L, f32x16 (&acc)[4][2], int half, int wr, int brow0,
                                 bool inner, int lane)
{
    if constexpr (SPLIT) {
        // column operand rows: the column tile, or the row tile at offset boff
        const unsigned short* bh_src = inner ? L.ahi : L.bhi;
        const unsigned short* bl_src = inner ? L.alo : L.blo;
        const int koff = 16 * half + 8 * (lane >> 5);
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
    } else {
        const float* bf_src = inner ? L.a : L.b;
#pragma unroll 4
        for (int kk = 16 * half; kk < 16 * half + 16; kk += 2) {
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

template <bool SPLIT, int SA, int SB>
__global__ __launch_bounds__(256, 2) void k_gram_mfma(const uint32_t* __restrict__ P, const uint16_t* __restrict__ OA,
                                                      const uint32_t* __restrict__ BS, int m, TileGeom g, int64_t n,
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
    const bool inner = tb < (ta + 1) * g.ratio;  // column block inside the row block
    const int boff = tb * g.tc - ta * g.tr;      // row of the column block inside the row tile (inner)
    const int nb1 = g.nbc + 1;
    const int ba0 = ta * g.ratio, ba1 = (ta + 1) * g.ratio;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;

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
    const int64_t c0 = sbeg / kChunk, c1 = (send + kChunk - 1) / kChunk;
    const int64_t cstride = (int64_t)kChunk * m;

    // pipeline: runs two chunks ahead, entries one chunk ahead
    const int rcol = chunk_run_col(ba0, ba1, tb, inner, lane);
    ChunkRun r_cur = chunk_run_unpack(chunk_run_load(BS, nb1, c0, true, c0, rcol), true);
    ChunkRegs<SA, SB> R_cur, R_prev;
#pragma unroll
    for (int k = 0; k < SA; ++k) R_prev.pa[k] = R_prev.oa[k] = 0;
#pragma unroll
    for (int k = 0; k < SB; ++k) R_prev.pb[k] = R_prev.ob[k] = 0;
    const uint32_t tcb = (uint32_t)g.tc * (SPLIT ? kBfStride * 2 : kF32Stride * 4);
    load_chunk<SA, SB>(R_cur, P, OA, c0 * cstride, r_cur, tid);  // c0 < c1: a range is never empty
    uint32_t v_next = chunk_run_load(BS, nb1, c0 + 1, c0 + 1 < c1, c0, rcol);
    ChunkRun r_prev{0, 0, 0, 0};
    int64_t c_prev = c0;

    const int brow0 = (inner ? boff : 0) + wc * 64;
    // a wave whose 128 x 64 block lies wholly below the diagonal (inner tiles:
    // its first row past its last column) has nothing to add to the upper
    // triangle, the only part the reduction keeps: it loads and scatters with
    // the others but leaves its accumulators at zero
    const bool below = inner && wr * 128 > brow0 + 63;

    for (int64_t c = c0; c < c1; ++c) {
        __syncthreads();
        // clear the previous chunk's slots, then scatter this chunk; a slot is
        // cleared and written by different waves, so a barrier orders the two
        if (c > c0) {
            put_chunk<SPLIT, SA, SB>(L, L.diag_ptr(), R_prev, r_prev, true, inner, boff, g.tc, P, OA, c_prev * cstride, tcb, tid);
            __syncthreads();
        }
        put_chunk<SPLIT, SA, SB>(L, L.diag_ptr(), R_cur, r_cur, false, inner, boff, g.tc, P, OA, c * cstride, tcb, tid);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SA; ++k) R_prev.oa[k] = R_cur.oa[k];
#pragma unroll
        for (int k = 0; k < SB; ++k) R_prev.ob[k] = R_cur.ob[k];
        r_prev = r_cur;
        c_prev = c;
        // loads for the next chunks fly while this chunk runs on the matrix cores;
        // the entry loads are unconditional (an empty run past the range reads
        // this chunk's entry 0), so no value merges after them and nothing
        // waits for them before the matrix-core block
        r_cur = chunk_run_unpack(v_next, c + 1 < c1);
        load_chunk<SA, SB>(R_cur, P, OA, (c + 1 < c1 ? c + 1 : c) * cstride, r_cur, tid);
        v_next = chunk_run_load(BS, nb1, c + 2, c + 2 < c1, c, rcol);
        // keep the scheduler from sinking those loads (or their address math)
        // into the matrix-core block, where their waits would stall it
        __builtin_amdgcn_sched_barrier(0);
        // raised issue priority for the matrix-core block: when both
        // workgroups of a CU reach it together, one runs ahead and the two
        // fall back into alternating scatter and matrix-core phases
        __builtin_amdgcn_s_setprio(1);
        if (!below) {
            mfma_step<SPLIT>(L, acc, 0, wr, brow0, inner, lane);
            mfma_step<SPLIT>(L, acc, 1, wr, brow0, inner, lane);
        }
        __builtin_amdgcn_s_setprio(0);
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
// Sparse Gram (FP32 values, exact products): each workgroup owns one W x W
// upper tile (row block A, column block B, W = min(p, 128)) and one span of
// chunks.  For every sample of a chunk, each of its kept entries in block A
// (one per thread) is multiplied with each of its kept entries in block B
// (staged in LDS) and the product is added into the tile at (row, column) --
// m^2 multiply-adds per sample in all instead of the dense tile's p^2.
//
// The adds are integer LDS atomics (the FP32 ones are far slower): over a
// range of at most 2048 samples the products are fixed point, v_a v_b 2^F
// rounded to the nearest integer, with F the largest integer for which
// c v^2 2^F + c / 2 < 2^31: v is the range's largest |value| (the pack's
// per-chunk maxima) and c the largest number of the range's samples that
// kept any one coordinate (k_range_counts).  An entry (j, k) receives one
// product per sample that kept both j and k -- at most c of them -- so its
// sum cannot overflow and is exact.  At the end of each range the integer tile is added
// into FP64 registers (sum * 2^-F, exact conversion) and cleared; the span's
// tile is written once as FP32 partials, which the fixed-order FP64 reduction
// sums.  Every sum is order-independent, so the result is deterministic.
// ---------------------------------------------------------------------------
constexpr int kSpRangeChunks = 64;                // chunks per fixed-point range (2048 samples)

// RC[r] = the largest number of samples of range r (kSpRangeChunks chunks)
// that kept one coordinate: a histogram of the range's indices in LDS, two
// 16-bit counters per word (a range has at most 2048 samples).
__global__ __launch_bounds__(1024) void k_range_counts(const uint16_t* __restrict__ idx, int64_t n, int m, int p,
                                                       uint32_t* __restrict__ RC)
{
    extern __shared__ uint32_t hist[];
    __shared__ uint32_t red[16];
    const int tid = threadIdx.x;
    const int nw = (p + 1) / 2;
    const int64_t i0 = (int64_t)blockIdx.x * kSpRangeChunks * kChunk;
    int64_t i1 = i0 + (int64_t)kSpRangeChunks * kChunk;
    if (i1 > n) i1 = n;
    for (int e = tid; e < nw; e += 1024) hist[e] = 0u;
    __syncthreads();
    const uint16_t* base = idx + i0 * (int64_t)m;
    const int64_t tot = (i1 - i0) * (int64_t)m;
#pragma unroll 4
    for (int64_t f = tid; f < tot; f += 1024) {
        const uint32_t j = base[f];
        atomicAdd(&hist[j >> 1], 1u << (16u * (j & 1u)));
    }
    __syncthreads();
    uint32_t mx = 0u;
    for (int e = tid; e < nw; e += 1024) {
        const uint32_t w = hist[e];
        const uint32_t lo = w & 0xffffu, hi = w >> 16;
        mx = lo > mx ? lo : mx;
        mx = hi > mx ? hi : mx;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t t = (uint32_t)__shfl_xor((int)mx, o, 64);
        mx = t > mx ? t : mx;
    }
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < 16; ++w) mx = red[w] > mx ? red[w] : mx;
        RC[blockIdx.x] = mx;
    }
}

constexpr int kSpW = 128;                         // tile edge (coordinates per block)
constexpr int kSpStride = kSpW + 1;               // accumulator words per tile row
constexpr int kSpThreads = 1024;                  // threads per workgroup (one workgroup per CU)
constexpr int kSpWaves = kSpThreads / 64;
constexpr int kSpEpt = kSpW * kSpW / kSpThreads;  // accumulators per thread (FP64 flush registers)
constexpr int kSpStage = 512;                     // staged column entries per wave (one segment)
constexpr int kSpUnitChunks = 1;                  // chunks per wave work unit (1 or 2)
constexpr int kSpG = 8;                           // 64-entry groups of a unit's column run loaded at once

// One CU's workgroup: the tile's integer accumulators, shared by the waves
// (integer atomics), and a private staging area per wave.  The column run of
// a unit is staged as (value bits, byte offset of the column in a tile row),
// two entries per uint4, each sample's entries padded with zero products (pad
// column kSpW) to a multiple of four, so that the products loop reads four at
// a time with no bounds.
struct SparseLds {
    int32_t acc[kSpW * kSpStride];
    uint4 stg[kSpWaves][kSpStage / 2];
    uint32_t next;  // the range's next unit (wave work queue)
};

__device__ inline void sp_atomic4(unsigned char* base, float va, const uint4& a, const uint4& b)
{
    atomicAdd(reinterpret_cast<int*>(base + a.y), (int)rintf(va * __uint_as_float(a.x)));
    atomicAdd(reinterpret_cast<int*>(base + a.w), (int)rintf(va * __uint_as_float(a.z)));
    atomicAdd(reinterpret_cast<int*>(base + b.y), (int)rintf(va * __uint_as_float(b.x)));
    atomicAdd(reinterpret_cast<int*>(base + b.w), (int)rintf(va * __uint_as_float(b.z)));
}

// Keeps the compiler from moving this wave's LDS accesses across the point;
// the LDS serves one wave's accesses in order, so no barrier is needed for the
// wave to read what it wrote.
__device__ inline void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The largest F with cnt (v 2^F)^2 (1 + 2^-22) + cnt / 2 < 2^31: at most cnt
// products of magnitude up to v^2 (their FP32 rounding included), each
// rounded by at most 1/2.  F stays within [-140, 100], so v 2^F is finite.
__device__ inline int sparse_scale(float vmax, uint32_t cnt)
{
    if (cnt == 0u || !(vmax > 0.0f)) return 0;
    const double lim = 2147483647.0 - 0.5 * (double)cnt;
    const double b = (double)cnt * (double)vmax * (double)vmax * (1.0 + 0x1p-22);
    int F = (int)floor(log2(lim / b));
    if (F > 100) F = 100;
    if (F < -140) F = -140;
    while (F > -140 && ldexp(b, F) >= lim) --F;
    while (F < 100 && ldexp(b, F + 1) < lim) ++F;
    return F;
}

// Runs of one unit: the two chunks' row-block and column-block runs (the
// second chunk's empty past the range).
struct SpUnitRuns {
    uint32_t ra0, nra, rb0, nrb;  // row runs of chunks a and b
    uint32_t ca0, nca, cb0, ncb;  // column runs
};

__global__ __launch_bounds__(kSpThreads, 4) void k_gram_sparse(const uint32_t* __restrict__ P,
                                                               const uint16_t* __restrict__ OA,
                                                               const uint32_t* __restrict__ BS,
                                                               const uint16_t* __restrict__ SS,
                                                               const uint32_t* __restrict__ CM,
                                                               const uint32_t* __restrict__ RC, int m, TileGeom g,
                                                               int64_t nchunks, int nsr, int64_t sr_chunks,
                                                               float* __restrict__ part)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SparseLds& L = *reinterpret_cast<SparseLds*>(smem_raw);
    const int64_t total = (int64_t)g.ntiles * nsr;
    const int64_t item = xcd_item(blockIdx.x, total);
    if (item >= total) return;
    const int sr = (int)(item / g.ntiles);
    const int tile = (int)(item % g.ntiles);
    int ta, tb;
    decode_rect_tile(tile, g, ta, tb);
    const int W = g.tc;
    const int nb1 = g.nbc + 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t c0 = (int64_t)sr * sr_chunks;
    int64_t c1 = c0 + sr_chunks;
    if (c1 > nchunks) c1 = nchunks;
    const int64_t cstride = (int64_t)kChunk * m;
    const int64_t sstride = (int64_t)g.nbc * kChunk;
    uint2* stg = reinterpret_cast<uint2*>(L.stg[wave]);
    const uint4* stg4 = L.stg[wave];

    for (int e = tid; e < kSpW * kSpStride; e += kSpThreads) L.acc[e] = 0;
    double accd[kSpEpt];
#pragma unroll
    for (int k = 0; k < kSpEpt; ++k) accd[k] = 0.0;
    bool bad = false;

    for (int64_t rc0 = c0; rc0 < c1; rc0 += kSpRangeChunks) {
        const int64_t rc1 = (rc0 + kSpRangeChunks < c1) ? rc0 + kSpRangeChunks : c1;
        const int units = (int)((rc1 - rc0 + kSpUnitChunks - 1) / kSpUnitChunks);
        if (tid == 0) L.next = 0u;
        // the range's scale, from its chunks' largest |value| (every wave alike)
        uint32_t mx = (rc0 + lane < rc1) ? CM[rc0 + lane] : 0u;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t t = (uint32_t)__shfl_xor((int)mx, o, 64);
            mx = t > mx ? t : mx;
        }
        if (mx >= 0x7f800000u) bad = true;  // a non-finite value: the tile becomes NaN
        const int F = bad ? 0 : sparse_scale(__uint_as_float(mx), RC[rc0 / kSpRangeChunks]);
        const float scale = ldexpf(1.0f, F);
        __syncthreads();  // L.next set; the previous range's flush done

        for (;;) {
            uint32_t u = 0;
            if (lane == 0) u = atomicAdd(&L.next, 1u);
            u = (uint32_t)__builtin_amdgcn_readfirstlane((int)u);
            if ((int)u >= units) break;
            const int64_t ca = rc0 + kSpUnitChunks * (int64_t)u;
            const bool has_b = kSpUnitChunks == 2 && ca + 1 < rc1;
            const int64_t cb = has_b ? ca + 1 : ca;
            // run bounds: lanes 0..3 chunk a, lanes 4..7 chunk b
            const int bsel = lane & 3;
            const int bcol = bsel == 0 ? ta : bsel == 1 ? ta + 1 : bsel == 2 ? tb : tb + 1;
            const uint32_t bv = BS[((lane & 4) ? cb : ca) * nb1 + bcol];
            SpUnitRuns R;
            R.ra0 = (uint32_t)__builtin_amdgcn_readlane((int)bv, 0);
            R.nra = (uint32_t)__builtin_amdgcn_readlane((int)bv, 1) - R.ra0;
            R.ca0 = (uint32_t)__builtin_amdgcn_readlane((int)bv, 2);
            R.nca = (uint32_t)__builtin_amdgcn_readlane((int)bv, 3) - R.ca0;
            R.rb0 = (uint32_t)__builtin_amdgcn_readlane((int)bv, 4);
            R.nrb = has_b ? (uint32_t)__builtin_amdgcn_readlane((int)bv, 5) - R.rb0 : 0u;
            R.cb0 = (uint32_t)__builtin_amdgcn_readlane((int)bv, 6);
            R.ncb = has_b ? (uint32_t)__builtin_amdgcn_readlane((int)bv, 7) - R.cb0 : 0u;
            const uint32_t nC = R.nca + R.ncb, nR = R.nra + R.nrb;
            // per-sample layout, lane = sample of the unit (chunk a: 0..31, chunk b: 32..63)
            const uint32_t ssv = SS[((lane < kChunk) ? ca : cb) * sstride + tb * kChunk + (lane & (kChunk - 1))];
            const uint32_t cs = (lane < kChunk) ? ssv : (has_b ? R.nca + ssv : nC);
            const uint32_t nxt = (uint32_t)__shfl_down((int)cs, 1, 64);
            const uint32_t cn = (lane == kChunk - 1) ? R.nca : (lane == 63 ? nC : nxt);
            const uint32_t plen = (cn - cs + 3u) & ~3u;
            uint32_t pen = plen;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t t = (uint32_t)__shfl_up((int)pen, d, 64);
                if (lane >= d) pen += t;
            }
            uint32_t pst = pen - plen;
            const uint32_t ptotal = (uint32_t)__builtin_amdgcn_readlane((int)pen, 63);
            int seg = 0, nseg = 1;
            if (ptotal > (uint32_t)kSpStage) {
                // greedy: a sample that would overflow the current segment starts the next
                uint32_t base = 0, my_base = 0;
                int id = 0;
                for (int t = 0; t < 64; ++t) {
                    const uint32_t tst = (uint32_t)__builtin_amdgcn_readlane((int)pst, t);
                    const uint32_t ten = (uint32_t)__builtin_amdgcn_readlane((int)pen, t);
                    if (ten - base > (uint32_t)kSpStage) {
                        ++id;
                        base = tst;
                    }
                    if (lane == t) {
                        seg = id;
                        my_base = base;
                    }
                }
                pst -= my_base;
                pen -= my_base;
                nseg = id + 1;
            }
            // the unit's entries, up to kSpG groups of 64 per run, requested
            // together so that one memory latency covers the unit
            auto gidx = [&](uint32_t q, uint32_t na, uint32_t a0, uint32_t b0, bool& inb) -> int64_t {
                inb = q >= na;
                return inb ? cb * cstride + b0 + (q - na) : ca * cstride + a0 + q;
            };
            // column entries: up to kSpG groups (indices two to a register)
            uint32_t cpv[kSpG], cov2[kSpG / 2];
#pragma unroll
            for (int gg = 0; gg < kSpG; ++gg) {
                cpv[gg] = 0u;
                if (gg % 2 == 0) cov2[gg / 2] = 0u;
                const uint32_t q = (uint32_t)(64 * gg + lane);
                bool inb;
                if ((uint32_t)(64 * gg) < nC) {
                    const int64_t gq = gidx(q < nC ? q : 0u, R.nca, R.ca0, R.cb0, inb);
                    cpv[gg] = P[gq];
                    cov2[gg / 2] |= (uint32_t)OA[gq] << (16 * (gg % 2));
                }
            }
            // stage one column entry (every lane calls: the lane reads need their sources active)
            auto stage = [&](uint32_t q, uint32_t pv, uint32_t ov, int k) {
                const bool live = q < nC;
                const int s = live ? (int)(ov >> 7) + (q >= R.nca ? kChunk : 0) : 0;
                const uint32_t scs = (uint32_t)__shfl((int)cs, s, 64);
                const uint32_t scn = (uint32_t)__shfl((int)cn, s, 64);
                const uint32_t spst = (uint32_t)__shfl((int)pst, s, 64);
                const uint32_t spen = (uint32_t)__shfl((int)pen, s, 64);
                const int sseg = __shfl(seg, s, 64);
                if (live && sseg == k) {
                    const uint32_t pos = spst + (q - scs);
                    stg[pos] = make_uint2(pv, (ov & 127u) * 4u);
                    if (q + 1 == scn)
                        for (uint32_t dd = pos + 1; dd < spen; ++dd) stg[dd] = make_uint2(0u, (uint32_t)kSpW * 4u);
                }
            };
            // products of one row entry with its sample's staged entries
            auto products = [&](uint32_t q, uint32_t pv, uint32_t ov, int k) {
                const bool live = q < nR;
                const int s = live ? (int)(ov >> 7) + (q >= R.nra ? kChunk : 0) : 0;
                const uint32_t u0 = (uint32_t)__shfl((int)pst, s, 64);
                const uint32_t u1 = (uint32_t)__shfl((int)pen, s, 64);
                const int sseg = __shfl(seg, s, 64);
                if (live && sseg == k) {
                    const float va = __uint_as_float(pv) * scale;
                    unsigned char* base =
                        reinterpret_cast<unsigned char*>(L.acc) + (ov & 127u) * (uint32_t)(kSpStride * 4);
                    uint32_t v = u0;
                    // eight entries per step: their four LDS reads are issued before the adds
                    for (; v + 8 <= u1; v += 8) {
                        const uint4 a = stg4[v / 2], b = stg4[v / 2 + 1], c = stg4[v / 2 + 2], d = stg4[v / 2 + 3];
                        sp_atomic4(base, va, a, b);
                        sp_atomic4(base, va, c, d);
                    }
                    if (v < u1) {
                        const uint4 a = stg4[v / 2], b = stg4[v / 2 + 1];
                        sp_atomic4(base, va, a, b);
                    }
                }
            };
            for (int k = 0; k < nseg; ++k) {
                wave_lds_fence();  // the previous unit's or segment's reads of the stage come first
#pragma unroll
                for (int gg = 0; gg < kSpG; ++gg)
                    if ((uint32_t)(64 * gg) < nC)
                        stage((uint32_t)(64 * gg + lane), cpv[gg], (cov2[gg / 2] >> (16 * (gg % 2))) & 0xffffu, k);
                for (uint32_t q0 = 64u * kSpG; q0 < nC; q0 += 64u) {  // long runs: further groups one by one
                    const uint32_t q = q0 + (uint32_t)lane;
                    bool inb;
                    const int64_t gq = gidx(q < nC ? q : 0u, R.nca, R.ca0, R.cb0, inb);
                    stage(q, P[gq], OA[gq], k);
                }
                wave_lds_fence();
                // row entries, one group of 64 at a time with the next group's loads in flight
                uint32_t rp = 0u, ro = 0u;
                if (nR > 0u) {
                    bool inb;
                    const int64_t gq = gidx(lane < (int)nR ? (uint32_t)lane : 0u, R.nra, R.ra0, R.rb0, inb);
                    rp = P[gq];
                    ro = OA[gq];
                }
                for (uint32_t q0 = 0; q0 < nR; q0 += 64u) {
                    const uint32_t q = q0 + (uint32_t)lane;
                    uint32_t np = 0u, no = 0u;
                    if (q0 + 64u < nR) {
                        const uint32_t qn = q + 64u;
                        bool inb;
                        const int64_t gq = gidx(qn < nR ? qn : 0u, R.nra, R.ra0, R.rb0, inb);
                        np = P[gq];
                        no = OA[gq];
                    }
                    products(q, rp, ro, k);
                    rp = np;
                    ro = no;
                }
            }
        }
        __syncthreads();  // every unit of the range is summed
        // the range's integer sums into FP64, then cleared for the next range
#pragma unroll
        for (int k = 0; k < kSpEpt; ++k) {
            const int e = tid + kSpThreads * k;
            const int i = e / W, j = e - (e / W) * W;
            if (e < W * W) {
                int32_t* a = &L.acc[i * kSpStride + j];
                accd[k] += ldexp((double)*a, -F);
                *a = 0;
            }
        }
    }
    float* out = part + ((int64_t)sr * g.ntiles + tile) * (int64_t)W * W;
#pragma unroll
    for (int k = 0; k < kSpEpt; ++k) {
        const int e = tid + kSpThreads * k;
        if (e < W * W) out[e] = bad ? __builtin_nanf("") : (float)accd[k];
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
    // the loads of eight ranges are issued together; the sum keeps range order
    const PT* pe = part + (int64_t)tile * per_tile + e;
    const int64_t rstride = (int64_t)g.ntiles * per_tile;
#pragma unroll 8
    for (int s = 0; s < nsplit; ++s) sum += (double)pe[(int64_t)s * rstride];
    const int boff = tb * g.tc - ta * g.tr;
    if (pdiag && tb < (ta + 1) * g.ratio && i == j + boff)
        for (int s = 0; s < nsplit; ++s) sum += pdiag[((int64_t)s * g.ntiles + tile) * g.tc + j];
    acc[(int64_t)(ta * g.tr + i) * g.p + (tb * g.tc + j)] += sum;
}

__global__ __launch_bounds__(256) void k_cov_finalize(const double* __restrict__ acc, int p, int lda, double sdiag,
                                                      double soff, double* __restrict__ C)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)p * p) return;
    const int j = (int)(g / p), k = (int)(g - (int64_t)(g / p) * p);
    // (min, max) lies in an upper tile; reading it for both (j, k) and (k, j)
    // makes the result exactly symmetric
    const int r = j < k ? j : k, c = j < k ? k : j;
    const double v = acc[(int64_t)r * lda + c];
    C[g] = (j == k) ? sdiag * v : soff * v;
}

// ---------------------------------------------------------------------------
// Host side: tiling plan and launches.
// ---------------------------------------------------------------------------
struct GramPlan {
    TileGeom geom;
    bool sparse;                    // the sparse form (k_gram_sparse) instead of dense tiles
    int nsplit, sa, sb;
    int64_t split_len, nchunks;
    size_t off_bytes;               // FP64 variant: per-sample block offsets
    size_t pk_bytes, bs_bytes;      // packed variants: packed chunks (P, then OA) and block starts
    size_t ss_bytes, cm_bytes, rc_bytes;  // sparse form: per-sample run starts, per-chunk largest |value|,
                                          // per-range largest coordinate count
    size_t part_bytes, diag_bytes;
};

static size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

// Block offsets per sample (FP64 variant): the kept count of a sample in a
// block of w coordinates is hypergeometric (m draws, w of p marked).
static double block_count_var(int p, int m, int w)
{
    return (p > 1) ? (double)m * ((double)w / p) * (1.0 - (double)w / p) * (double)(p - m) / (p - 1) : 0.0;
}

// Register slots per thread for a chunk's run in a block of w coordinates:
// 256 entries per slot, enough for the mean plus four standard deviations of
// the chunk's count (a sum of kChunk independent hypergeometric counts),
// rounded up to a power of two, at most 8 (longer runs take the uniform
// overflow loop).
static int run_slots(int p, int m, int w)
{
    const double mu = (double)kChunk * m * w / p;
    const double sd = sqrt((double)kChunk * block_count_var(p, m, w));
    const int need = (int)((mu + 4.0 * sd + 255.999) / 256.0);
    int k = 1;
    while (k < need && k < 8) k <<= 1;
    return k;
}

// Which Gram form runs (algo: 0 = the faster by the cost model below, 1 =
// dense tiles, 2 = sparse).  FP64 plans have the dense FP64 form only.  The
// model prices each form from rates measured on MI355X (256 CUs, scaled by
// the CU count): dense tiles execute n p^2 / 2 multiply-adds (x 3 products
// for split plans) at 8.2e14 (split) or 6.0e13 (FP32) per second; the sparse
// form costs n (5.4e-11 s per output tile + 3.9e-13 s m^2 / 2).
static bool use_sparse(int prec, int p, int m, int64_t n, int algo, const DeviceInfo& dev)
{
    if (prec == 0) return false;
    if (algo == 1) return false;
    if (algo == 2) return true;
    const double cu = (double)dev.cus / 256.0;
    const double dense = (double)n * 0.5 * (double)p * (double)p * (prec == 2 ? 3.0 : 1.0) /
                         ((prec == 2 ? 8.2e14 : 6.0e13) * cu);
    const double nb = (double)(p < kSpW ? 1 : p / kSpW);
    const double sparse = (double)n * (5.4e-11 * nb * (nb + 1.0) / 2.0 + 3.9e-13 * 0.5 * (double)m * (double)m) / cu;
    return sparse < dense;
}

// Super-ranges of the sparse form: work items are (super-range, tile), one
// resident per CU; the count is chosen so that the items fill whole rounds of
// the chip (fewer rounds preferred on ties: each item writes one partial tile).
static int sparse_super_ranges(int64_t ntiles, int64_t nchunks, const DeviceInfo& dev)
{
    const int64_t slots = (int64_t)dev.cus;
    int best = 1;
    double best_eff = -1.0;
    for (int R = 1; R <= 64; ++R) {
        int64_t nsr = (R * slots) / ntiles;
        if (nsr < 1) nsr = 1;
        if (nsr > nchunks) nsr = nchunks;
        const int64_t items = nsr * ntiles;
        const double eff = (double)items / (double)(((items + slots - 1) / slots) * slots);
        if (eff > best_eff + 1e-3) {
            best_eff = eff;
            best = (int)nsr;
        }
    }
    return best;
}

static GramPlan gram_plan(int prec, int p, int m, int64_t n, const DeviceInfo& dev, int algo)
{
    GramPlan g;
    g.sparse = use_sparse(prec, p, m, n, algo, dev);
    g.ss_bytes = g.cm_bytes = g.rc_bytes = 0;
    if (g.sparse) {
        g.geom = make_geom(p, kSpW, kSpW);
        g.sa = g.sb = 0;
        const int64_t nchunks = (n + kChunk - 1) / kChunk;
        g.nchunks = nchunks;
        g.nsplit = sparse_super_ranges(g.geom.ntiles, nchunks, dev);
        // a super-range is whole fixed-point ranges (except the last)
        int64_t per = (nchunks + g.nsplit - 1) / g.nsplit;
        per = ((per + kSpRangeChunks - 1) / kSpRangeChunks) * kSpRangeChunks;
        g.nsplit = (int)((nchunks + per - 1) / per);
        g.split_len = per;  // chunks per super-range
        const size_t nn = (size_t)(n > 0 ? n : 0);
        g.off_bytes = 0;
        g.pk_bytes = up256(nn * (size_t)m * 4) + up256(nn * (size_t)m * 2);
        g.bs_bytes = up256((size_t)nchunks * (g.geom.nbc + 1) * 4);
        g.ss_bytes = up256((size_t)nchunks * g.geom.nbc * kChunk * 2);
        g.cm_bytes = up256((size_t)nchunks * 4);
        g.rc_bytes = up256((size_t)((nchunks + kSpRangeChunks - 1) / kSpRangeChunks) * 4);
        g.part_bytes = up256((size_t)g.nsplit * g.geom.ntiles * (size_t)g.geom.tr * g.geom.tc * sizeof(float));
        g.diag_bytes = 0;
        return g;
    }
    g.geom = (prec == 0) ? make_geom(p, kTileF64, kTileF64) : make_geom(p, kTR, kTC);
    g.sa = run_slots(p, m, g.geom.tr);
    g.sb = run_slots(p, m, g.geom.tc);
    if (g.sb > g.sa) g.sb = g.sa;
    const int64_t nchunks = (n + kChunk - 1) / kChunk;
    g.nchunks = nchunks;
    int64_t ns = (prec == 0) ? 1 : (n + kMaxSamplesPerSplit - 1) / kMaxSamplesPerSplit;
    const int64_t want = ((int64_t)dev.cus * 4 + g.geom.ntiles - 1) / g.geom.ntiles;  // enough workgroups
    if (ns < want) ns = want;
    if (ns > nchunks) ns = nchunks;
    if (ns < 1) ns = 1;
    const int64_t chunks_per = (nchunks + ns - 1) / ns;
    g.split_len = chunks_per * kChunk;
    g.nsplit = (int)((n + g.split_len - 1) / g.split_len);
    if (g.nsplit < 1) g.nsplit = 1;
    const size_t nn = (size_t)(n > 0 ? n : 0);
    if (prec == 0) {
        g.off_bytes = up256(nn * (g.geom.nbc + 1) * 4);
        g.pk_bytes = g.bs_bytes = 0;
    } else {
        g.off_bytes = 0;
        g.pk_bytes = up256(nn * (size_t)m * 4) + up256(nn * (size_t)m * 2);  // P (4 B per entry), then OA (2 B)
        g.bs_bytes = up256((size_t)nchunks * (g.geom.nbc + 1) * 4);
    }
    const size_t pe = (prec == 0) ? sizeof(double) : sizeof(float);
    g.part_bytes = up256((size_t)g.nsplit * g.geom.ntiles * (size_t)g.geom.tr * g.geom.tc * pe);
    g.diag_bytes = (prec == 2) ? (size_t)g.nsplit * g.geom.ntiles * (size_t)g.geom.tc * sizeof(double) : 0;
    return g;
}

size_t covariance_workspace(int prec, int p, int m, int64_t n, const DeviceInfo& dev, int algo)
{
    if (n <= 0) return 0;
    GramPlan g = gram_plan(prec, p, m, n, dev, algo);
    return g.off_bytes + g.pk_bytes + g.bs_bytes + g.ss_bytes + g.cm_bytes + g.rc_bytes + g.part_bytes + g.diag_bytes;
}

bool covariance_is_sparse(int prec, int p, int m, int64_t n, const DeviceInfo& dev, int algo)
{
    return use_sparse(prec, p, m, n, algo, dev);
}

template <bool SPLIT, int SA, int SB>
static void launch_mfma_kernel(const GramPlan& g, int64_t grid, const uint32_t* P, const uint16_t* OA,
                               const uint32_t* BS, int m, int64_t n, float* part, double* pdiag, hipStream_t s)
{
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram_mfma<SPLIT, SA, SB>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(MfmaLds<SPLIT>));
        attr_set = true;
    }
    {
        ProfScope ps_(SPLIT ? "gram_bf16x3" : "gram_f32", s);
        hipLaunchKernelGGL((k_gram_mfma<SPLIT, SA, SB>), dim3((unsigned)grid), dim3(256), sizeof(MfmaLds<SPLIT>), s,
                           P, OA, BS, m, g.geom, n, g.nsplit, g.split_len, part, pdiag);
    }
}

template <bool SPLIT>
static void dispatch_mfma(const GramPlan& g, int64_t grid, const uint32_t* P, const uint16_t* OA,
                          const uint32_t* BS, int m, int64_t n, float* part, double* pdiag, hipStream_t s)
{
#define PDS_GRAM_CASE(A, B)                                                                   \
    if (g.sa == A && g.sb == B) {                                                             \
        launch_mfma_kernel<SPLIT, A, B>(g, grid, P, OA, BS, m, n, part, pdiag, s);                    \
        return;                                                                               \
    }
    PDS_GRAM_CASE(1, 1)
    PDS_GRAM_CASE(2, 1)
    PDS_GRAM_CASE(2, 2)
    PDS_GRAM_CASE(4, 1)
    PDS_GRAM_CASE(4, 2)
    PDS_GRAM_CASE(4, 4)
    PDS_GRAM_CASE(8, 1)
    PDS_GRAM_CASE(8, 2)
    PDS_GRAM_CASE(8, 4)
    PDS_GRAM_CASE(8, 8)
#undef PDS_GRAM_CASE
}

constexpr int kLdsMax = 160 * 1024;  // LDS of one workgroup on gfx950

static size_t pack_lds_bytes(int nbc, int nt = 256)
{
    return ((size_t)kChunk * (nbc + 1) + (size_t)kChunk * nbc + (size_t)nt / 64) * 4;
}

static void pack_attrs()
{
    static bool pack_attr = false;
    if (!pack_attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram_pack<false, 0, 256>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)pack_lds_bytes(65536 / kSpW));
        const void* staged[] = {reinterpret_cast<const void*>(&k_gram_pack<true, 0, 256>),
                                reinterpret_cast<const void*>(&k_gram_pack<true, 16, 256>),
                                reinterpret_cast<const void*>(&k_gram_pack<true, 32, 256>),
                                reinterpret_cast<const void*>(&k_gram_pack<true, 32, 512>)};
        for (const void* k : staged) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMax);
        pack_attr = true;
    }
}

static hipError_t launch_pack(const GramPlan& g, int m, const float* vals, const uint16_t* idx, int64_t n,
                              int rowbytes, int eb, int split, uint32_t* P, uint16_t* OA, uint32_t* BS, uint16_t* SS,
                              uint32_t* CM, hipStream_t s)
{
    const bool stage = (size_t)kChunk * m * 2 <= (size_t)kPackStageBytes &&
                       pack_lds_bytes(g.geom.nbc, 512) + kPackStageBytes <= (size_t)kLdsMax &&
                       (reinterpret_cast<uintptr_t>(idx) & 15) == 0;
    const int64_t tot = (int64_t)kChunk * m;  // entries of a full chunk
    const int nt = (stage && tot > 256 * 32) ? 512 : 256;
    // the staged rows take what they need (more workgroups per CU than a fixed 32 KB)
    const size_t lds = pack_lds_bytes(g.geom.nbc, nt) + (stage ? (((size_t)kChunk * m * 2 + 15) & ~(size_t)15) : 0);
    pack_attrs();
    ProfScope ps_("gram_pack", s);
#define PDS_PACK(ST, VR, NT)                                                                                    \
    hipLaunchKernelGGL((k_gram_pack<ST, VR, NT>), dim3((unsigned)g.nchunks), dim3(NT), lds, s, vals, idx, n, m,  \
                       g.geom.tr, g.geom.tc, g.geom.nbc, rowbytes, eb, split, P, OA, BS, SS, CM)
    if (!stage)
        PDS_PACK(false, 0, 256);
    else if (tot <= 256 * 16)
        PDS_PACK(true, 16, 256);
    else if (tot <= 256 * 32)
        PDS_PACK(true, 32, 256);
    else if (tot <= 512 * 32)
        PDS_PACK(true, 32, 512);
    else
        PDS_PACK(true, 0, 256);
#undef PDS_PACK
    return hipGetLastError();
}

hipError_t launch_covariance_accumulate(int prec, int p, int m, const void* vals, const uint16_t* idx, int64_t n,
                                        double* acc, void* ws, size_t ws_bytes, const DeviceInfo& dev,
                                        hipStream_t s, int algo)
{
    (void)ws_bytes;
    if (n <= 0) return hipSuccess;
    GramPlan g = gram_plan(prec, p, m, n, dev, algo);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    void* part = w + g.off_bytes + g.pk_bytes + g.bs_bytes + g.ss_bytes + g.cm_bytes + g.rc_bytes;
    // FP64 diagonal sums: split plans' dense form only
    double* pdiag = (prec == 2 && !g.sparse)
                        ? reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(part) + g.part_bytes)
                        : nullptr;
    const int64_t total = (int64_t)g.geom.ntiles * g.nsplit;
    const int64_t grid = ((total + 7) / 8) * 8;
    hipError_t e;
    if (g.sparse) {
        uint32_t* P = reinterpret_cast<uint32_t*>(w);
        uint16_t* OA = reinterpret_cast<uint16_t*>(w + up256((size_t)n * (size_t)m * 4));
        uint32_t* BS = reinterpret_cast<uint32_t*>(w + g.pk_bytes);
        uint16_t* SS = reinterpret_cast<uint16_t*>(w + g.pk_bytes + g.bs_bytes);
        uint32_t* CM = reinterpret_cast<uint32_t*>(w + g.pk_bytes + g.bs_bytes + g.ss_bytes);
        uint32_t* RC = reinterpret_cast<uint32_t*>(w + g.pk_bytes + g.bs_bytes + g.ss_bytes + g.cm_bytes);
        e = launch_pack(g, m, reinterpret_cast<const float*>(vals), idx, n, 1, 128, 0, P, OA, BS, SS, CM, s);
        if (e != hipSuccess) return e;
        {
            static bool rc_attr = false;
            if (!rc_attr) {
                (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_range_counts),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, 65536 * 2);
                rc_attr = true;
            }
            const int64_t nranges = (g.nchunks + kSpRangeChunks - 1) / kSpRangeChunks;
            ProfScope ps_("range_counts", s);
            hipLaunchKernelGGL(k_range_counts, dim3((unsigned)nranges), dim3(1024), (size_t)((p + 1) / 2) * 4, s, idx,
                               n, m, p, RC);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        static bool sp_attr = false;
        if (!sp_attr) {
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram_sparse),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(SparseLds));
            sp_attr = true;
        }
        const int64_t items = (int64_t)g.geom.ntiles * g.nsplit;
        {
            ProfScope ps_("gram_sparse", s);
            hipLaunchKernelGGL(k_gram_sparse, dim3((unsigned)(((items + 7) / 8) * 8)), dim3(kSpThreads), sizeof(SparseLds),
                               s, P, OA, BS, SS, CM, RC, m, g.geom, g.nchunks, g.nsplit, g.split_len,
                               reinterpret_cast<float*>(part));
        }
    } else if (prec == 0) {
        uint32_t* off = reinterpret_cast<uint32_t*>(w);
        {
            const int64_t threads = n * (int64_t)(g.geom.nbc + 1);
            ProfScope ps_("block_offsets", s);
            hipLaunchKernelGGL(k_block_offsets, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, idx, n, m,
                               g.geom.tc, g.geom.nbc, off);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        ProfScope ps_("gram_f64", s);
        hipLaunchKernelGGL(k_gram_f64, dim3((unsigned)grid), dim3(256), 0, s, reinterpret_cast<const double*>(vals),
                           idx, off, m, g.geom, n, g.nsplit, g.split_len, reinterpret_cast<double*>(part));
    } else {
        uint32_t* P = reinterpret_cast<uint32_t*>(w);
        uint16_t* OA = reinterpret_cast<uint16_t*>(w + up256((size_t)n * (size_t)m * 4));
        uint32_t* BS = reinterpret_cast<uint32_t*>(w + g.pk_bytes);
        const bool split = (prec == 2);
        const int rowbytes = split ? kBfStride * 2 : kF32Stride * 4;
        e = launch_pack(g, m, reinterpret_cast<const float*>(vals), idx, n, rowbytes, split ? 2 : 4, split ? 1 : 0, P,
                        OA, BS, nullptr, nullptr, s);
        if (e != hipSuccess) return e;
        if (split)
            dispatch_mfma<true>(g, grid, P, OA, BS, m, n, reinterpret_cast<float*>(part), pdiag, s);
        else
            dispatch_mfma<false>(g, grid, P, OA, BS, m, n, reinterpret_cast<float*>(part), nullptr, s);
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

hipError_t launch_covariance_finalize(int prec, int p, int lda, int m, int64_t n_total, const double* acc, double* C,
                                      hipStream_t s)
{
    (void)prec;
    const double sdiag = (double)p / ((double)m * (double)n_total);
    const double soff = ((double)p * (double)(p - 1)) / ((double)m * (double)(m - 1) * (double)n_total);
    const int64_t tot = (int64_t)p * p;
    {
        ProfScope ps_("cov_finalize", s);
        hipLaunchKernelGGL(k_cov_finalize, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, acc, p, lda, sdiag,
                           soff, C);
    }
    return hipGetLastError();
}

}  // namespace pds
