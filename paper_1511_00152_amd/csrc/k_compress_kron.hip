// Split-BF16 matrix-core transform for the split plan at p = 4096 (Sec. III,
// eq. ROS): H_4096 = H_64 (x) H_64, so for the row-major 64 x 64 reshape X of
// D x (X[r][c] = D_{64r+c} x_{64r+c}) the transform is Y = H_64 X H_64 with
// Y[r][c] = y_{64r+c} (times 1/64, applied as 1/8 in each factor's +-1
// entries).  Both factors are products on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation:
//   stage 1  Z = X H_64  (A operand: 8 consecutive values of a row of X,
//            straight from memory; B operand: constant +-1/8 entries of H_64)
//   stage 2  Y = H_64 Z  (B operand: Z as it sits in stage 1's accumulator
//            registers; the K index runs over Z's rows in the order those
//            registers hold them, and the constant A operand H_64[r'][k] uses
//            the same order, so no data moves between the stages).
// Every FP32 operand is split exactly into three BF16 parts by truncation,
// v = hi + mid + lo (8 + 8 + 8 significand bits), so each product is exact and
// the only rounding is the FP32 accumulation.  The result goes to LDS once for
// the gather of the kept entries.  One wave per sample, persistent.
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

typedef __bf16 kbf16x8 __attribute__((ext_vector_type(8)));
typedef float kf32x16 __attribute__((ext_vector_type(16)));

struct Parts8 {
    uint32_t w[4];  // 8 bf16 values, two per word, lower index in the low half
};

__device__ inline kbf16x8 as_bf16x8(const Parts8& q)
{
    return __builtin_bit_cast(kbf16x8, q);
}

// Exact three-way split of 8 floats into bf16 hi, mid, lo parts.
__device__ inline void split3(const float (&v)[8], Parts8& hi, Parts8& mid, Parts8& lo)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t a = __float_as_uint(v[2 * k]), b = __float_as_uint(v[2 * k + 1]);
        const uint32_t ah = a & 0xFFFF0000u, bh = b & 0xFFFF0000u;
        const float ra = v[2 * k] - __uint_as_float(ah), rb = v[2 * k + 1] - __uint_as_float(bh);
        const uint32_t am = __float_as_uint(ra) & 0xFFFF0000u, bm = __float_as_uint(rb) & 0xFFFF0000u;
        const float la = ra - __uint_as_float(am), lb = rb - __uint_as_float(bm);
        hi.w[k] = (ah >> 16) | bh;
        mid.w[k] = (am >> 16) | bm;
        lo.w[k] = (__float_as_uint(la) >> 16) | (__float_as_uint(lb) & 0xFFFF0000u);
    }
}

// bf16 bits of H_64[a][b] / 8 (+-0.125): each stage carries half of the
// transform's 1/64, which, a power of two, changes no rounding
__device__ inline uint32_t hsign_bits(int a, int b)
{
    return (__popc(a & b) & 1) ? 0xBE00u : 0x3E00u;
}

// stage-2 K order: logical slot (h, j) of K-block (rb, kk) is row
// 32 rb + 16 kk + 8 (j / 4) + 4 h + (j % 4) of Z (the accumulator layout)
__device__ inline int zrow(int rb, int kk, int h, int j) { return 32 * rb + 16 * kk + 8 * (j >> 2) + 4 * h + (j & 3); }

constexpr int kKronP = 4096;
constexpr int kKronPad = kKronP + kKronP / 32;
constexpr int kKronIdxRegs = 8;  // kept indices per lane requested ahead (m <= 512 entirely)

// Half rb of a lane's share of row x (8 x 16 B): element 64 (32 rb + i32) +
// 16 kb + 8 h + j in cur[8 rb + 2 kb + j / 4], the layout stage 1 consumes
__device__ inline void kron_load_half(float4 (&cur)[16], const float* __restrict__ x, int rb, int i32, int h)
{
#pragma unroll
    for (int q = 8 * rb; q < 8 * rb + 8; ++q)
        cur[q] = reinterpret_cast<const float4*>(x + 64 * (32 * rb + i32) + 16 * ((q >> 1) & 3) + 8 * h)[q & 1];
}

__global__ __launch_bounds__(256, 2) void k_compress_kron4096(uint64_t seed, int m, const float* __restrict__ X,
                                                              int64_t n, int64_t ldx, const uint16_t* __restrict__ idx,
                                                              float* __restrict__ vals)
{
    __shared__ float ybuf[4][kKronPad];
    __shared__ uint32_t negbits[kKronP / 32];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int i32 = lane & 31, h = lane >> 5;
    float* yb = ybuf[wave];

    for (int b = tid; b < kKronP / 256; b += 256) {
        u64x4 blk = sign_block(seed, (uint64_t)b);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            negbits[b * 8 + 2 * w] = (uint32_t)blk.w[w];
            negbits[b * 8 + 2 * w + 1] = (uint32_t)(blk.w[w] >> 32);
        }
    }
    __syncthreads();

    // Constant +-1/8 operands.  Stage 1's B operand at (kb, cb) holds
    // H[16 kb + 8 h + j][32 cb + i32], j < 8; the row index splits into
    // disjoint bits 16 kb + 8 h and j, so the entry is the sign of
    // popc((16 kb + 8 h) & c) times the sign of popc(j & c): one 8-entry
    // pattern per lane (hb_base) and one sign per (kb, cb) (hb_neg).  Stage 2's
    // A operand at (rb2, rb, kk) holds H[32 rb2 + i32][zrow(rb, kk, h, j)]; the
    // column splits into 32 rb + 16 kk + 4 h and 8 (j / 4) + j % 4 likewise
    // (ha_base, ha_neg).  A sign flips the sign bits of all eight bf16 values.
    uint32_t hb_base[4], ha_base[4], hb_neg[8], ha_neg[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        hb_base[k] = hsign_bits(2 * k, i32) | (hsign_bits(2 * k + 1, i32) << 16);
        ha_base[k] = hsign_bits(i32, zrow(0, 0, 0, 2 * k)) | (hsign_bits(i32, zrow(0, 0, 0, 2 * k + 1)) << 16);
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
            hb_neg[kb * 2 + cb] = (__popc((16 * kb + 8 * h) & (32 * cb + i32)) & 1) ? 0x80008000u : 0u;
#pragma unroll
    for (int rb2 = 0; rb2 < 2; ++rb2)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int kk = 0; kk < 2; ++kk)
                ha_neg[(rb2 * 2 + rb) * 2 + kk] =
                    (__popc((32 * rb2 + i32) & (32 * rb + 16 * kk + 4 * h)) & 1) ? 0x80008000u : 0u;

    // this lane's signs: element 64 (32 rb + i32) + 16 kb + 8 h + j
    uint64_t negmask = 0;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int e = 64 * (32 * rb + i32) + 16 * kb + 8 * h + j;
                negmask |= (uint64_t)((negbits[e >> 5] >> (e & 31)) & 1u) << (32 * rb + 8 * kb + j);
            }

    // A lane's share of a row (16 x 16 B) is requested as the previous row's
    // registers free up: half once stage 1 has consumed it, half once stage 2
    // has consumed half of Z, so the loads fly during stage 2 and the gather
    // of the previous sample.  The first kKronIdxRegs x 64 kept indices of a
    // sample are requested when its stage 1 starts.
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    float4 cur[16];
    if ((int64_t)blockIdx.x * 4 + wave < n) {
        kron_load_half(cur, X + ((int64_t)blockIdx.x * 4 + wave) * ldx, 0, i32, h);
        kron_load_half(cur, X + ((int64_t)blockIdx.x * 4 + wave) * ldx, 1, i32, h);
    }
    for (int64_t i = (int64_t)blockIdx.x * 4 + wave; i < n; i += nwaves) {
        const uint16_t* ix = idx + i * (int64_t)m;
        uint32_t ixr[kKronIdxRegs];
#pragma unroll
        for (int u = 0; u < kKronIdxRegs; ++u) ixr[u] = lane + 64 * u < m ? ix[lane + 64 * u] : 0u;
        // the next row (this one again at the wave's last sample, a harmless reload)
        const float* xn = X + (i + nwaves < n ? i + nwaves : i) * ldx;
        // the sign bits are re-read from this register every sample: otherwise
        // the 64 per-element sign words are hoisted out of the loop and take
        // 64 registers for the whole kernel
        asm volatile("" : "+v"(negmask));
        // stage 1: Z = X H
        kf32x16 z[2][2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int r = 0; r < 16; ++r) z[rb][cb][r] = 0.0f;
        // each split-and-multiply block below is scheduled on its own, which
        // bounds the registers live at once
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const float4 u0 = cur[rb * 8 + kb * 2], u1 = cur[rb * 8 + kb * 2 + 1];
                float v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const uint32_t neg = (uint32_t)((negmask >> (32 * rb + 8 * kb + j)) & 1u);
                    v[j] = __uint_as_float(__float_as_uint(v[j]) ^ (neg << 31));
                }
                Parts8 ph, pm, pl;
                split3(v, ph, pm, pl);
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    Parts8 hw;
#pragma unroll
                    for (int k = 0; k < 4; ++k) hw.w[k] = hb_base[k] ^ hb_neg[kb * 2 + cb];
                    const kbf16x8 hb = as_bf16x8(hw);
                    z[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(ph), hb, z[rb][cb], 0, 0, 0);
                    z[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(pm), hb, z[rb][cb], 0, 0, 0);
                    z[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(pl), hb, z[rb][cb], 0, 0, 0);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        kron_load_half(cur, xn, 0, i32, h);
        __builtin_amdgcn_sched_barrier(0);
        // stage 2: Y = H Z, K over Z's rows in accumulator order.  Column block
        // cb of Y needs only column block cb of Z, so each is finished and
        // written out (Y[r][c] = y_{64 r + c}; the lane holds column
        // 32 cb + i32 of rows 32 rb2 + 8 (v / 4) + 4 h + v % 4) before the next.
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            kf32x16 y[2];
#pragma unroll
            for (int rb2 = 0; rb2 < 2; ++rb2)
#pragma unroll
                for (int r = 0; r < 16; ++r) y[rb2][r] = 0.0f;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int kk = 0; kk < 2; ++kk) {
                    float v[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) v[j] = z[rb][cb][8 * kk + j];
                    Parts8 ph, pm, pl;
                    split3(v, ph, pm, pl);
#pragma unroll
                    for (int rb2 = 0; rb2 < 2; ++rb2) {
                        Parts8 aw;
#pragma unroll
                        for (int k = 0; k < 4; ++k) aw.w[k] = ha_base[k] ^ ha_neg[(rb2 * 2 + rb) * 2 + kk];
                        const kbf16x8 ha = as_bf16x8(aw);
                        y[rb2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ha, as_bf16x8(ph), y[rb2], 0, 0, 0);
                        y[rb2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ha, as_bf16x8(pm), y[rb2], 0, 0, 0);
                        y[rb2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ha, as_bf16x8(pl), y[rb2], 0, 0, 0);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            if (cb == 0) {
                kron_load_half(cur, xn, 1, i32, h);
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int rb2 = 0; rb2 < 2; ++rb2)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int e = 64 * (32 * rb2 + 8 * (v >> 2) + 4 * h + (v & 3)) + 32 * cb + i32;
                    yb[lds_pad<float>(e)] = y[rb2][v];
                }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float* out = vals + i * (int64_t)m;
#pragma unroll
        for (int u = 0; u < kKronIdxRegs; ++u)
            if (lane + 64 * u < m) out[lane + 64 * u] = yb[lds_pad<float>((int)ixr[u])];
        for (int t = lane + 64 * kKronIdxRegs; t < m; t += 64) out[t] = yb[lds_pad<float>((int)ix[t])];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

bool kron_transform_ok(int p, const void* X, int64_t ldx)
{
    return p == kKronP && ((uintptr_t)X % 16 == 0) && ((ldx * 4) % 16 == 0);
}

hipError_t launch_compress_kron(uint64_t seed, int m, const float* X, int64_t n, int64_t ldx, const uint16_t* idx,
                                float* vals, const DeviceInfo& dev, hipStream_t s)
{
    static int per_cu = 0;
    if (per_cu == 0) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_compress_kron4096, 256, 0) != hipSuccess || b < 1)
            b = 1;
        per_cu = b;
    }
    int64_t grid = (int64_t)dev.cus * per_cu;
    const int64_t need = (n + 3) / 4;
    if (grid > need) grid = need;
    {
        ProfScope ps_("compress", s);
        hipLaunchKernelGGL(k_compress_kron4096, dim3((unsigned)grid), dim3(256), 0, s, seed, m, X, n, ldx, idx, vals);
    }
    return hipGetLastError();
}

}  // namespace pds
