// Device-side building blocks shared by the kernels of libpds (gfx950).
//
// Random numbers: the method draws one sign per coordinate and, per sample,
// m distinct coordinates.  Both come from the counter-based generator
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11), implemented here from
// its published definition, so every draw is a pure function of
// (seed, stream, index) and independent of the launch shape.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pds {

// Philox4x64 round constants (multipliers and Weyl key increments of the
// published generator).
constexpr uint64_t kPhiloxMul0 = 0xD2E7470EE14C6C93ULL;
constexpr uint64_t kPhiloxMul1 = 0xCA5A826395121157ULL;
constexpr uint64_t kPhiloxKeyInc0 = 0x9E3779B97F4A7C15ULL;
constexpr uint64_t kPhiloxKeyInc1 = 0xBB67AE8584CAA73BULL;

struct u64x4 {
    uint64_t w[4];
};

__host__ __device__ inline void mul_hi_lo(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo)
{
#if defined(__HIP_DEVICE_COMPILE__)
    // four 32 x 32 -> 64 partial products with the carries folded into the
    // multiply-adds (none of the sums can exceed 2^64 - 1)
    const uint32_t al = (uint32_t)a, ah = (uint32_t)(a >> 32), bl = (uint32_t)b, bh = (uint32_t)(b >> 32);
    const uint64_t p0 = (uint64_t)al * bl;
    const uint64_t p1 = (uint64_t)al * bh + (p0 >> 32);
    const uint64_t p2 = (uint64_t)ah * bl + (uint32_t)p1;
    hi = (uint64_t)ah * bh + (p1 >> 32) + (p2 >> 32);
    lo = (p2 << 32) | (uint32_t)p0;
#else
    unsigned __int128 p = (unsigned __int128)a * b;
    lo = (uint64_t)p;
    hi = (uint64_t)(p >> 64);
#endif
}

// One Philox4x64-10 block for counter (c0, c1, c2, c3) and key (k0, k1).
__host__ __device__ inline u64x4 philox_block(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                              uint64_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kPhiloxKeyInc0;
            k1 += kPhiloxKeyInc1;
        }
        uint64_t h0, l0, h1, l1;
        mul_hi_lo(kPhiloxMul0, c0, h0, l0);
        mul_hi_lo(kPhiloxMul1, c2, h1, l1);
        uint64_t n0 = h1 ^ c1 ^ k0;
        uint64_t n2 = h0 ^ c3 ^ k1;
        c0 = n0;
        c1 = l1;
        c2 = n2;
        c3 = l0;
    }
    u64x4 out;
    out.w[0] = c0;
    out.w[1] = c1;
    out.w[2] = c2;
    out.w[3] = c3;
    return out;
}

// Sign stream: D_j = -1 iff bit (j mod 64) of 64-bit word ((j/64) mod 4) of
// block (j/256, 0, 1, 0) under key (seed, 0) is set.
__host__ __device__ inline u64x4 sign_block(uint64_t seed, uint64_t block)
{
    return philox_block(block, 0, 1, 0, seed, 0);
}

// Per-sample 32-bit word stream for the sampler: blocks (b, i, 0, 0) under
// key (seed, 0); each 64-bit word yields its low half, then its high half.
struct WordStream {
    uint64_t seed, sample, block;
    uint64_t buf[4];
    int pos;  // 0..8, 8 = empty

    __device__ inline void init(uint64_t seed_, uint64_t sample_)
    {
        seed = seed_;
        sample = sample_;
        block = 0;
        pos = 8;
    }
    // position the stream at 32-bit word index widx
    __device__ inline void seek(uint64_t widx)
    {
        block = widx >> 3;
        pos = 8;
        const int skip = (int)(widx & 7);
        if (skip) {
            u64x4 b = philox_block(block, sample, 0, 0, seed, 0);
            buf[0] = b.w[0];
            buf[1] = b.w[1];
            buf[2] = b.w[2];
            buf[3] = b.w[3];
            ++block;
            pos = skip;
        }
    }
    __device__ inline uint32_t next()
    {
        if (pos == 8) {
            u64x4 b = philox_block(block, sample, 0, 0, seed, 0);
            buf[0] = b.w[0];
            buf[1] = b.w[1];
            buf[2] = b.w[2];
            buf[3] = b.w[3];
            ++block;
            pos = 0;
        }
        // select word pos>>1 without dynamic register indexing
        uint64_t w = (pos < 4) ? ((pos < 2) ? buf[0] : buf[1]) : ((pos < 6) ? buf[2] : buf[3]);
        uint32_t r = (pos & 1) ? (uint32_t)(w >> 32) : (uint32_t)w;
        ++pos;
        return r;
    }
};

// Uniform integer in [0, range), range >= 1, by Lemire's multiply-and-reject
// method (ACM TOMACS 2019): the high half of word * range, rejecting the
// (2^32 mod range) words whose low half falls below that count.
__device__ inline uint32_t uniform_below(WordStream& s, uint32_t range)
{
    uint64_t prod = (uint64_t)s.next() * range;
    uint32_t low = (uint32_t)prod;
    if (low < range) {
        uint32_t thresh = (0u - range) % range;
        while (low < thresh) {
            prod = (uint64_t)s.next() * range;
            low = (uint32_t)prod;
        }
    }
    return (uint32_t)(prod >> 32);
}

// Padded LDS address of element e of a transform buffer: one extra 32-bit
// slot every 32 elements spreads strided accesses over the LDS banks.
template <typename T>
__host__ __device__ constexpr int lds_pad(int e)
{
    return (sizeof(T) == 4) ? (e + (e >> 5)) : (e + (e >> 4));
}

}  // namespace pds
