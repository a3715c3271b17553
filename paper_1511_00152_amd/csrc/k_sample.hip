// Exact-m sampling without replacement (Sec. I setup; App. B): for each
// sample, the m kept coordinates out of p, uniformly over all m-subsets, by
// Floyd's algorithm (Bentley & Floyd, CACM 1987): for t = p-m .. p-1 draw r
// uniform on {0..t}; keep r, or keep t when r is already kept.  Draws are
// Lemire's method on the sample's own Philox word stream, so the subset of
// sample i is a function of (seed, i) only.
//
// One lane per sample.  The kept-set bitmaps of the wave's samples live in
// LDS, word w of lane l at w * (spw + 1) + l: an odd stride, so both the
// Floyd loop (each lane at its own random word) and the emission below (the
// lanes at consecutive words of one sample) spread over the LDS banks.
// Emission is cooperative, one sample at a time: each lane takes a contiguous
// run of bitmap words, a wave prefix sum of their popcounts gives its output
// position, and the lanes store the ascending indices side by side, so the
// index rows are written with coalesced stores.
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

constexpr int kSampleLdsBytes = 34816;  // 64 samples x 128 words x stride 65 at p = 4096

__device__ inline int wave_exclusive_scan(int v, int lane)
{
    int incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    return incl - v;
}

__global__ __launch_bounds__(64) void k_sample_indices(uint64_t seed, int p, int m, int64_t n, uint64_t i0,
                                                       int spw, int words, uint16_t* __restrict__ idx)
{
    extern __shared__ uint32_t bitmap[];  // [words][spw + 1]
    const int lane = threadIdx.x;
    const int stride = spw + 1;
    const int64_t r = (int64_t)blockIdx.x * spw + lane;

    for (int e = lane; e < words * stride; e += 64) bitmap[e] = 0u;
    __syncthreads();

    if (lane < spw && r < n) {
        const uint64_t sample = i0 + (uint64_t)r;
        // Fast path: draw t uses word t - (p - m) of the stream while no draw
        // has been rejected; the Philox block after the current one is computed
        // before the current block's set updates, so its arithmetic overlaps
        // the LDS round trips.  At the first rejection (probability below
        // range / 2^32 per draw) the lane continues on the exact sequential
        // stream from the next word.
        uint64_t blk = 0;
        u64x4 cur = philox_block(0, sample, 0, 0, seed, 0);
        int t = p - m;
        int64_t rejected_word = -1;
        while (t < p) {
            const u64x4 nxt = philox_block(blk + 1, sample, 0, 0, seed, 0);
            uint32_t w[8];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                w[2 * q] = (uint32_t)cur.w[q];
                w[2 * q + 1] = (uint32_t)(cur.w[q] >> 32);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (t < p && rejected_word < 0) {
                    const uint32_t range = (uint32_t)(t + 1);
                    const uint64_t prod = (uint64_t)w[q] * range;
                    const uint32_t low = (uint32_t)prod;
                    if (low < range && low < (0u - range) % range) {
                        rejected_word = (int64_t)(blk * 8 + q);
                    } else {
                        const uint32_t c = (uint32_t)(prod >> 32);
                        uint32_t* wc = &bitmap[(c >> 5) * stride + lane];
                        const uint32_t bit = 1u << (c & 31);
                        const uint32_t old = *wc;
                        if (old & bit)
                            bitmap[((uint32_t)t >> 5) * stride + lane] |= 1u << (t & 31);
                        else
                            *wc = old | bit;
                        ++t;
                    }
                }
            }
            if (rejected_word >= 0) break;
            cur = nxt;
            ++blk;
        }
        if (rejected_word >= 0) {
            WordStream ws;
            ws.init(seed, sample);
            ws.seek((uint64_t)rejected_word + 1);
            // finish the rejected draw: Lemire redraws with the same range
            {
                const uint32_t range = (uint32_t)(t + 1);
                const uint32_t thresh = (0u - range) % range;
                uint64_t prod;
                uint32_t low;
                do {
                    prod = (uint64_t)ws.next() * range;
                    low = (uint32_t)prod;
                } while (low < thresh);
                const uint32_t c = (uint32_t)(prod >> 32);
                uint32_t* wc = &bitmap[(c >> 5) * stride + lane];
                const uint32_t bit = 1u << (c & 31);
                if (*wc & bit)
                    bitmap[((uint32_t)t >> 5) * stride + lane] |= 1u << (t & 31);
                else
                    *wc |= bit;
                ++t;
            }
            for (; t < p; ++t) {
                const uint32_t c = uniform_below(ws, (uint32_t)(t + 1));
                uint32_t* wc = &bitmap[(c >> 5) * stride + lane];
                const uint32_t bit = 1u << (c & 31);
                if (*wc & bit)
                    bitmap[((uint32_t)t >> 5) * stride + lane] |= 1u << (t & 31);
                else
                    *wc |= bit;
            }
        }
    }
    __syncthreads();

    // cooperative, coalesced emission of each sample's ascending index row
    const int wpl = (words + 63) / 64;  // bitmap words per lane
    const int w0 = lane * wpl;
    for (int k = 0; k < spw; ++k) {
        const int64_t rk = (int64_t)blockIdx.x * spw + k;
        if (rk >= n) break;
        int cnt = 0;
        for (int q = 0; q < wpl; ++q)
            if (w0 + q < words) cnt += __popc(bitmap[(w0 + q) * stride + k]);
        int pos = wave_exclusive_scan(cnt, lane);
        uint16_t* out = idx + rk * (int64_t)m;
        for (int q = 0; q < wpl; ++q) {
            if (w0 + q >= words) break;
            uint32_t bits = bitmap[(w0 + q) * stride + k];
            while (bits) {
                int b = __builtin_ctz(bits);
                out[pos++] = (uint16_t)((w0 + q) * 32 + b);
                bits &= bits - 1u;
            }
        }
    }
}

hipError_t launch_sample_indices(uint64_t seed, int p, int m, int64_t n, uint64_t i0, uint16_t* idx,
                                 const DeviceInfo& dev, hipStream_t s)
{
    (void)dev;
    if (n <= 0) return hipSuccess;
    const int words = (p + 31) / 32;
    int spw = kSampleLdsBytes / (words * 4) - 1;
    if (spw > 64) spw = 64;
    if (spw < 1) spw = 1;
    const size_t lds = (size_t)words * (spw + 1) * 4;
    const int64_t blocks = (n + spw - 1) / spw;
    {
        ProfScope ps_("sample_indices", s);
        hipLaunchKernelGGL(k_sample_indices, dim3((unsigned)blocks), dim3(64), lds, s, seed, p, m, n, i0, spw, words,
                       idx);
    }
    return hipGetLastError();
}

}  // namespace pds
