// Exact-m sampling without replacement (Sec. I setup; App. B): for each
// sample, the m kept coordinates out of p, uniformly over all m-subsets, by
// Floyd's algorithm (Bentley & Floyd, CACM 1987): for t = p-m .. p-1 draw r
// uniform on {0..t}; keep r, or keep t when r is already kept.  Draws are
// Lemire's method on the sample's own Philox word stream, so the subset of
// sample i is a function of (seed, i) only.
//
// One lane per sample.  The kept-set bitmaps of the wave's samples live in
// LDS, word-interleaved across lanes (word w of lane l at w * spw + l) so that
// lanes touching arbitrary words of their own bitmaps hit distinct banks.
// The ascending index list is emitted by scanning the bitmap.
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

constexpr int kSampleLdsBytes = 32768;

__global__ __launch_bounds__(64) void k_sample_indices(uint64_t seed, int p, int m, int64_t n, uint64_t i0,
                                                       int spw, int words, uint16_t* __restrict__ idx)
{
    extern __shared__ uint32_t bitmap[];  // [words][spw]
    const int lane = threadIdx.x;
    const int64_t r = (int64_t)blockIdx.x * spw + lane;

    for (int e = lane; e < words * spw; e += 64) bitmap[e] = 0u;
    __syncthreads();

    if (lane < spw && r < n) {
        WordStream ws;
        ws.init(seed, i0 + (uint64_t)r);
        for (int t = p - m; t < p; ++t) {
            uint32_t c = uniform_below(ws, (uint32_t)(t + 1));
            uint32_t* wc = &bitmap[(c >> 5) * spw + lane];
            uint32_t bit = 1u << (c & 31);
            uint32_t cur = *wc;
            if (cur & bit) {
                bitmap[((uint32_t)t >> 5) * spw + lane] |= 1u << (t & 31);
            } else {
                *wc = cur | bit;
            }
        }
        uint16_t* out = idx + r * (int64_t)m;
        int c = 0;
        for (int w = 0; w < words; ++w) {
            uint32_t bits = bitmap[w * spw + lane];
            while (bits) {
                int b = __builtin_ctz(bits);
                out[c++] = (uint16_t)(w * 32 + b);
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
    int spw = kSampleLdsBytes / (words * 4);
    if (spw > 64) spw = 64;
    if (spw < 1) spw = 1;
    const size_t lds = (size_t)words * spw * 4;
    const int64_t blocks = (n + spw - 1) / spw;
    hipLaunchKernelGGL(k_sample_indices, dim3((unsigned)blocks), dim3(64), lds, s, seed, p, m, n, i0, spw, words,
                       idx);
    return hipGetLastError();
}

}  // namespace pds
