// Exact-m sampling without replacement (Sec. I setup; App. B): for each
// sample, the m kept coordinates out of p, uniformly over all m-subsets, by
// Floyd's algorithm (Bentley & Floyd, CACM 1987): for t = p-m .. p-1 draw r
// uniform on {0..t}; keep r, or keep t when r is already kept.  Draws are
// Lemire's method on the sample's own Philox word stream, so the subset of
// sample i is a function of (seed, i) only.
//
// One lane per sample (with at most 32 samples per wave, the upper 32 lanes
// evaluate every other Philox block for the lower ones).  The kept-set
// bitmaps of the wave's samples live in LDS, word w of lane l at
// w * (spw + 1) + l: an odd stride, so both the
// Floyd loop (each lane at its own random word) and the emission below (the
// lanes at consecutive words of one sample) spread over the LDS banks.
// Emission is cooperative, one sample at a time: each lane takes a contiguous
// run of bitmap words, a wave prefix sum of their popcounts gives its output
// position, and the lanes store the ascending indices side by side, so the
// index rows are written with coalesced stores.
#include "pds_device.hpp"
#include "pds_internal.hpp"
#include "pds_sample.hpp"

namespace pds {

// Bitmap budget per 64-lane workgroup: 32 samples (stride 33) at p = 4096, so
// that nine workgroups share a CU and the cooperative emission's latencies are
// covered by the other waves (64 samples per wave, four waves per CU, leave
// them exposed: 2.6 against 1.9 ms at n = 2^20, p = 4096, m = 410).
constexpr int kSampleLdsBytes = 16896;

__global__ __launch_bounds__(64) void k_sample_indices(uint64_t seed, int p, int m, int64_t n, uint64_t i0,
                                                       int spw, int words, uint16_t* __restrict__ idx)
{
    extern __shared__ uint32_t bitmap[];  // [words][spw + 1]
    const int lane = threadIdx.x;
    const int stride = spw + 1;
    const int64_t r = (int64_t)blockIdx.x * spw + lane;

    for (int e = lane; e < words * stride; e += 64) bitmap[e] = 0u;
    __syncthreads();
    if (spw <= 32) {
        // lane q + 32 evaluates every other Philox block for lane q's sample
        const int q = lane & 31;
        const int64_t rq = (int64_t)blockIdx.x * spw + q;
        const bool owner = lane < 32 && q < spw && rq < n;
        floyd_bitmap_pair(seed, i0 + (uint64_t)rq, p, m, bitmap, stride, q, owner);
    } else if (lane < spw && r < n) {
        floyd_bitmap(seed, i0 + (uint64_t)r, p, m, bitmap, stride, lane);
    }
    __syncthreads();

    // cooperative, coalesced emission of each sample's ascending index row
    for (int k = 0; k < spw; ++k) {
        const int64_t rk = (int64_t)blockIdx.x * spw + k;
        if (rk >= n) break;
        uint16_t* out = idx + rk * (int64_t)m;
        emit_sorted(bitmap, stride, k, words, lane, [&](int pos, int c) { out[pos] = (uint16_t)c; });
    }
}

hipError_t launch_sample_indices(uint64_t seed, int p, int m, int64_t n, uint64_t i0, uint16_t* idx,
                                 const DeviceInfo& dev, hipStream_t s)
{
    (void)dev;
    if (n <= 0) return hipSuccess;
    const int words = (p + 31) / 32;
    int spw = kSampleLdsBytes / (words * 4) - 1;
    if (spw > 32) spw = 32;  // lane pairs (at most 32 samples per wave)
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
