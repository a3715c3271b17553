// K-means++ seeding on compressed data (Alg. 1 seeds its rounds with
// K-means++; Arthur & Vassilvitskii's D^2 sampling with the sparsified
// distance of Sec. VI): the first center is a uniformly chosen sample, each
// next one is sample i with probability D(i)^2 / sum_j D(j)^2, D(i)^2 the
// smallest distance of sample i over its own kept coordinates to the centers
// chosen so far.  A chosen sample's center is its zero-filled compressed
// vector.  Uniform doubles u = (w >> 11) 2^-53 from the 64-bit words of
// Philox4x64-10 blocks with key (seed, 0) and counter (b, 0, 2, 0), one word
// per center in order.
//
// Per center, two launches, no host round trip:
//   select  one workgroup: u; the first center from u n; later ones from the
//           prefix sums of D^2 (per-block sums scanned in a fixed order, then
//           the chosen block's samples in ascending order); writes the
//           zero-filled center row
//   dist    one thread per sample: the distance to the newest center over the
//           sample's kept coordinates in ascending order with fused
//           multiply-adds (center row in LDS; the rows staged through LDS in
//           chunks of entries so the loads stay coalesced), D^2 = min(D^2, d);
//           per-block sums of D^2 in a fixed order
// The distances are those of a sequential FP64 loop; only the order of the
// prefix sums differs from a sequential scan, which can move a draw that
// lands within rounding of a boundary between two samples.
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

constexpr int kPPDistThreads = 256;    // samples per dist workgroup (one block of the prefix sums)
constexpr int kPPSelThreads = 1024;
constexpr int kPPCenterLds = 65536;    // center row in LDS up to this many bytes

__device__ inline double pp_uniform(uint64_t seed, uint64_t rep, int k)
{
    const u64x4 b = philox_block((uint64_t)(k >> 2), rep, 2, 0, seed, 0);
    return (double)(b.w[k & 3] >> 11) * (1.0 / 9007199254740992.0);
}

// Entries of a chunk staged per sample (32 FP32 or 16 FP64 values).
template <typename T>
struct PPChunk {
    static constexpr int E = sizeof(T) == 8 ? 16 : 32;
    static constexpr size_t bytes = (size_t)kPPDistThreads * (E + 1) * (sizeof(T) + sizeof(uint32_t));
};

// One thread per sample; the workgroup's 256 rows are staged through LDS a
// chunk of entries at a time with loads spread over the rows' contiguous
// entries, then each thread adds its own row's terms in ascending order.
template <typename T, bool LDS>
__global__ __launch_bounds__(kPPDistThreads) void k_pp_dist(const T* __restrict__ vals,
                                                           const uint16_t* __restrict__ idx, int64_t n, int m,
                                                           int p, const double* __restrict__ center, int first,
                                                           double* __restrict__ d2, double* __restrict__ bsum)
{
    constexpr int E = PPChunk<T>::E;
    extern __shared__ __align__(16) unsigned char pp_sh[];
    __shared__ double red[kPPDistThreads];
    const double* c = center;
    size_t off = 0;
    if (LDS) {
        double* cl = reinterpret_cast<double*>(pp_sh);
        for (int j = threadIdx.x; j < p; j += kPPDistThreads) cl[j] = center[j];
        c = cl;
        off = (size_t)p * sizeof(double);
    }
    T* sv = reinterpret_cast<T*>(pp_sh + off);
    uint32_t* si = reinterpret_cast<uint32_t*>(pp_sh + off + (size_t)kPPDistThreads * (E + 1) * sizeof(T));
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * kPPDistThreads;
    const int rows = n - i0 < kPPDistThreads ? (int)(n - i0) : kPPDistThreads;
    // a thread's share of a chunk: E entries, all loads in flight together;
    // the next chunk's loads are issued before the current chunk is summed
    T rv[E];
    uint32_t ri[E];
    auto load = [&](int e0) {
        const int ne = m - e0 < E ? m - e0 : E;
#pragma unroll
        for (int sidx = 0; sidx < E; ++sidx) {
            const int q = t + sidx * kPPDistThreads;
            const int r = q / E, cc = q % E;
            if (r < rows && cc < ne) {
                const int64_t g = (i0 + r) * m + e0 + cc;
                rv[sidx] = vals[g];
                ri[sidx] = idx[g];
            }
        }
    };
    double d = 0.0;
    load(0);
    for (int e0 = 0; e0 < m; e0 += E) {
        const int ne = m - e0 < E ? m - e0 : E;
        __syncthreads();
#pragma unroll
        for (int sidx = 0; sidx < E; ++sidx) {
            const int q = t + sidx * kPPDistThreads;
            const int r = q / E, cc = q % E;
            if (r < rows && cc < ne) {
                sv[r * (E + 1) + cc] = rv[sidx];
                si[r * (E + 1) + cc] = ri[sidx];
            }
        }
        __syncthreads();
        if (e0 + E < m) load(e0 + E);
        if (t < rows) {
            for (int cc = 0; cc < ne; ++cc) {
                const uint32_t j = si[t * (E + 1) + cc];
                const double diff = (double)sv[t * (E + 1) + cc] - (j < (uint32_t)p ? c[j] : 0.0);
                d = fma(diff, diff, d);
            }
        }
    }
    double v = 0.0;
    if (t < rows) {
        const int64_t i = i0 + t;
        if (!first) {
            const double old = d2[i];
            if (!(d < old)) d = old;
        }
        d2[i] = d;
        v = d;
    }
    red[t] = v;
    __syncthreads();
    for (int s = kPPDistThreads / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    if (t == 0) bsum[blockIdx.x] = red[0];
}

// One workgroup.  Thread t owns the consecutive blocks [t*per, (t+1)*per).
template <typename T>
__global__ __launch_bounds__(kPPSelThreads) void k_pp_select(const T* __restrict__ vals,
                                                            const uint16_t* __restrict__ idx, int64_t n, int m,
                                                            int p, uint64_t seed, uint64_t rep, int k,
                                                            const double* __restrict__ d2,
                                                            const double* __restrict__ bsum, int64_t nb,
                                                            double* __restrict__ centers,
                                                            int64_t* __restrict__ chosen)
{
    __shared__ double part[kPPSelThreads];
    __shared__ double scan[kPPSelThreads];
    __shared__ int64_t pick;
    const int t = threadIdx.x;
    const double u = pp_uniform(seed, rep, k);
    if (k == 0) {
        if (t == 0) {
            int64_t c = (int64_t)(u * (double)n);
            if (c >= n) c = n - 1;
            pick = c;
        }
    } else {
        const int64_t per = (nb + kPPSelThreads - 1) / kPPSelThreads;
        const int64_t b0 = t * per;
        int64_t b1 = b0 + per;
        if (b1 > nb) b1 = nb;
        double s = 0.0;
        for (int64_t b = b0; b < b1; ++b) s += bsum[b];
        part[t] = s;
        __syncthreads();
        // inclusive scan of the thread sums (Hillis-Steele, fixed order)
        scan[t] = part[t];
        __syncthreads();
        for (int off = 1; off < kPPSelThreads; off <<= 1) {
            const double add = t >= off ? scan[t - off] : 0.0;
            __syncthreads();
            scan[t] += add;
            __syncthreads();
        }
        const double total = scan[kPPSelThreads - 1];
        const double target = u * total;
        if (t == 0) pick = n - 1;
        __syncthreads();
        const double before = t > 0 ? scan[t - 1] : 0.0;
        // the first thread whose inclusive prefix exceeds the target walks its
        // blocks, then the chosen block's samples, in ascending order
        if (scan[t] > target && !(before > target)) {
            double run = before;
            int64_t bsel = b1 - 1;
            for (int64_t b = b0; b < b1; ++b) {
                if (run + bsum[b] > target) {
                    bsel = b;
                    break;
                }
                run += bsum[b];
            }
            const int64_t i0 = bsel * kPPDistThreads;
            int64_t i1 = i0 + kPPDistThreads;
            if (i1 > n) i1 = n;
            int64_t c = i1 - 1;
            for (int64_t i = i0; i < i1; ++i) {
                run += d2[i];
                if (run > target) {
                    c = i;
                    break;
                }
            }
            pick = c;
        }
    }
    __syncthreads();
    const int64_t c = pick;
    double* mu = centers + (int64_t)k * p;
    for (int j = t; j < p; j += kPPSelThreads) mu[j] = 0.0;
    __syncthreads();
    for (int a = t; a < m; a += kPPSelThreads) {
        const int j = idx[c * m + a];
        if (j < p) mu[j] = (double)vals[c * m + a];
    }
    if (t == 0 && chosen) chosen[k] = c;
}

static int64_t pp_blocks(int64_t n) { return (n + kPPDistThreads - 1) / kPPDistThreads; }

size_t kmeanspp_workspace(int64_t n)
{
    const size_t a = ((size_t)n * sizeof(double) + 255) & ~(size_t)255;
    const size_t b = ((size_t)pp_blocks(n) * sizeof(double) + 255) & ~(size_t)255;
    return a + b;
}

template <typename T>
static hipError_t launch_pp_t(int p, int m, const T* vals, const uint16_t* idx, int64_t n, int K, uint64_t seed,
                              uint64_t rep, double* centers, int64_t* chosen, void* ws, hipStream_t s)
{
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    double* d2 = reinterpret_cast<double*>(w);
    double* bsum = reinterpret_cast<double*>(w + (((size_t)n * sizeof(double) + 255) & ~(size_t)255));
    const int64_t nb = pp_blocks(n);
    const size_t clds = (size_t)p * sizeof(double);
    const bool lds = clds <= (size_t)kPPCenterLds;
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pp_dist<T, true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(kPPCenterLds + PPChunk<T>::bytes));
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pp_dist<T, false>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)PPChunk<T>::bytes);
        attr = true;
    }
    for (int k = 0; k < K; ++k) {
        {
            ProfScope ps_("kmpp_select", s);
            hipLaunchKernelGGL((k_pp_select<T>), dim3(1), dim3(kPPSelThreads), 0, s, vals, idx, n, m, p, seed, rep, k,
                               d2, bsum, nb, centers, chosen);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (k + 1 == K) break;
        {
            ProfScope ps_("kmpp_dist", s);
            const double* c = centers + (int64_t)k * p;
            if (lds)
                hipLaunchKernelGGL((k_pp_dist<T, true>), dim3((unsigned)nb), dim3(kPPDistThreads),
                                   clds + PPChunk<T>::bytes, s, vals, idx, n, m, p, c, k == 0 ? 1 : 0, d2, bsum);
            else
                hipLaunchKernelGGL((k_pp_dist<T, false>), dim3((unsigned)nb), dim3(kPPDistThreads),
                                   PPChunk<T>::bytes, s, vals, idx, n, m, p, c, k == 0 ? 1 : 0, d2, bsum);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_kmeanspp(int prec, int p, int m, const void* vals, const uint16_t* idx, int64_t n, int K,
                           uint64_t seed, uint64_t rep, double* centers, int64_t* chosen, void* ws, hipStream_t s)
{
    if (prec == 0)
        return launch_pp_t(p, m, reinterpret_cast<const double*>(vals), idx, n, K, seed, rep, centers, chosen, ws, s);
    return launch_pp_t(p, m, reinterpret_cast<const float*>(vals), idx, n, K, seed, rep, centers, chosen, ws, s);
}

// Best of several starting points: after start r's last round, its centers and
// assignments replace the kept ones when its final objective is below every
// earlier start's (so ties keep the earliest).  Every thread takes the
// decision from the objectives alone, so no workgroup waits for another.
__global__ __launch_bounds__(256) void k_keep_best(int r, int T, const double* __restrict__ obj,
                                                   const double* __restrict__ centers, int64_t kp,
                                                   const int32_t* __restrict__ assign, int64_t n,
                                                   double* __restrict__ centers_best,
                                                   int32_t* __restrict__ assign_best, int32_t* __restrict__ best)
{
    const double mine = obj[(int64_t)r * T + T - 1];
    bool take = true;
    for (int q = 0; q < r; ++q)
        if (!(mine < obj[(int64_t)q * T + T - 1])) take = false;
    if (!take) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < kp + n; e += stride) {
        if (e < kp)
            centers_best[e] = centers[e];
        else
            assign_best[e - kp] = assign[e - kp];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *best = r;
}

hipError_t launch_keep_best(int r, int T, const double* obj, const double* centers, int64_t kp, const int32_t* assign,
                            int64_t n, double* centers_best, int32_t* assign_best, int32_t* best, const DeviceInfo& dev,
                            hipStream_t s)
{
    int64_t grid = (kp + n + 255) / 256;
    if (grid > (int64_t)dev.cus * 4) grid = (int64_t)dev.cus * 4;
    hipLaunchKernelGGL(k_keep_best, dim3((unsigned)grid), dim3(256), 0, s, r, T, obj, centers, kp, assign, n,
                       centers_best, assign_best, best);
    return hipGetLastError();
}

}  // namespace pds
