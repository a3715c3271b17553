// Sample-mean estimator on compressed data (Sec. IV, Thm. "sampleMean"): the
// p/m-rescaled mean of the zero-filled compressed samples, streamed into an FP64
// accumulator of per-coordinate sums.
//
// The kept entries (vals, idx) are read as one flat stream of n*m pairs: a sum
// per coordinate does not care which row an entry came from.  Two launches:
//   partial  workgroup = (range of the flat stream, block of up to 8192
//            coordinates): FP64 sums of the range's entries in LDS (LDS FP64
//            atomic adds; entries of other coordinate blocks are skipped), then
//            one row of per-range partial sums
//   reduce   per coordinate, the range partials in ascending range order
//            (sixteen fixed groups of ranges combined in group order), added to
//            the caller's accumulator; on finalize scaled by p/(m n_total)
// HBM-bound: 6 bytes per kept entry (FP32 value + 16-bit index; 10 for FP64
// plans) read once, plus the partial rows (8 p bytes per range, written and
// read once; the range count keeps them to a few percent of the stream).
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

constexpr int kMeanThreads = 512;
constexpr int kMeanBlockCols = 8192;  // coordinates per LDS block (64 KB of FP64 sums)
constexpr int kMeanReduceCols = 64;   // coordinates per reduce workgroup
constexpr int kMeanReduceGroups = 16; // fixed groups of ranges per reduce workgroup

template <typename T>
__device__ inline void mean_add(double* acc, T v, uint32_t c, uint32_t cbase, uint32_t cb)
{
    const uint32_t o = c - cbase;
    if (o < cb) atomicAdd(acc + o, (double)v);
}

template <typename T>
struct Quad;
template <>
struct Quad<float> {
    float v[4];
    __device__ inline void load(const float* p)
    {
        const float4 q = *reinterpret_cast<const float4*>(p);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    }
};
template <>
struct Quad<double> {
    double v[4];
    __device__ inline void load(const double* p)
    {
        const double2 a = *reinterpret_cast<const double2*>(p);
        const double2 b = *reinterpret_cast<const double2*>(p + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
};

// One workgroup per (flat range, coordinate block).  VEC: vals 16-byte and idx
// 8-byte aligned, so quads of entries load as one vector each; per_range is a
// multiple of 4, so every range starts on a quad.
template <typename T, bool VEC>
__global__ __launch_bounds__(kMeanThreads) void k_mean_partial(const T* __restrict__ vals,
                                                              const uint16_t* __restrict__ idx, int64_t total,
                                                              int64_t per_range, int cb, int p,
                                                              double* __restrict__ part)
{
    extern __shared__ double acc[];
    for (int c = threadIdx.x; c < cb; c += kMeanThreads) acc[c] = 0.0;
    __syncthreads();
    const int64_t e0 = (int64_t)blockIdx.x * per_range;
    int64_t e1 = e0 + per_range;
    if (e1 > total) e1 = total;
    const uint32_t cbase = blockIdx.y * (uint32_t)cb;
    int64_t tail = e0;
    if (VEC && e1 > e0) {
        const int64_t nq = (e1 - e0) >> 2;
        int64_t q = threadIdx.x;
        // two quads per thread in flight
        for (; q + kMeanThreads < nq; q += 2 * kMeanThreads) {
            const int64_t f0 = e0 + 4 * q, f1 = f0 + 4 * kMeanThreads;
            Quad<T> a, b;
            a.load(vals + f0);
            b.load(vals + f1);
            const uint2 ia = *reinterpret_cast<const uint2*>(idx + f0);
            const uint2 ib = *reinterpret_cast<const uint2*>(idx + f1);
            mean_add(acc, a.v[0], ia.x & 0xffffu, cbase, cb);
            mean_add(acc, a.v[1], ia.x >> 16, cbase, cb);
            mean_add(acc, a.v[2], ia.y & 0xffffu, cbase, cb);
            mean_add(acc, a.v[3], ia.y >> 16, cbase, cb);
            mean_add(acc, b.v[0], ib.x & 0xffffu, cbase, cb);
            mean_add(acc, b.v[1], ib.x >> 16, cbase, cb);
            mean_add(acc, b.v[2], ib.y & 0xffffu, cbase, cb);
            mean_add(acc, b.v[3], ib.y >> 16, cbase, cb);
        }
        if (q < nq) {
            const int64_t f0 = e0 + 4 * q;
            Quad<T> a;
            a.load(vals + f0);
            const uint2 ia = *reinterpret_cast<const uint2*>(idx + f0);
            mean_add(acc, a.v[0], ia.x & 0xffffu, cbase, cb);
            mean_add(acc, a.v[1], ia.x >> 16, cbase, cb);
            mean_add(acc, a.v[2], ia.y & 0xffffu, cbase, cb);
            mean_add(acc, a.v[3], ia.y >> 16, cbase, cb);
        }
        tail = e0 + 4 * nq;
    }
    for (int64_t f = tail + threadIdx.x; f < e1; f += kMeanThreads) mean_add(acc, vals[f], idx[f], cbase, cb);
    __syncthreads();
    double* out = part + (int64_t)blockIdx.x * p + cbase;
    for (int c = threadIdx.x; c < cb; c += kMeanThreads) out[c] = acc[c];
}

// Workgroup = kMeanReduceCols coordinates x kMeanReduceGroups groups of ranges.
// Group g sums ranges [g*per_g, (g+1)*per_g) in ascending order; the groups are
// then added in ascending order, then to acc.
__global__ __launch_bounds__(kMeanReduceCols* kMeanReduceGroups) void k_mean_reduce(const double* __restrict__ part,
                                                                                  int64_t nranges, int p,
                                                                                  double* __restrict__ acc,
                                                                                  int finalize, double scale,
                                                                                  double* __restrict__ mean_out)
{
    __shared__ double gsum[kMeanReduceGroups][kMeanReduceCols];
    const int cl = threadIdx.x % kMeanReduceCols, g = threadIdx.x / kMeanReduceCols;
    const int c = blockIdx.x * kMeanReduceCols + cl;
    const int64_t per_g = (nranges + kMeanReduceGroups - 1) / kMeanReduceGroups;
    int64_t r0 = g * per_g, r1 = r0 + per_g;
    if (r1 > nranges) r1 = nranges;
    double s = 0.0;
    if (c < p) {
        const double* pc = part + c;
#pragma unroll 8
        for (int64_t r = r0; r < r1; ++r) s += pc[r * p];
    }
    gsum[g][cl] = s;
    __syncthreads();
    if (g == 0 && c < p) {
        double t = 0.0;
        for (int k = 0; k < kMeanReduceGroups; ++k) t += gsum[k][cl];
        t = acc[c] + t;
        acc[c] = t;
        if (finalize) mean_out[c] = t * scale;
    }
}

struct MeanPlan {
    int cb, ncb;
    int64_t per_range, nranges;
};

static MeanPlan mean_plan(int p, int m, int64_t n, const DeviceInfo& dev)
{
    MeanPlan k;
    k.cb = p < kMeanBlockCols ? p : kMeanBlockCols;
    k.ncb = (p + k.cb - 1) / k.cb;
    const int64_t total = n * (int64_t)m;
    // about four workgroups per CU; each range at least 64 p entries so that
    // the partial rows stay a few percent of the stream
    int64_t nr = ((int64_t)dev.cus * 4 + k.ncb - 1) / k.ncb;
    const int64_t maxr = (total + 64 * (int64_t)p - 1) / (64 * (int64_t)p);
    if (nr > maxr) nr = maxr;
    if (nr < 1) nr = 1;
    int64_t per = (total + nr - 1) / nr;
    per = (per + 3) & ~(int64_t)3;
    if (per < 4) per = 4;
    k.per_range = per;
    k.nranges = total > 0 ? (total + per - 1) / per : 0;
    return k;
}

size_t mean_workspace(int p, int m, int64_t n, const DeviceInfo& dev)
{
    const MeanPlan k = mean_plan(p, m, n, dev);
    return (size_t)k.nranges * (size_t)p * sizeof(double);
}

hipError_t launch_mean(int prec, int p, int m, const void* vals, const uint16_t* idx, int64_t n, double* acc,
                       int finalize, int64_t n_total, double* mean_out, void* ws, const DeviceInfo& dev,
                       hipStream_t s)
{
    const MeanPlan k = mean_plan(p, m, n, dev);
    double* part = reinterpret_cast<double*>(ws);
    const int64_t total = n * (int64_t)m;
    if (total > 0) {
        ProfScope ps_("mean_partial", s);
        const dim3 grid((unsigned)k.nranges, (unsigned)k.ncb);
        const size_t lds = (size_t)k.cb * sizeof(double);
        const bool vec = ((uintptr_t)idx & 7) == 0 && ((uintptr_t)vals & 15) == 0;
        if (prec == 0) {
            const double* v = reinterpret_cast<const double*>(vals);
            if (vec)
                hipLaunchKernelGGL((k_mean_partial<double, true>), grid, dim3(kMeanThreads), lds, s, v, idx, total,
                                   k.per_range, k.cb, p, part);
            else
                hipLaunchKernelGGL((k_mean_partial<double, false>), grid, dim3(kMeanThreads), lds, s, v, idx, total,
                                   k.per_range, k.cb, p, part);
        } else {
            const float* v = reinterpret_cast<const float*>(vals);
            if (vec)
                hipLaunchKernelGGL((k_mean_partial<float, true>), grid, dim3(kMeanThreads), lds, s, v, idx, total,
                                   k.per_range, k.cb, p, part);
            else
                hipLaunchKernelGGL((k_mean_partial<float, false>), grid, dim3(kMeanThreads), lds, s, v, idx, total,
                                   k.per_range, k.cb, p, part);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        ProfScope ps_("mean_reduce", s);
        const double scale = finalize ? (double)p / ((double)m * (double)n_total) : 0.0;
        hipLaunchKernelGGL(k_mean_reduce, dim3((unsigned)((p + kMeanReduceCols - 1) / kMeanReduceCols)),
                           dim3(kMeanReduceCols * kMeanReduceGroups), 0, s, part, total > 0 ? k.nranges : 0, p, acc,
                           finalize, scale, mean_out);
    }
    return hipGetLastError();
}

}  // namespace pds
