// One-pass compression (Alg. 1, first loop): y_i = H D x_i (Sec. III, eq. ROS)
// with H the normalized Sylvester Walsh-Hadamard matrix, then the kept
// entries vals_i[t] = y_i[idx_i[t]] (w_i = R_i R_i^T y_i, Sec. I setup).
//
// Fast path (256 <= p <= 4096, 16-byte aligned rows): one wavefront per
// sample, E = p/64 elements per lane in registers.  The transform is the
// tensor product of 2x2 butterflies over the log2(p) bits of the element
// index, and those commute, so each lane first applies the butterflies of the
// bits it holds in registers; the remaining bits (spread across lanes) are
// brought into registers by transposes through LDS, R bits at a time.  The
// last layout is written to LDS once more and the kept entries are gathered
// from there.  X is read once, coalesced; latency is hidden by the many resident waves.  Persistent: each wave loops over
// samples with a grid-wide stride.
//
// Generic path (any p, any alignment): one workgroup per sample, all
// butterfly stages in a staging buffer (LDS, or a workspace slice for very
// large p) with barriers between stages.
#include "pds_device.hpp"
#include "pds_fast.hpp"
#include "pds_internal.hpp"

namespace pds {

template <typename T, int L>
__global__ __launch_bounds__(64) void k_compress_fast(uint64_t seed, int m, const T* __restrict__ X, int64_t n,
                                                      int64_t ldx, const uint16_t* __restrict__ idx,
                                                      T* __restrict__ vals)
{
    constexpr int P = 1 << L;
    constexpr int E = P / 64;
    constexpr int LV = FastLV<T, L>::value;
    using Lay = FastLayout<L, LV>;
    constexpr int NPH = Lay::kPhases;
    constexpr int PADDED = lds_pad<T>(P - 1) + 1;

    __shared__ T buf[PADDED];
    __shared__ uint32_t negbits[P / 32];

    const int lane = threadIdx.x;

    // signs of D for all p coordinates (bit set = -1), one Philox block per 256
    for (int b = lane; b < P / 256; b += 64) {
        u64x4 blk = sign_block(seed, (uint64_t)b);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            negbits[b * 8 + 2 * w] = (uint32_t)blk.w[w];
            negbits[b * 8 + 2 * w + 1] = (uint32_t)(blk.w[w] >> 32);
        }
    }
    __syncthreads();
    // this lane's signs in the load layout
    uint64_t negmask = 0;
    {
        const int lp = Lay::lane_part(0, lane);
#pragma unroll
        for (int ri = 0; ri < E; ++ri) {
            const int e = lp | Lay::reg_part(0, ri);
            negmask |= (uint64_t)((negbits[e >> 5] >> (e & 31)) & 1u) << ri;
        }
    }
    const T scale = (T)(1.0 / sqrt((double)P));

    int64_t i = blockIdx.x;
    const int64_t stride = gridDim.x;
    if (i >= n) return;
    T x[E];
    load_row<T, L>(x, X + i * ldx, lane);

    for (; i < n; i += stride) {

#pragma unroll
        for (int ri = 0; ri < E; ++ri) x[ri] = flip_sign<T>(x[ri], (uint32_t)((negmask >> ri) & 1u));

#pragma unroll
        for (int ph = 0; ph < NPH; ++ph) {
            if (ph > 0) {
                // transpose: current layout out, next layout in
                // lane and register parts of an element index have disjoint
                // bits, so pad(lane | reg) = pad(lane) + pad(reg): one base
                // register per phase plus compile-time offsets
                __syncthreads();
                T* base_old = buf + lds_pad<T>(Lay::lane_part(ph - 1, lane));
#pragma unroll
                for (int ri = 0; ri < E; ++ri) base_old[lds_pad<T>(Lay::reg_part(ph - 1, ri))] = x[ri];
                __syncthreads();
                const T* base_new = buf + lds_pad<T>(Lay::lane_part(ph, lane));
#pragma unroll
                for (int ri = 0; ri < E; ++ri) x[ri] = base_new[lds_pad<T>(Lay::reg_part(ph, ri))];
            }
            butterflies<E, T>(x, Lay::group_size(ph));
        }

        __syncthreads();
        {
            T* base = buf + lds_pad<T>(Lay::lane_part(NPH - 1, lane));
#pragma unroll
            for (int ri = 0; ri < E; ++ri) base[lds_pad<T>(Lay::reg_part(NPH - 1, ri))] = x[ri] * scale;
        }
        // the registers are free again: start loading the next row under the gather
        if (i + stride < n) load_row<T, L>(x, X + (i + stride) * ldx, lane);
        __syncthreads();
        const uint16_t* ix = idx + i * (int64_t)m;
        T* out = vals + i * (int64_t)m;
        for (int t = lane; t < m; t += 64) out[t] = buf[lds_pad<T>((int)ix[t])];
    }
}

// ---------------------------------------------------------------------------
// Generic path
// ---------------------------------------------------------------------------
constexpr int kGenericThreads = 256;
constexpr size_t kGenericLdsLimit = 65536;

template <typename T>
__global__ __launch_bounds__(kGenericThreads) void k_compress_generic(uint64_t seed, int p, int m,
                                                                      const T* __restrict__ X, int64_t n,
                                                                      int64_t ldx, const uint16_t* __restrict__ idx,
                                                                      T* __restrict__ vals, T* gscratch,
                                                                      int use_lds)
{
    extern __shared__ unsigned char smem[];
    uint32_t* negbits = reinterpret_cast<uint32_t*>(smem);
    const int nwords = (p + 31) / 32;
    const size_t sign_bytes = ((size_t)nwords * 4 + 15) & ~(size_t)15;
    T* buf = use_lds ? reinterpret_cast<T*>(smem + sign_bytes) : gscratch + (size_t)blockIdx.x * p;
    const int tid = threadIdx.x;

    const int nblocks = (p + 255) / 256;
    for (int b = tid; b < nblocks; b += kGenericThreads) {
        u64x4 blk = sign_block(seed, (uint64_t)b);
        for (int w = 0; w < 8; ++w) {
            int word = b * 8 + w;
            if (word < nwords) negbits[word] = (w & 1) ? (uint32_t)(blk.w[w >> 1] >> 32) : (uint32_t)blk.w[w >> 1];
        }
    }
    __syncthreads();
    const T scale = (T)(1.0 / sqrt((double)p));

    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const T* row = X + i * ldx;
        for (int j = tid; j < p; j += kGenericThreads)
            buf[j] = flip_sign<T>(row[j], (negbits[j >> 5] >> (j & 31)) & 1u);
        for (int h = 1; h < p; h <<= 1) {
            if (!use_lds) __threadfence();
            __syncthreads();
            if (!use_lds) __threadfence();
            for (int q = tid; q < p / 2; q += kGenericThreads) {
                int a = (q / h) * 2 * h + (q % h);
                T u = buf[a], v = buf[a + h];
                buf[a] = u + v;
                buf[a + h] = u - v;
            }
        }
        if (!use_lds) __threadfence();
        __syncthreads();
        if (!use_lds) __threadfence();
        const uint16_t* ix = idx + i * (int64_t)m;
        T* out = vals + i * (int64_t)m;
        for (int t = tid; t < m; t += kGenericThreads) out[t] = buf[ix[t]] * scale;
        if (!use_lds) __threadfence();
        __syncthreads();
        if (!use_lds) __threadfence();
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static int64_t generic_grid(int64_t n, const DeviceInfo& dev) { return n < (int64_t)dev.cus * 4 ? n : (int64_t)dev.cus * 4; }

static size_t generic_lds_bytes(int p, size_t elem)
{
    const int nwords = (p + 31) / 32;
    const size_t sign_bytes = ((size_t)nwords * 4 + 15) & ~(size_t)15;
    const size_t buf = (size_t)p * elem;
    return (sign_bytes + buf <= kGenericLdsLimit) ? sign_bytes + buf : sign_bytes;
}

static bool fast_path_ok(int p, const void* X, int64_t ldx, size_t elem)
{
    if (p < 256 || p > 4096) return false;
    if (((uintptr_t)X) % 16 != 0) return false;
    if ((ldx * (int64_t)elem) % 16 != 0) return false;
    return true;
}

size_t compress_workspace(int prec, int p, int64_t n, const DeviceInfo& dev)
{
    const size_t elem = (prec == 0) ? sizeof(double) : sizeof(float);
    const int nwords = (p + 31) / 32;
    const size_t sign_bytes = ((size_t)nwords * 4 + 15) & ~(size_t)15;
    if (sign_bytes + (size_t)p * elem <= kGenericLdsLimit) return 0;
    return (size_t)generic_grid(n, dev) * (size_t)p * elem;
}

template <typename T>
static hipError_t launch_fast(int L, uint64_t seed, int m, const T* X, int64_t n, int64_t ldx, const uint16_t* idx,
                              T* vals, const DeviceInfo& dev, hipStream_t s)
{
    // one resident wave per slot the chip can hold; the stride loop covers the rest
    switch (L) {
#define PDS_FAST_CASE(LL)                                                                                 \
    case LL: {                                                                                            \
        static int per_cu = 0;                                                                            \
        if (per_cu == 0) {                                                                                \
            int b = 0;                                                                                    \
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_compress_fast<T, LL>, 64, 0) !=       \
                    hipSuccess ||                                                                         \
                b < 1)                                                                                    \
                b = 4;                                                                                    \
            per_cu = b;                                                                                   \
        }                                                                                                 \
        int64_t grid = (int64_t)dev.cus * per_cu;                                                         \
        if (grid > n) grid = n;                                                                           \
        { ProfScope ps_("compress", s); hipLaunchKernelGGL((k_compress_fast<T, LL>), dim3((unsigned)grid), dim3(64), 0, s, seed, m, X, n, \
                           ldx, idx, vals); }                                                               \
        break;                                                                                            \
    }
        PDS_FAST_CASE(8)
        PDS_FAST_CASE(9)
        PDS_FAST_CASE(10)
        PDS_FAST_CASE(11)
        PDS_FAST_CASE(12)
#undef PDS_FAST_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_generic(uint64_t seed, int p, int m, const T* X, int64_t n, int64_t ldx,
                                 const uint16_t* idx, T* vals, void* ws, const DeviceInfo& dev, hipStream_t s)
{
    const int64_t grid = generic_grid(n, dev);
    const int nwords = (p + 31) / 32;
    const size_t sign_bytes = ((size_t)nwords * 4 + 15) & ~(size_t)15;
    const bool use_lds = sign_bytes + (size_t)p * sizeof(T) <= kGenericLdsLimit;
    const size_t lds = generic_lds_bytes(p, sizeof(T));
    {
        ProfScope ps_("compress", s);
        hipLaunchKernelGGL((k_compress_generic<T>), dim3((unsigned)grid), dim3(kGenericThreads), lds, s, seed, p, m, X,
                       n, ldx, idx, vals, reinterpret_cast<T*>(ws), use_lds ? 1 : 0);
    }
    return hipGetLastError();
}

hipError_t launch_compress(int prec, uint64_t seed, int p, int m, const void* X, int64_t n, int64_t ldx,
                           const uint16_t* idx, void* vals, void* ws, size_t ws_bytes, const DeviceInfo& dev,
                           hipStream_t s)
{
    (void)ws_bytes;
    if (n <= 0) return hipSuccess;
    int L = 0;
    while ((1 << L) < p) ++L;
    if (prec == 0) {
        const double* Xd = reinterpret_cast<const double*>(X);
        double* vd = reinterpret_cast<double*>(vals);
        if (fast_path_ok(p, X, ldx, sizeof(double)) && p <= 2048)
            return launch_fast<double>(L, seed, m, Xd, n, ldx, idx, vd, dev, s);
        return launch_generic<double>(seed, p, m, Xd, n, ldx, idx, vd, ws, dev, s);
    }
    const float* Xf = reinterpret_cast<const float*>(X);
    float* vf = reinterpret_cast<float*>(vals);
    if (prec == 2 && kron_transform_ok(p, X, ldx)) return launch_compress_kron(seed, m, Xf, n, ldx, idx, vf, dev, s);
    if (fast_path_ok(p, X, ldx, sizeof(float))) return launch_fast<float>(L, seed, m, Xf, n, ldx, idx, vf, dev, s);
    return launch_generic<float>(seed, p, m, Xf, n, ldx, idx, vf, ws, dev, s);
}

}  // namespace pds
