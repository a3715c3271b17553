// Quality of principal components estimated from the covariance estimate:
// the fraction of explained variance of the column-sampling comparison
// (Sec. II), ||X U^T||_F^2 / ||X||_F^2 for k orthonormal components (the rows
// of U) and data rows X.
//
// One pass over X, the dots on the FP64 matrix cores (below).  The squared
// dots and the squares of X are summed per thread, then per workgroup and
// over workgroups in a fixed order.
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

constexpr int kEvThreads = 256;
constexpr int kEvMaxK = 32;
constexpr int kEvGrid = 1024;  // workgroups; two FP64 partials each

typedef double ev_d4 __attribute__((ext_vector_type(4)));

constexpr int kEvRB = 1;   // 16-row blocks per wave: a tile of 64 kEvRB rows (2 or 4: 12.7 and 14.6 ms)
constexpr int kEvKS = 16;  // coordinates per step (32: 10.95 ms, 64: 12.9 ms, against 10.87)

// The dots on the FP64 matrix cores: a workgroup takes tiles of 64 kEvRB rows
// (grid-stride, fixed assignment) and walks the coordinates kEvKS at a time,
// the X chunk (as FP64) and the matching coordinates of the components staged
// in LDS with the next chunk's loads in flight; wave w multiplies its kEvRB
// blocks of 16 rows with NB blocks of 16 components on v_mfma_f64_16x16x4f64
// (operand lane l: row / component l mod 16, coordinate l div 16; result
// register r of lane l: row l div 16 + 4 r, component l mod 16).  Components
// past k are zero rows, so their dots are zero.
template <typename T, int NB>
__global__ __launch_bounds__(kEvThreads) void k_explained(const double* __restrict__ U, int k,
                                                          const T* __restrict__ X, int64_t n, int p, int64_t ldx,
                                                          double* __restrict__ part)
{
    constexpr int KS = kEvKS, RB = kEvRB, TR = 64 * RB;  // tile rows
    constexpr int XPER = TR * KS / kEvThreads;          // staged x per thread
    constexpr int XTR = KS / XPER;                       // threads per row
    constexpr int UPER = (KS * 16 * NB) / kEvThreads;   // staged component entries per thread
    constexpr int UTR = KS / UPER;                       // threads per component
    __shared__ double xs[TR][KS + 1];
    __shared__ double us[KS][16 * NB + 1];
    __shared__ double red[2][kEvThreads];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int xr = t / XTR, xc = (t % XTR) * XPER;
    const int ur = t / UTR, uc = (t % UTR) * UPER;
    double num = 0.0, den = 0.0;
    const int64_t ntiles = (n + TR - 1) / TR;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * TR;
        const int64_t row = r0 + xr;
        const T* xrow = X + (row < n ? row : 0) * ldx;
        double xv[XPER], uv[UPER];
        auto load = [&](int c0) {
#pragma unroll
            for (int q = 0; q < XPER; ++q) {
                const int c = c0 + xc + q;
                xv[q] = (row < n && c < p) ? (double)xrow[c] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < UPER; ++q) {
                const int c = c0 + uc + q;
                uv[q] = (ur < k && c < p) ? U[(int64_t)ur * p + c] : 0.0;
            }
        };
        ev_d4 acc[RB][NB];
#pragma unroll
        for (int a = 0; a < RB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[a][b] = (ev_d4){0.0, 0.0, 0.0, 0.0};
        load(0);
        for (int c0 = 0; c0 < p; c0 += KS) {
            __syncthreads();  // the previous step's operand reads are done
#pragma unroll
            for (int q = 0; q < XPER; ++q) {
                xs[xr][xc + q] = xv[q];
                den = fma(xv[q], xv[q], den);
            }
#pragma unroll
            for (int q = 0; q < UPER; ++q) us[uc + q][ur] = uv[q];
            __syncthreads();
            if (c0 + KS < p) load(c0 + KS);
#pragma unroll
            for (int kk = 0; kk < KS; kk += 4) {
                double bv[NB];
#pragma unroll
                for (int b = 0; b < NB; ++b) bv[b] = us[kk + lk][16 * b + li];
#pragma unroll
                for (int a = 0; a < RB; ++a) {
                    const double av = xs[16 * (RB * wave + a) + li][kk + lk];
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[b], acc[a][b], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int a = 0; a < RB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) num = fma(acc[a][b][r], acc[a][b][r], num);
    }
    red[0][t] = num;
    red[1][t] = den;
    __syncthreads();
    for (int s = kEvThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
            red[0][t] += red[0][t + s];
            red[1][t] += red[1][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        part[2 * blockIdx.x] = red[0][0];
        part[2 * blockIdx.x + 1] = red[1][0];
    }
}

__global__ __launch_bounds__(kEvThreads) void k_explained_reduce(const double* __restrict__ part, int nwg,
                                                                 double* __restrict__ out2)
{
    __shared__ double red[2][kEvThreads];
    const int t = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int w = t; w < nwg; w += kEvThreads) {
        a += part[2 * w];
        b += part[2 * w + 1];
    }
    red[0][t] = a;
    red[1][t] = b;
    __syncthreads();
    for (int s = kEvThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
            red[0][t] += red[0][t + s];
            red[1][t] += red[1][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        out2[0] = red[0][0];
        out2[1] = red[1][0];
    }
}

size_t explained_workspace() { return (size_t)kEvGrid * 2 * sizeof(double); }

int explained_max_k() { return kEvMaxK; }

template <typename T>
static void launch_explained_t(const double* U, int k, const T* X, int64_t n, int p, int64_t ldx, double* part,
                               int grid, hipStream_t s)
{
    if (k <= 16)
        hipLaunchKernelGGL((k_explained<T, 1>), dim3(grid), dim3(kEvThreads), 0, s, U, k, X, n, p, ldx, part);
    else
        hipLaunchKernelGGL((k_explained<T, 2>), dim3(grid), dim3(kEvThreads), 0, s, U, k, X, n, p, ldx, part);
}

hipError_t launch_explained(const double* U, int k, const void* X, int x_f64, int64_t n, int p, int64_t ldx,
                            double* out2, void* ws, hipStream_t s)
{
    double* part = reinterpret_cast<double*>(ws);
    const int64_t ntiles = (n + 64 * kEvRB - 1) / (64 * kEvRB);
    const int grid = ntiles < kEvGrid ? (int)ntiles : kEvGrid;
    {
        ProfScope ps_("explained", s);
        if (x_f64)
            launch_explained_t(U, k, reinterpret_cast<const double*>(X), n, p, ldx, part, grid, s);
        else
            launch_explained_t(U, k, reinterpret_cast<const float*>(X), n, p, ldx, part, grid, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_explained_reduce, dim3(1), dim3(kEvThreads), 0, s, part, grid, out2);
    return hipGetLastError();
}

}  // namespace pds
