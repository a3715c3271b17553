// Quality of principal components estimated from the covariance estimate:
// the fraction of explained variance of the column-sampling comparison
// (Sec. II), ||X U^T||_F^2 / ||X||_F^2 for k orthonormal components (the rows
// of U) and data rows X.
//
// One pass over X.  A workgroup takes 64-row tiles (grid-stride, fixed
// assignment) and walks the coordinates in chunks of 32: the X chunk (as FP64)
// and the matching 32 coordinates of every component are staged in LDS, and
// each thread accumulates the dot products of 4 rows with 1 or 2 components in
// FP64.  The squared dots and the squares of X are summed per thread, then per
// workgroup and over workgroups in a fixed order.
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

constexpr int kEvRows = 64;
constexpr int kEvChunk = 32;
constexpr int kEvThreads = 256;
constexpr int kEvMaxK = 32;
constexpr int kEvGrid = 1024;  // workgroups; two FP64 partials each

template <typename T, int NV>
__global__ __launch_bounds__(kEvThreads) void k_explained(const double* __restrict__ U, int k,
                                                          const T* __restrict__ X, int64_t n, int p, int64_t ldx,
                                                          double* __restrict__ part)
{
    __shared__ double xs[kEvRows][kEvChunk + 1];
    __shared__ double us[kEvMaxK][kEvChunk + 1];
    __shared__ double red[2][kEvThreads];
    const int t = threadIdx.x, rg = t >> 4, vg = t & 15;
    double num = 0.0, den = 0.0;
    const int64_t ntiles = (n + kEvRows - 1) / kEvRows;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * kEvRows;
        double acc[4][NV];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[i][v] = 0.0;
        for (int c0 = 0; c0 < p; c0 += kEvChunk) {
            // X chunk: 8 passes of 8 rows, 32 consecutive coordinates per row
            const int lc = t & 31, c = c0 + lc;
#pragma unroll
            for (int pass = 0; pass < 8; ++pass) {
                const int lr = pass * 8 + (t >> 5);
                const int64_t r = r0 + lr;
                const double x = (r < n && c < p) ? (double)X[r * ldx + c] : 0.0;
                xs[lr][lc] = x;
                den += x * x;
            }
            for (int e = t; e < kEvMaxK * kEvChunk; e += kEvThreads) {
                const int j = e / kEvChunk, cc = e % kEvChunk;
                us[j][cc] = (j < k && c0 + cc < p) ? U[(int64_t)j * p + c0 + cc] : 0.0;
            }
            __syncthreads();
#pragma unroll 8
            for (int cc = 0; cc < kEvChunk; ++cc) {
                double u[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) u[v] = us[vg + 16 * v][cc];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const double x = xs[4 * rg + i][cc];
#pragma unroll
                    for (int v = 0; v < NV; ++v) acc[i][v] = fma(x, u[v], acc[i][v]);
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int v = 0; v < NV; ++v) num += acc[i][v] * acc[i][v];
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
    const int64_t ntiles = (n + kEvRows - 1) / kEvRows;
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
