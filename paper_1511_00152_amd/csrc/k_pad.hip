// Zero-padding of rows whose dimension is not a power of two (the Hadamard
// transform of Sec. III needs one; the paper used a DCT for p = 784).
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

// Rows of width p_data copied into rows of the plan's width p_pad (a power of
// two) with zeros after column p_data: the transform of Sec. III then acts on
// [x; 0], whose norm and sample mean and covariance (up to zero rows and
// columns) are those of x.
template <typename T>
__global__ __launch_bounds__(256) void k_pad_rows(const T* __restrict__ X, int64_t n, int64_t p_data, int64_t ldx,
                                                  T* __restrict__ Xp, int64_t p_pad)
{
    const int64_t total = n * p_pad;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t r = e / p_pad, j = e - r * p_pad;
        Xp[e] = j < p_data ? X[r * ldx + j] : (T)0;
    }
}

hipError_t launch_pad_rows(int x_f64, const void* X, int64_t n, int64_t p_data, int64_t ldx, void* Xp, int64_t p_pad,
                           const DeviceInfo& dev, hipStream_t s)
{
    int64_t grid = (n * p_pad + 255) / 256;
    if (grid > (int64_t)dev.cus * 16) grid = (int64_t)dev.cus * 16;
    if (grid < 1) return hipSuccess;
    if (x_f64)
        hipLaunchKernelGGL(k_pad_rows<double>, dim3((unsigned)grid), dim3(256), 0, s,
                           reinterpret_cast<const double*>(X), n, p_data, ldx, reinterpret_cast<double*>(Xp), p_pad);
    else
        hipLaunchKernelGGL(k_pad_rows<float>, dim3((unsigned)grid), dim3(256), 0, s, reinterpret_cast<const float*>(X),
                           n, p_data, ldx, reinterpret_cast<float*>(Xp), p_pad);
    return hipGetLastError();
}

}  // namespace pds
