// DCT preconditioner (Sec. III; Sec. VII uses it at p = 784): any fast
// orthonormal transform whose entries are all O(1/sqrt(p)) may stand in for
// the normalized Hadamard matrix, and Thm. 1 holds for the orthonormal DCT-II
// with eta = 1/2.  Here y = C D x with the plan's signs D and
//     C[j][k] = s_j cos(pi (2k + 1) j / (2p)),  s_0 = sqrt(1/p), s_j = sqrt(2/p),
// for any p (no power-of-two restriction), followed by the same exact-m
// sampling as the Hadamard plans.
//
// The transform is a dense product Y = (X D) T with the table
// T[k][j] = C[j][k] (p x p, FP64, built on the device from cospi of the exact
// reduced angle), computed in FP64 on the matrix cores: FP64 keeps the result
// within a few units of FP64 rounding of the definition, so the one rounding
// of an FP32 plan is the final store.  Work per sample is p^2
// multiply-adds, against p log p for the Hadamard transform; at the sizes the
// paper uses the DCT for (p = 784, tens of thousands of samples) that is a
// few milliseconds.
//
// Tiling: a workgroup owns 64 samples x 64 outputs; 16 input coordinates at a
// time are staged in LDS as FP64 (the sign applied on the way in; the next
// step's loads in flight meanwhile), each wave multiplying a 32 x 32 quarter
// as 2 x 2 products of 16 x 16 x 4.  The finished 64 x 64 block goes to LDS
// (over the staging buffers) and each sample's kept coordinates inside its 64
// columns (a contiguous run of the ascending index row, found by binary
// search) are written out, so Y never reaches memory.
#include "pds_device.hpp"
#include "pds_internal.hpp"

namespace pds {

constexpr int kDctTile = 64;  // samples and outputs per workgroup
constexpr int kDctK = 16;     // input coordinates staged per step (32: 2.56 against 2.20 ms, lower occupancy)
constexpr int kDctMaxP = 8192;

// angle index r = (2k + 1) j reduced mod 4p: cos(pi r / (2p)) has period 4p in r
__device__ inline double dct_coef(int p, int j, int k)
{
    const int64_t r = ((int64_t)(2 * k + 1) * j) % (4 * (int64_t)p);
    const double s = (j == 0) ? sqrt(1.0 / p) : sqrt(2.0 / p);
    return s * cospi((double)r / (2.0 * p));
}

__global__ __launch_bounds__(256) void k_dct_table(int p, double* __restrict__ T)
{
    const int64_t tot = (int64_t)p * p;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int k = (int)(e / p), j = (int)(e - (int64_t)k * p);
        T[e] = dct_coef(p, j, k);
    }
}

// first t in [0, m) with row[t] >= key (m if none)
__device__ inline int lower_bound_u16(const uint16_t* __restrict__ row, int m, int key)
{
    int lo = 0, hi = m;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int)row[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

typedef double dct_d4 __attribute__((ext_vector_type(4)));

// LDS of one workgroup: the staged operands during the product, then the
// finished 64 x 64 block for the gather (the two never live together)
struct DctStage {
    double a[kDctTile][kDctK + 1];  // [sample][coordinate], signed x
    double b[kDctK][kDctTile + 1];  // [coordinate][output]
};
union DctLds {
    DctStage st;
    double y[kDctTile][kDctTile + 1];
};

template <class TX, class TV>
__global__ __launch_bounds__(256) void k_dct_compress(uint64_t seed, int p, int m, const TX* __restrict__ X,
                                                      int64_t n, int64_t ldx, const double* __restrict__ T,
                                                      const uint16_t* __restrict__ idx, TV* __restrict__ vals)
{
    __shared__ DctLds L;
    __shared__ uint32_t neg[kDctMaxP / 32];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * kDctTile;
    const int j0 = blockIdx.y * kDctTile;

    // sign bits of all p coordinates (one Philox block per 256)
    for (int b = tid; b < (p + 255) / 256; b += 256) {
        const u64x4 blk = sign_block(seed, (uint64_t)b);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            neg[b * 8 + 2 * w] = (uint32_t)blk.w[w];
            neg[b * 8 + 2 * w + 1] = (uint32_t)(blk.w[w] >> 32);
        }
    }

    // staging assignment: x of sample as, coordinates ak .. ak + 3; table
    // row bk, outputs bj .. bj + 3.  The next step's operands are loaded into
    // registers while the matrix cores work on the current one.
    constexpr int PER = kDctK / 4;        // staged values of each kind per thread
    constexpr int TPR = kDctTile / PER;   // threads per staged table row
    const int as = tid >> 2, ak = (tid & 3) * PER;
    const int bk = tid / TPR, bj = (tid % TPR) * PER;
    const int64_t xi = i0 + as;
    const TX* xrow = X + (xi < n ? xi : 0) * ldx;
    TX xv[PER];
    double tv[PER];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int k = k0 + ak + q;
            xv[q] = (xi < n && k < p) ? xrow[k] : (TX)0;
            const int kb = k0 + bk, j = j0 + bj + q;
            tv[q] = (kb < p && j < p) ? T[(int64_t)kb * p + j] : 0.0;
        }
    };
    load(0);

    // wave (wr, wc) owns rows 32 wr .. +32 and outputs 32 wc .. +32 of the
    // block: 2 x 2 products of 16 x 16 on v_mfma_f64_16x16x4f64 (operand lane
    // l: row / column l mod 16, k = l div 16; result register r of lane l:
    // row l div 16 + 4 r, column l mod 16)
    const int wr = wave >> 1, wc = wave & 1;
    const int li = lane & 15, lk = lane >> 4;
    dct_d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (dct_d4){0.0, 0.0, 0.0, 0.0};

    for (int k0 = 0; k0 < p; k0 += kDctK) {
        __syncthreads();  // the previous step's operand reads are done (and neg is written)
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int k = k0 + ak + q;
            double v = (double)xv[q];
            if (k < p && ((neg[k >> 5] >> (k & 31)) & 1u)) v = -v;
            L.st.a[as][ak + q] = v;
            L.st.b[bk][bj + q] = tv[q];
        }
        __syncthreads();
        if (k0 + kDctK < p) load(k0 + kDctK);
#pragma unroll
        for (int kk = 0; kk < kDctK; kk += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) av[r] = L.st.a[32 * wr + 16 * r + li][kk + lk];
#pragma unroll
            for (int c = 0; c < 2; ++c) bv[c] = L.st.b[kk + lk][32 * wc + 16 * c + li];
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[r], bv[c], acc[r][c], 0, 0, 0);
        }
    }
    __syncthreads();  // every wave is done with the staged operands
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) L.y[32 * wr + 16 * r + lk + 4 * q][32 * wc + 16 * c + li] = acc[r][c][q];
    __syncthreads();

    // kept coordinates of each sample inside [j0, j0 + 64): four threads per sample
    const int s = tid >> 2, sub = tid & 3;
    const int64_t i = i0 + s;
    if (i < n) {
        const uint16_t* row = idx + i * (int64_t)m;
        const int t0 = lower_bound_u16(row, m, j0);
        const int t1 = lower_bound_u16(row, m, j0 + kDctTile);
        TV* out = vals + i * (int64_t)m;
        for (int t = t0 + sub; t < t1; t += 4) out[t] = (TV)L.y[s][(int)row[t] - j0];
    }
}

size_t dct_compress_workspace(int p)
{
    return (size_t)p * (size_t)p * sizeof(double);
}

hipError_t launch_dct_compress(int prec, uint64_t seed, int p, int m, const void* X, int64_t n, int64_t ldx,
                               const uint16_t* idx, void* vals, void* ws, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (p > kDctMaxP) return hipErrorInvalidValue;
    double* T = reinterpret_cast<double*>(ws);
    {
        const int64_t tot = (int64_t)p * p;
        int64_t blocks = (tot + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        ProfScope ps_("dct_table", s);
        hipLaunchKernelGGL(k_dct_table, dim3((unsigned)blocks), dim3(256), 0, s, p, T);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)((n + kDctTile - 1) / kDctTile), (unsigned)((p + kDctTile - 1) / kDctTile));
    ProfScope ps_("compress", s);
    if (prec == 0) {  // FP64 plans take FP64 rows and keep FP64 values
        hipLaunchKernelGGL((k_dct_compress<double, double>), grid, dim3(256), 0, s, seed, p, m,
                           reinterpret_cast<const double*>(X), n, ldx, T, idx, reinterpret_cast<double*>(vals));
    } else {
        hipLaunchKernelGGL((k_dct_compress<float, float>), grid, dim3(256), 0, s, seed, p, m,
                           reinterpret_cast<const float*>(X), n, ldx, T, idx, reinterpret_cast<float*>(vals));
    }
    return hipGetLastError();
}

// mu = (C D)^T mu' = D C^T mu': out[k][j] = D_j sum_i C[i][j] mu'[k][i], FP64,
// one thread per (center, coordinate).  C[i][j] = s_i cos(i t), t = pi (2j + 1)
// / (2p): the cosines advance by a rotation through t (two FMAs per term),
// restarted from cospi / sinpi of the exactly reduced angle every 32 terms, so
// no coefficient carries more than a few dozen roundings.
__global__ __launch_bounds__(256) void k_dct_unmix(uint64_t seed, int p, const double* __restrict__ cpre,
                                                   double* __restrict__ cout)
{
    extern __shared__ double mu[];  // the center's p pre-image coordinates
    const int k = blockIdx.y;
    const int j = blockIdx.x * 256 + threadIdx.x;
    for (int i = threadIdx.x; i < p; i += 256) mu[i] = cpre[(int64_t)k * p + i];
    __syncthreads();
    if (j >= p) return;
    const int64_t a = 2 * (int64_t)j + 1;
    const double ct = cospi((double)a / (2.0 * p)), st = sinpi((double)a / (2.0 * p));
    double sum = 0.0;  // sum over i >= 1 of cos(i t) mu_i
    for (int b = 1; b < p; b += 32) {
        const double arg = (double)((a * b) % (4 * (int64_t)p)) / (2.0 * p);
        double c = cospi(arg), s = sinpi(arg);
        const int e = (b + 32 < p) ? b + 32 : p;
        for (int i = b; i < e; ++i) {
            sum = fma(c, mu[i], sum);
            const double cn = c * ct - s * st;
            s = fma(s, ct, c * st);
            c = cn;
        }
    }
    const double v = sqrt(2.0 / p) * sum + sqrt(1.0 / p) * mu[0];
    const u64x4 blk = sign_block(seed, (uint64_t)(j >> 8));
    const uint64_t w = blk.w[(j >> 6) & 3];
    cout[(int64_t)k * p + j] = ((w >> (j & 63)) & 1ull) ? -v : v;
}

hipError_t launch_dct_unmix(uint64_t seed, int p, const double* cpre, int K, double* cout, hipStream_t s)
{
    if (K <= 0) return hipSuccess;
    if (p > kDctMaxP) return hipErrorInvalidValue;
    ProfScope ps_("unmix", s);
    hipLaunchKernelGGL(k_dct_unmix, dim3((unsigned)((p + 255) / 256), (unsigned)K), dim3(256),
                       (size_t)p * sizeof(double), s, seed, p, cpre, cout);
    return hipGetLastError();
}

}  // namespace pds
