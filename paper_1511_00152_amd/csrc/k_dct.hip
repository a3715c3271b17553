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

// ---------------------------------------------------------------------------
// Fast form (p = 2^a 3^b 5^c 7^d, p <= 2048): O(p log p) per sample.
// Makhoul's reordering turns the DCT-II into one complex DFT of the same
// length: with v_n = x_{2n} (n < ceil(p/2)) and v_{p-1-n} = x_{2n+1},
//     sum_n x_n cos(pi k (2n + 1) / (2p)) = Re(e^{-i pi k / (2p)} V_k),
// V = DFT(v).  Two samples share one complex transform (z = v1 + i 2^e v2,
// 2^e bringing the two norms within a factor of two, so that the rounding of
// the one transform stays relative to each sample's own norm; V1_k =
// (Z_k + conj Z_{-k}) / 2, V2_k = 2^-e (Z_k - conj Z_{-k}) / (2i)).  The FFT
// is a mixed-radix decimation in frequency done in place in one LDS buffer
// (radix 4, 2, 3, 5 or 7 per stage; each butterfly reads and rewrites its own
// R positions, so a stage needs no second buffer), every twiddle read from a
// table of e^{-2 pi i k / p} built from cospi / sinpi of the exact angles, all
// in FP64.  Its output is in digit-reversed order, so Z_k is read at
// rev(k); only the kept coordinates are separated and rotated, straight into
// vals.  One wave per pair of samples.
// ---------------------------------------------------------------------------
constexpr int kFftMaxP = 2048;
constexpr int kFftMaxStages = 12;

struct FftPlan {
    int nf;
    int r[kFftMaxStages];
};

// radices of p, in the order the stages run: fours, then a two, then threes,
// fives and sevens; nf = 0 when p has another prime factor
static FftPlan fft_plan(int p)
{
    FftPlan f{};
    int n = p;
    const int rs[5] = {4, 2, 3, 5, 7};
    for (int ri = 0; ri < 5; ++ri)
        while (n % rs[ri] == 0 && f.nf < kFftMaxStages) {
            f.r[f.nf++] = rs[ri];
            n /= rs[ri];
        }
    if (n != 1) f.nf = 0;
    return f;
}

bool dct_fast_ok(int p)
{
    return p >= 2 && p <= kFftMaxP && fft_plan(p).nf > 0;
}

// W[k] = e^{-2 pi i k / p}; Q[k] = s_k (cos(pi k / (2p)), sin(pi k / (2p)))
__global__ __launch_bounds__(256) void k_dct_fft_tables(int p, double2* __restrict__ W, double2* __restrict__ Q)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= p) return;
    const double a = 2.0 * (double)k / (double)p;  // exact for the power-of-two part; one rounding otherwise
    W[k] = make_double2(cospi(a), -sinpi(a));
    const double b = (double)k / (2.0 * (double)p);
    const double sk = (k == 0) ? sqrt(1.0 / p) : sqrt(2.0 / p);
    Q[k] = make_double2(sk * cospi(b), sk * sinpi(b));
}

__device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// quotient of k by a radix of the plan (compile-time divisors)
__device__ inline int div_radix(int k, int R)
{
    switch (R) {
        case 2: return k >> 1;
        case 3: return k / 3;
        case 4: return k >> 2;
        case 5: return k / 5;
        default: return k / 7;
    }
}

// position of frequency k in the in-place transform's output: with k =
// u_1 + R_1 (u_2 + R_2 (u_3 + ...)), at sum_i u_i p / (R_1 ... R_i)
__device__ inline int digit_rev(int k, const FftPlan& fp, int p)
{
    int pos = 0, len = p;
    for (int f = 0; f < fp.nf; ++f) {
        const int R = fp.r[f];
        const int q = div_radix(k, R);
        len = div_radix(len, R);
        pos += (k - q * R) * len;
        k = q;
    }
    return pos;
}

// One in-place decimation-in-frequency stage of radix R over sub-transforms
// of length L = R mm: butterfly (block, j) reads positions base + j + t mm
// (t < R) and writes y_u = (sum_t a_t e^{-2 pi i t u / R}) e^{-2 pi i j u / L}
// back to base + j + u mm.  Butterflies own disjoint positions, so lanes need
// no ordering inside a stage.
template <int R>
__device__ inline void dif_stage(double2* __restrict__ A, int N, int L, const double2* __restrict__ W, int lane)
{
    double2 root[R];  // e^{-2 pi i k / R}
#pragma unroll
    for (int k = 0; k < R; ++k) root[k] = W[k * (N / R)];
    const int mm = L / R;
    const int tw = N / L;  // W step of e^{-2 pi i / L}
    const float inv_mm = 1.0f / (float)mm;
    for (int b = lane; b < N / R; b += 64) {
        int blk = (int)((float)b * inv_mm);  // b < 2^11: exact up to one step, corrected below
        if (blk * mm > b) --blk;
        if ((blk + 1) * mm <= b) ++blk;
        const int j = b - blk * mm;
        const int base = blk * L + j;
        double2 a[R];
#pragma unroll
        for (int t = 0; t < R; ++t) a[t] = A[base + t * mm];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            double2 acc = a[0];
#pragma unroll
            for (int t = 1; t < R; ++t) {
                const double2 w = root[(t * u) % R];
                acc.x = fma(a[t].x, w.x, fma(-a[t].y, w.y, acc.x));
                acc.y = fma(a[t].x, w.y, fma(a[t].y, w.x, acc.y));
            }
            // j u < L: the twiddle index stays below N
            A[base + u * mm] = (u == 0 || j == 0) ? acc : cmul(acc, W[tw * j * u]);
        }
    }
}

// KQ: row elements per lane held in registers (p <= 64 KQ).  The next pair's
// rows are requested as soon as the current pair's are in LDS, so their loads
// fly during the transform.
template <class TX, class TV, int KQ>
__global__ __launch_bounds__(64) void k_dct_fft(uint64_t seed, int p, int m, const TX* __restrict__ X, int64_t n,
                                                int64_t ldx, const double2* __restrict__ W,
                                                const double2* __restrict__ Q, FftPlan fp,
                                                const uint16_t* __restrict__ idx, TV* __restrict__ vals)
{
    extern __shared__ double2 fbuf[];  // p complex: the transform, in place
    __shared__ uint32_t neg[kFftMaxP / 32];
    const int lane = threadIdx.x;
    for (int b = lane; b < (p + 255) / 256; b += 64) {
        const u64x4 blk = sign_block(seed, (uint64_t)b);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            neg[b * 8 + 2 * w] = (uint32_t)blk.w[w];
            neg[b * 8 + 2 * w + 1] = (uint32_t)(blk.w[w] >> 32);
        }
    }
    wave_lds_sync();
    const int64_t npairs = (n + 1) / 2;
    TX xa[KQ], xb[KQ];
    auto load_pair = [&](int64_t pr) {
        const int64_t i1 = 2 * pr, i2 = i1 + 1;
        const TX* x1 = X + i1 * ldx;
        const TX* x2 = X + (i2 < n ? i2 : i1) * ldx;
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            const int j = lane + 64 * q;
            xa[q] = j < p ? x1[j] : (TX)0;
            xb[q] = (j < p && i2 < n) ? x2[j] : (TX)0;
        }
    };
    if ((int64_t)blockIdx.x < npairs) load_pair(blockIdx.x);
    for (int64_t pr = blockIdx.x; pr < npairs; pr += gridDim.x) {
        const int64_t i1 = 2 * pr, i2 = i1 + 1;
        const bool two = i2 < n;
        double2* A = fbuf;
        // signed rows, Makhoul order: x_j goes to j / 2 (j even) or p - 1 - (j - 1) / 2 (j odd)
        double ss1 = 0.0, ss2 = 0.0;
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            const int j = lane + 64 * q;
            if (j < p) {
                const double sg = ((neg[j >> 5] >> (j & 31)) & 1u) ? -1.0 : 1.0;
                const int pos = (j & 1) ? p - 1 - (j >> 1) : (j >> 1);
                const double a = (double)xa[q], b = (double)xb[q];
                ss1 = fma(a, a, ss1);
                ss2 = fma(b, b, ss2);
                A[pos] = make_double2(sg * a, sg * b);
            }
        }
        if (pr + gridDim.x < npairs) load_pair(pr + gridDim.x);
        // the joint transform's rounding is relative to the larger of the two
        // norms: the second sample is scaled by a power of two (exact) that
        // brings its norm within a factor of two of the first's, and scaled
        // back after the separation
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            ss1 += __shfl_xor(ss1, off, 64);
            ss2 += __shfl_xor(ss2, off, 64);
        }
        int e = 0;
        if (ss1 > 0.0 && ss2 > 0.0 && ss1 < INFINITY && ss2 < INFINITY) {
            int e1, e2;
            (void)frexp(ss1, &e1);
            (void)frexp(ss2, &e2);
            e = (e1 - e2) / 2;
        }
        wave_lds_sync();
        if (e != 0) {
            for (int j = lane; j < p; j += 64) A[j].y = ldexp(A[j].y, e);
            wave_lds_sync();
        }
        int len = p;
        for (int f = 0; f < fp.nf; ++f) {
            switch (fp.r[f]) {
                case 2: dif_stage<2>(A, p, len, W, lane); break;
                case 3: dif_stage<3>(A, p, len, W, lane); break;
                case 4: dif_stage<4>(A, p, len, W, lane); break;
                case 5: dif_stage<5>(A, p, len, W, lane); break;
                default: dif_stage<7>(A, p, len, W, lane); break;
            }
            wave_lds_sync();
            len = div_radix(len, fp.r[f]);
        }
        // kept coordinates only: separate the two spectra at k and apply
        // e^{-i pi k / (2p)} s_k (Z_k and Z_{p-k} sit at their digit-reversed positions)
        {
            const uint16_t* ix1 = idx + i1 * (int64_t)m;
            TV* o1 = vals + i1 * (int64_t)m;
            for (int t = lane; t < m; t += 64) {
                const int k = ix1[t];
                const double2 zk = A[digit_rev(k, fp, p)], zm = A[digit_rev(k == 0 ? 0 : p - k, fp, p)];
                const double2 q = Q[k];
                const double r1 = 0.5 * (zk.x + zm.x), i1v = 0.5 * (zk.y - zm.y);
                o1[t] = (TV)fma(q.x, r1, q.y * i1v);
            }
        }
        if (two) {
            const uint16_t* ix2 = idx + i2 * (int64_t)m;
            TV* o2 = vals + i2 * (int64_t)m;
            for (int t = lane; t < m; t += 64) {
                const int k = ix2[t];
                const double2 zk = A[digit_rev(k, fp, p)], zm = A[digit_rev(k == 0 ? 0 : p - k, fp, p)];
                const double2 q = Q[k];
                const double r2 = 0.5 * (zk.y + zm.y), i2v = -0.5 * (zk.x - zm.x);
                o2[t] = (TV)ldexp(fma(q.x, r2, q.y * i2v), -e);
            }
        }
        wave_lds_sync();  // the next pair overwrites the buffer
    }
}

size_t dct_compress_workspace(int p)
{
    if (dct_fast_ok(p)) return 2 * (size_t)p * sizeof(double2) + 256;
    return (size_t)p * (size_t)p * sizeof(double);
}

hipError_t launch_dct_compress(int prec, uint64_t seed, int p, int m, const void* X, int64_t n, int64_t ldx,
                               const uint16_t* idx, void* vals, void* ws, const DeviceInfo& dev, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (p > kDctMaxP) return hipErrorInvalidValue;
    if (dct_fast_ok(p)) {
        double2* W = reinterpret_cast<double2*>(ws);
        double2* Q = reinterpret_cast<double2*>(reinterpret_cast<unsigned char*>(ws) +
                                                ((p * sizeof(double2) + 255) & ~(size_t)255));
        {
            ProfScope ps_("dct_table", s);
            hipLaunchKernelGGL(k_dct_fft_tables, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, s, p, W, Q);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const FftPlan fp = fft_plan(p);
        const size_t lds = (size_t)p * sizeof(double2);
        static bool attr = false;
        if (!attr) {
            const void* ks[] = {reinterpret_cast<const void*>(&k_dct_fft<double, double, 16>),
                                reinterpret_cast<const void*>(&k_dct_fft<double, double, 32>),
                                reinterpret_cast<const void*>(&k_dct_fft<float, float, 16>),
                                reinterpret_cast<const void*>(&k_dct_fft<float, float, 32>)};
            for (const void* k : ks)
                (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kFftMaxP * (int)sizeof(double2));
            attr = true;
        }
        int per_cu = (int)((160 * 1024) / (lds + 1024));
        if (per_cu < 1) per_cu = 1;
        if (per_cu > 16) per_cu = 16;
        const int64_t npairs = (n + 1) / 2;
        int64_t grid = (int64_t)dev.cus * per_cu;
        if (grid > npairs) grid = npairs;
        ProfScope ps_("compress", s);
#define PDS_DCT_FFT(T, KQ)                                                                                   \
    hipLaunchKernelGGL((k_dct_fft<T, T, KQ>), dim3((unsigned)grid), dim3(64), lds, s, seed, p, m,            \
                       reinterpret_cast<const T*>(X), n, ldx, W, Q, fp, idx, reinterpret_cast<T*>(vals))
        if (prec == 0) {
            if (p <= 64 * 16)
                PDS_DCT_FFT(double, 16);
            else
                PDS_DCT_FFT(double, 32);
        } else {
            if (p <= 64 * 16)
                PDS_DCT_FFT(float, 16);
            else
                PDS_DCT_FFT(float, 32);
        }
#undef PDS_DCT_FFT
        return hipGetLastError();
    }
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
