// C ABI of libpds (declared in include/pds.h): argument validation, plans,
// workspace queries and kernel launches.  Validation happens on the host before
// any HIP call, so every error path is testable without a GPU.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/pds.h"
#include "pds_batch.hpp"
#include "pds_device.hpp"
#include "pds_internal.hpp"

struct pds_plan_s {
    int64_t p;
    int64_t m;
    uint64_t seed;
    int32_t prec;
    int32_t gram;       // pds_gram_algo
    int32_t transform;  // pds_transform
    int64_t pg;         // Gram dimension: p, or the next power of two for DCT plans
};

struct pds_batch_s {
    std::vector<pds_batch_desc> descs;
    int T = 0;
    int pmax = 0;
    pds::BatchTuning tune{};
    size_t ws_bytes = 0;
    // bound state
    unsigned char* ws = nullptr;
    std::vector<unsigned char> host_tables;  // staging copy, alive while uploads may be in flight
    pds::BatchTables tables{};
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int kernels_per_kmeans = 0;
};

namespace {

thread_local char g_err[512] = {0};

pds_status fail(pds_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

pds_status hip_fail(hipError_t e, const char* where)
{
    return fail(PDS_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

constexpr int kMaxDevices = 64;
pds::DeviceInfo g_dev[kMaxDevices];
bool g_dev_ok[kMaxDevices] = {false};
std::mutex g_dev_mu;

}  // namespace

namespace pds {

hipError_t device_info(DeviceInfo& info)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < kMaxDevices) {
        std::lock_guard<std::mutex> lk(g_dev_mu);
        if (!g_dev_ok[dev]) {
            int cus = 0;
            e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e != hipSuccess) return e;
            g_dev[dev].cus = cus > 0 ? cus : 1;
            g_dev[dev].device = dev;
            g_dev_ok[dev] = true;
        }
        info = g_dev[dev];
        return hipSuccess;
    }
    info.cus = 256;
    info.device = dev;
    return hipSuccess;
}

// ---- per-kernel event timing ------------------------------------------------
namespace {
struct ProfRecord {
    const char* name;
    hipEvent_t start, stop;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof;
}  // namespace

ProfScope::ProfScope(const char* name, hipStream_t s) : slot_(-1), s_(s)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    ProfRecord r{name, nullptr, nullptr};
    if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess) return;
    if (hipEventRecord(r.start, s) != hipSuccess) return;
    g_prof.push_back(r);
    slot_ = (int)g_prof.size() - 1;
}

ProfScope::~ProfScope()
{
    if (slot_ < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (slot_ < (int)g_prof.size()) (void)hipEventRecord(g_prof[slot_].stop, s_);
}

}  // namespace pds

// Scratch array of pds_kmeans_step_noalloc: one copy per GPU, reserved with
// the code object and kept until the process ends.  In host code `scratch`
// names a host-side stand-in, not device memory: kernels and copies take the
// device address that hipGetSymbolAddress returns for the current device,
// looked up once per device and cached.
static constexpr size_t kNoAllocScratchBytes = PDS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
void* g_scratch_ptr[kMaxDevices] = {nullptr};
std::mutex g_scratch_mu;

// `dev` must be the current device.
hipError_t noalloc_scratch(int dev, void** out)
{
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

static pds_status check_plan(pds_plan plan)
{
    if (!plan) return fail(PDS_E_ARG, "plan is NULL");
    return PDS_OK;
}

// Workspace sizes are computed for the chip the call will run on; host-only
// queries (no current device) size for 256 compute units.
static pds::DeviceInfo query_dev_or_default()
{
    pds::DeviceInfo d;
    d.cus = 256;
    d.device = 0;
    int count = 0;
    if (hipGetDeviceCount(&count) == hipSuccess && count > 0) {
        pds::DeviceInfo q;
        if (pds::device_info(q) == hipSuccess) d = q;
    } else {
        (void)hipGetLastError();
    }
    return d;
}

extern "C" {

pds_status pds_plan_create(pds_plan* out, int64_t p, int64_t m, uint64_t seed, int32_t prec)
{
    if (!out) return fail(PDS_E_ARG, "out is NULL");
    *out = nullptr;
    if (prec != PDS_F64 && prec != PDS_F32 && prec != PDS_SPLIT_BF16)
        return fail(PDS_E_ARG, "unknown precision %d", (int)prec);
    if (p < 2 || p > 65536 || !is_pow2(p))
        return fail(PDS_E_UNSUPPORTED, "p = %lld: must be a power of two in [2, 65536]", (long long)p);
    if (m < 1 || m > p) return fail(PDS_E_M, "m = %lld: must satisfy 1 <= m <= p = %lld", (long long)m, (long long)p);
    pds_plan pl = new (std::nothrow) pds_plan_s;
    if (!pl) return fail(PDS_E_ARG, "out of host memory");
    pl->p = p;
    pl->m = m;
    pl->seed = seed;
    pl->prec = prec;
    pl->gram = PDS_GRAM_AUTO;
    pl->transform = PDS_TRANSFORM_HADAMARD;
    pl->pg = p;
    *out = pl;
    return PDS_OK;
}

pds_status pds_plan_create_dct(pds_plan* out, int64_t p, int64_t m, uint64_t seed, int32_t prec)
{
    if (!out) return fail(PDS_E_ARG, "out is NULL");
    *out = nullptr;
    if (prec != PDS_F64 && prec != PDS_F32 && prec != PDS_SPLIT_BF16)
        return fail(PDS_E_ARG, "unknown precision %d", (int)prec);
    if (p < 2 || p > PDS_DCT_MAX_P)
        return fail(PDS_E_UNSUPPORTED, "p = %lld: DCT plans take p in [2, %d]", (long long)p, (int)PDS_DCT_MAX_P);
    if (m < 1 || m > p) return fail(PDS_E_M, "m = %lld: must satisfy 1 <= m <= p = %lld", (long long)m, (long long)p);
    pds_plan pl = new (std::nothrow) pds_plan_s;
    if (!pl) return fail(PDS_E_ARG, "out of host memory");
    pl->p = p;
    pl->m = m;
    pl->seed = seed;
    pl->prec = prec;
    pl->gram = PDS_GRAM_AUTO;
    pl->transform = PDS_TRANSFORM_DCT;
    int64_t pg = 2;
    while (pg < p) pg <<= 1;
    pl->pg = pg;
    *out = pl;
    return PDS_OK;
}

pds_status pds_plan_transform(pds_plan plan, int32_t* transform)
{
    if (!plan) return fail(PDS_E_ARG, "plan is NULL");
    if (!transform) return fail(PDS_E_ARG, "transform is NULL");
    *transform = plan->transform;
    return PDS_OK;
}

pds_status pds_plan_set_gram(pds_plan plan, int32_t algo)
{
    if (pds_status st = check_plan(plan)) return st;
    if (algo != PDS_GRAM_AUTO && algo != PDS_GRAM_DENSE && algo != PDS_GRAM_SPARSE)
        return fail(PDS_E_ARG, "unknown Gram form %d", (int)algo);
    if (algo == PDS_GRAM_SPARSE && plan->prec == PDS_F64)
        return fail(PDS_E_UNSUPPORTED, "the sparse Gram form takes FP32 values (FP32 and split plans)");
    plan->gram = algo;
    return PDS_OK;
}

pds_status pds_plan_gram(pds_plan plan, int64_t n, int32_t* algo)
{
    if (pds_status st = check_plan(plan)) return st;
    if (!algo) return fail(PDS_E_ARG, "algo is NULL");
    if (n < 0) return fail(PDS_E_ARG, "n < 0");
    pds::DeviceInfo dev = query_dev_or_default();
    *algo = pds::covariance_is_sparse(plan->prec, (int)plan->pg, (int)plan->m, n, dev, plan->gram) ? PDS_GRAM_SPARSE
                                                                                                  : PDS_GRAM_DENSE;
    return PDS_OK;
}

pds_status pds_plan_destroy(pds_plan plan)
{
    delete plan;
    return PDS_OK;
}

pds_status pds_signs(pds_plan plan, int8_t* D_host)
{
    if (pds_status st = check_plan(plan)) return st;
    if (!D_host) return fail(PDS_E_ARG, "D_host is NULL");
    for (int64_t b = 0; b * 256 < plan->p; ++b) {
        pds::u64x4 blk = pds::sign_block(plan->seed, (uint64_t)b);
        for (int64_t j = b * 256; j < plan->p && j < (b + 1) * 256; ++j) {
            uint64_t w = blk.w[(j >> 6) & 3];
            D_host[j] = ((w >> (j & 63)) & 1ull) ? (int8_t)-1 : (int8_t)1;
        }
    }
    return PDS_OK;
}

static size_t kmeans_best_workspace(int prec, int p, int m, int64_t n, int K, const pds::DeviceInfo& dev);
static size_t kmeans_run_workspace(int prec, int p, int m, int64_t n, int K, const pds::DeviceInfo& dev);

pds_status pds_workspace_size(pds_plan plan, int32_t op, int64_t n, int32_t K, size_t* bytes)
{
    if (pds_status st = check_plan(plan)) return st;
    if (!bytes) return fail(PDS_E_ARG, "bytes is NULL");
    if (n < 0) return fail(PDS_E_ARG, "n < 0");
    pds::DeviceInfo dev = query_dev_or_default();
    const int p = (int)plan->p, m = (int)plan->m;
    switch (op) {
        case PDS_OP_COMPRESS:
            *bytes = plan->transform == PDS_TRANSFORM_DCT ? pds::dct_compress_workspace(p)
                                                          : pds::compress_workspace(plan->prec, p, n, dev);
            return PDS_OK;
        case PDS_OP_COVARIANCE:
            *bytes = pds::covariance_workspace(plan->prec, (int)plan->pg, m, n, dev, plan->gram);
            return PDS_OK;
        case PDS_OP_KMEANS:
            if (K < 1 || K > 1024) return fail(PDS_E_ARG, "K = %d: must be in [1, 1024]", (int)K);
            *bytes = pds::kmeans_workspace(plan->prec, p, m, n, K, dev);
            return PDS_OK;
        case PDS_OP_KMEANS2:
            if (K < 1 || K > 1024) return fail(PDS_E_ARG, "K = %d: must be in [1, 1024]", (int)K);
            *bytes = pds::kmeans2_workspace(plan->prec, p, n, K, dev);
            return PDS_OK;
        case PDS_OP_MEAN:
            *bytes = pds::mean_workspace(p, m, n, dev);
            return PDS_OK;
        case PDS_OP_KMEANSPP:
            *bytes = pds::kmeanspp_workspace(n);
            return PDS_OK;
        case PDS_OP_KMEANS_BEST:
            if (K < 1 || K > 1024) return fail(PDS_E_ARG, "K = %d: must be in [1, 1024]", (int)K);
            *bytes = kmeans_best_workspace(plan->prec, p, m, n, K, dev);
            return PDS_OK;
        case PDS_OP_KMEANS_RUN:
            if (K < 1 || K > 1024) return fail(PDS_E_ARG, "K = %d: must be in [1, 1024]", (int)K);
            *bytes = kmeans_run_workspace(plan->prec, p, m, n, K, dev);
            return PDS_OK;
        default:
            return fail(PDS_E_ARG, "unknown op %d", (int)op);
    }
}

pds_status pds_covariance_acc_size(pds_plan plan, size_t* bytes)
{
    if (pds_status st = check_plan(plan)) return st;
    if (!bytes) return fail(PDS_E_ARG, "bytes is NULL");
    *bytes = (size_t)plan->pg * (size_t)plan->pg * sizeof(double);
    return PDS_OK;
}

pds_status pds_compress(pds_plan plan, const void* X, int64_t n, int64_t ldx, uint64_t i0, void* vals, uint16_t* idx,
                        void* ws, size_t ws_bytes, void* stream)
{
    if (pds_status st = check_plan(plan)) return st;
    if (n < 0) return fail(PDS_E_ARG, "n < 0");
    if (n == 0) return PDS_OK;
    if (!X || !vals || !idx) return fail(PDS_E_ARG, "X, vals and idx must be non-NULL");
    if (ldx < plan->p) return fail(PDS_E_ARG, "ldx = %lld < p = %lld", (long long)ldx, (long long)plan->p);
    pds::DeviceInfo dev;
    hipError_t e = pds::device_info(dev);
    if (e != hipSuccess) return hip_fail(e, "pds_compress");
    const bool dct = plan->transform == PDS_TRANSFORM_DCT;
    const size_t need = dct ? pds::dct_compress_workspace((int)plan->p)
                            : pds::compress_workspace(plan->prec, (int)plan->p, n, dev);
    if (need > 0 && (!ws || ws_bytes < need))
        return fail(PDS_E_WORKSPACE, "compress needs %zu workspace bytes, got %zu", need, ws ? ws_bytes : (size_t)0);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!dct && pds::compress_fused_ok(plan->prec, (int)plan->p, X, ldx)) {
        e = pds::launch_compress_fused(plan->seed, (int)plan->p, (int)plan->m, reinterpret_cast<const float*>(X), n,
                                       ldx, i0, reinterpret_cast<float*>(vals), idx, dev, s);
        if (e != hipSuccess) return hip_fail(e, "compress (fused sampler)");
        return PDS_OK;
    }
    e = pds::launch_sample_indices(plan->seed, (int)plan->p, (int)plan->m, n, i0, idx, dev, s);
    if (e != hipSuccess) return hip_fail(e, "sample_indices");
    if (dct) {
        e = pds::launch_dct_compress(plan->prec, plan->seed, (int)plan->p, (int)plan->m, X, n, ldx, idx, vals, ws, dev,
                                     s);
        if (e != hipSuccess) return hip_fail(e, "compress (DCT)");
        return PDS_OK;
    }
    e = pds::launch_compress(plan->prec, plan->seed, (int)plan->p, (int)plan->m, X, n, ldx, idx, vals, ws, ws_bytes,
                             dev, s);
    if (e != hipSuccess) return hip_fail(e, "compress");
    return PDS_OK;
}

pds_status pds_covariance(pds_plan plan, const void* vals, const uint16_t* idx, int64_t n, double* acc,
                          int32_t finalize, int64_t n_total, double* C_out, void* ws, size_t ws_bytes, void* stream)
{
    if (pds_status st = check_plan(plan)) return st;
    if (plan->m < 2) return fail(PDS_E_M, "covariance needs m >= 2 (it divides by m - 1)");
    if (n < 0) return fail(PDS_E_ARG, "n < 0");
    if (!acc) return fail(PDS_E_ARG, "acc is NULL");
    if (n > 0 && (!vals || !idx)) return fail(PDS_E_ARG, "vals and idx must be non-NULL");
    if (finalize && (!C_out || n_total < 1)) return fail(PDS_E_ARG, "finalize needs C_out and n_total >= 1");
    if (n == 0 && !finalize) return PDS_OK;
    pds::DeviceInfo dev;
    hipError_t e = pds::device_info(dev);
    if (e != hipSuccess) return hip_fail(e, "pds_covariance");
    const size_t need = pds::covariance_workspace(plan->prec, (int)plan->pg, (int)plan->m, n, dev, plan->gram);
    if (need > 0 && (!ws || ws_bytes < need))
        return fail(PDS_E_WORKSPACE, "covariance needs %zu workspace bytes, got %zu", need, ws ? ws_bytes : (size_t)0);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (n > 0) {
        e = pds::launch_covariance_accumulate(plan->prec, (int)plan->pg, (int)plan->m, vals, idx, n, acc, ws, ws_bytes,
                                              dev, s, plan->gram);
        if (e != hipSuccess) return hip_fail(e, "covariance accumulate");
    }
    if (finalize) {
        e = pds::launch_covariance_finalize(plan->prec, (int)plan->p, (int)plan->pg, (int)plan->m, n_total, acc, C_out,
                                            s);
        if (e != hipSuccess) return hip_fail(e, "covariance finalize");
    }
    return PDS_OK;
}

pds_status pds_sample_mean(pds_plan plan, const void* vals, const uint16_t* idx, int64_t n, double* acc,
                           int32_t finalize, int64_t n_total, double* mean_out, void* ws, size_t ws_bytes,
                           void* stream)
{
    if (pds_status st = check_plan(plan)) return st;
    if (n < 0) return fail(PDS_E_ARG, "n < 0");
    if (!acc) return fail(PDS_E_ARG, "acc is NULL");
    if (n > 0 && (!vals || !idx)) return fail(PDS_E_ARG, "vals and idx must be non-NULL");
    if (finalize && (!mean_out || n_total < 1)) return fail(PDS_E_ARG, "finalize needs mean_out and n_total >= 1");
    if (finalize && mean_out == acc) return fail(PDS_E_ARG, "acc and mean_out must not alias");
    if (n == 0 && !finalize) return PDS_OK;
    pds::DeviceInfo dev;
    hipError_t e = pds::device_info(dev);
    if (e != hipSuccess) return hip_fail(e, "pds_sample_mean");
    const size_t need = pds::mean_workspace((int)plan->p, (int)plan->m, n, dev);
    if (need > 0 && (!ws || ws_bytes < need))
        return fail(PDS_E_WORKSPACE, "sample_mean needs %zu workspace bytes, got %zu", need, ws ? ws_bytes : (size_t)0);
    e = pds::launch_mean(plan->prec, (int)plan->p, (int)plan->m, vals, idx, n, acc, finalize, n_total, mean_out, ws,
                         dev, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "sample_mean");
    return PDS_OK;
}

pds_status pds_pad_rows(const void* X, int32_t x_prec, int64_t n, int64_t p_data, int64_t ldx, void* Xp, int64_t p_pad,
                        void* stream)
{
    if (n < 0) return fail(PDS_E_ARG, "n < 0");
    if (n == 0) return PDS_OK;
    if (!X || !Xp) return fail(PDS_E_ARG, "X and Xp must be non-NULL");
    if (p_data < 1 || p_pad < p_data || ldx < p_data)
        return fail(PDS_E_ARG, "need 1 <= p_data <= p_pad and ldx >= p_data (p_data = %lld, p_pad = %lld, ldx = %lld)",
                    (long long)p_data, (long long)p_pad, (long long)ldx);
    if (x_prec != PDS_F64 && x_prec != PDS_F32) return fail(PDS_E_ARG, "x_prec must be PDS_F64 or PDS_F32");
    if (X == Xp) return fail(PDS_E_ARG, "X and Xp must not alias");
    pds::DeviceInfo dev;
    hipError_t e = pds::device_info(dev);
    if (e != hipSuccess) return hip_fail(e, "pds_pad_rows");
    e = pds::launch_pad_rows(x_prec == PDS_F64, X, n, p_data, ldx, Xp, p_pad, dev, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "pad_rows");
    return PDS_OK;
}

pds_status pds_explained_variance(const double* U, int32_t k, const void* X, int32_t x_prec, int64_t n, int64_t p,
                                  int64_t ldx, double* out2, void* ws, size_t ws_bytes, void* stream)
{
    if (!U || !X || !out2) return fail(PDS_E_ARG, "U, X and out2 must be non-NULL");
    if (k < 1 || k > pds::explained_max_k())
        return fail(PDS_E_ARG, "k = %d: must be in [1, %d]", (int)k, pds::explained_max_k());
    if (n < 1 || p < 1 || p > (1 << 30)) return fail(PDS_E_ARG, "n = %lld, p = %lld", (long long)n, (long long)p);
    if (ldx < p) return fail(PDS_E_ARG, "ldx = %lld < p = %lld", (long long)ldx, (long long)p);
    if (x_prec != PDS_F64 && x_prec != PDS_F32) return fail(PDS_E_ARG, "x_prec must be PDS_F64 or PDS_F32");
    if (!ws || ws_bytes < pds::explained_workspace())
        return fail(PDS_E_WORKSPACE, "explained_variance needs %zu workspace bytes", pds::explained_workspace());
    hipError_t e = pds::launch_explained(U, (int)k, X, x_prec == PDS_F64, n, (int)p, ldx, out2, ws,
                                         reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "explained_variance");
    return PDS_OK;
}

pds_status pds_kmeanspp(pds_plan plan, const void* vals, const uint16_t* idx, int64_t n, int32_t K, int32_t replicate,
                        double* centers, int64_t* chosen, void* ws, size_t ws_bytes, void* stream)
{
    if (pds_status st = check_plan(plan)) return st;
    if (n < 1) return fail(PDS_E_ARG, "kmeanspp: n = %lld < 1", (long long)n);
    if (K < 1 || K > 1024) return fail(PDS_E_ARG, "K = %d: must be in [1, 1024]", (int)K);
    if (replicate < 0) return fail(PDS_E_ARG, "replicate = %d < 0", (int)replicate);
    if (!vals || !idx || !centers) return fail(PDS_E_ARG, "vals, idx and centers must be non-NULL");
    const size_t need = pds::kmeanspp_workspace(n);
    if (!ws || ws_bytes < need)
        return fail(PDS_E_WORKSPACE, "kmeanspp needs %zu workspace bytes, got %zu", need, ws ? ws_bytes : (size_t)0);
    hipError_t e = pds::launch_kmeanspp(plan->prec, (int)plan->p, (int)plan->m, vals, idx, n, K, plan->seed,
                                        (uint64_t)replicate, centers, chosen, ws, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kmeanspp");
    return PDS_OK;
}

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace of pds_kmeans_best: the K-means step's, the seeding's, two center
// buffers and one assignment buffer.
static size_t kmeans_best_workspace(int prec, int p, int m, int64_t n, int K, const pds::DeviceInfo& dev)
{
    return al256(pds::kmeans_workspace(prec, p, m, n, K, dev)) + al256(pds::kmeanspp_workspace(n)) +
           2 * al256((size_t)K * p * sizeof(double)) + al256((size_t)n * sizeof(int32_t));
}

// Workspace of pds_kmeans_run: the K-means step's and one center buffer.
static size_t kmeans_run_workspace(int prec, int p, int m, int64_t n, int K, const pds::DeviceInfo& dev)
{
    return al256(pds::kmeans_workspace(prec, p, m, n, K, dev)) + al256((size_t)K * p * sizeof(double));
}

pds_status pds_kmeans_best(pds_plan plan, const void* vals, const uint16_t* idx, int64_t n, int32_t K, int32_t T,
                           int32_t R, double* centers_out, int32_t* assign_out, double* objectives, int32_t* best,
                           void* ws, size_t ws_bytes, void* stream)
{
    if (pds_status st = check_plan(plan)) return st;
    if (n < 1) return fail(PDS_E_ARG, "kmeans_best: n = %lld < 1", (long long)n);
    if (K < 1 || K > 1024) return fail(PDS_E_ARG, "K = %d: must be in [1, 1024]", (int)K);
    if (T < 1 || R < 1 || R > 1024) return fail(PDS_E_ARG, "T = %d, R = %d: need T >= 1 and 1 <= R <= 1024", T, R);
    if (!vals || !idx || !centers_out || !assign_out || !objectives || !best)
        return fail(PDS_E_ARG, "vals, idx, centers_out, assign_out, objectives and best must be non-NULL");
    pds::DeviceInfo dev;
    hipError_t e = pds::device_info(dev);
    if (e != hipSuccess) return hip_fail(e, "pds_kmeans_best");
    const int p = (int)plan->p, m = (int)plan->m;
    const size_t need = kmeans_best_workspace(plan->prec, p, m, n, K, dev);
    if (!ws || ws_bytes < need)
        return fail(PDS_E_WORKSPACE, "kmeans_best needs %zu workspace bytes, got %zu", need, ws ? ws_bytes : (size_t)0);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    const size_t km_bytes = pds::kmeans_workspace(plan->prec, p, m, n, K, dev);
    void* km_ws = w;
    w += al256(km_bytes);
    void* pp_ws = w;
    w += al256(pds::kmeanspp_workspace(n));
    double* ca = reinterpret_cast<double*>(w);
    w += al256((size_t)K * p * sizeof(double));
    double* cb = reinterpret_cast<double*>(w);
    w += al256((size_t)K * p * sizeof(double));
    int32_t* asg = reinterpret_cast<int32_t*>(w);
    for (int r = 0; r < R; ++r) {
        e = pds::launch_kmeanspp(plan->prec, p, m, vals, idx, n, K, plan->seed, (uint64_t)r, ca, nullptr, pp_ws, s);
        if (e != hipSuccess) return hip_fail(e, "kmeans_best seeding");
        double* a = ca;
        double* c = cb;
        for (int t = 0; t < T; ++t) {
            // after the first round the workspace holds this data's per-workgroup scales
            e = pds::launch_kmeans_step(plan->prec, p, m, vals, idx, n, K, a, c, asg,
                                        objectives + (int64_t)r * T + t, km_ws, km_bytes, dev, s, r > 0 || t > 0);
            if (e != hipSuccess) return hip_fail(e, "kmeans_best round");
            std::swap(a, c);
        }
        e = pds::launch_keep_best(r, T, objectives, a, (int64_t)K * p, asg, n, centers_out, assign_out, best, dev, s);
        if (e != hipSuccess) return hip_fail(e, "kmeans_best keep");
    }
    return PDS_OK;
}

pds_status pds_kmeans_step(pds_plan plan, const void* vals, const uint16_t* idx, int64_t n, int32_t K,
                           const double* centers_in, double* centers_out, int32_t* assign, double* objective, void* ws,
                           size_t ws_bytes, void* stream)
{
    if (pds_status st = check_plan(plan)) return st;
    if (n < 0) return fail(PDS_E_ARG, "n < 0");
    if (K < 1 || K > 1024) return fail(PDS_E_ARG, "K = %d: must be in [1, 1024]", (int)K);
    if (n == 0) return PDS_OK;
    if (!vals || !idx || !centers_in || !centers_out || !assign || !objective)
        return fail(PDS_E_ARG, "vals, idx, centers_in, centers_out, assign and objective must be non-NULL");
    if (centers_in == centers_out) return fail(PDS_E_ARG, "centers_in and centers_out must not alias");
    pds::DeviceInfo dev;
    hipError_t e = pds::device_info(dev);
    if (e != hipSuccess) return hip_fail(e, "pds_kmeans_step");
    const size_t need = pds::kmeans_workspace(plan->prec, (int)plan->p, (int)plan->m, n, K, dev);
    if (!ws || ws_bytes < need)
        return fail(PDS_E_WORKSPACE, "kmeans_step needs %zu workspace bytes, got %zu", need, ws ? ws_bytes : (size_t)0);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    e = pds::launch_kmeans_step(plan->prec, (int)plan->p, (int)plan->m, vals, idx, n, K, centers_in, centers_out,
                                assign, objective, ws, ws_bytes, dev, s);
    if (e != hipSuccess) return hip_fail(e, "kmeans_step");
    return PDS_OK;
}

pds_status pds_kmeans_run(pds_plan plan, const void* vals, const uint16_t* idx, int64_t n, int32_t K, int32_t T,
                          const double* centers_in, double* centers_out, int32_t* assign, double* objectives, void* ws,
                          size_t ws_bytes, void* stream)
{
    if (pds_status st = check_plan(plan)) return st;
    if (n < 0) return fail(PDS_E_ARG, "n < 0");
    if (K < 1 || K > 1024) return fail(PDS_E_ARG, "K = %d: must be in [1, 1024]", (int)K);
    if (T < 1) return fail(PDS_E_ARG, "T = %d < 1", (int)T);
    if (n == 0) return PDS_OK;
    if (!vals || !idx || !centers_in || !centers_out || !assign || !objectives)
        return fail(PDS_E_ARG, "vals, idx, centers_in, centers_out, assign and objectives must be non-NULL");
    if (centers_in == centers_out) return fail(PDS_E_ARG, "centers_in and centers_out must not alias");
    pds::DeviceInfo dev;
    hipError_t e = pds::device_info(dev);
    if (e != hipSuccess) return hip_fail(e, "pds_kmeans_run");
    const int p = (int)plan->p, m = (int)plan->m;
    const size_t km_bytes = pds::kmeans_workspace(plan->prec, p, m, n, K, dev);
    const size_t need = kmeans_run_workspace(plan->prec, p, m, n, K, dev);
    if (!ws || ws_bytes < need)
        return fail(PDS_E_WORKSPACE, "kmeans_run needs %zu workspace bytes, got %zu", need, ws ? ws_bytes : (size_t)0);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    double* tmp = reinterpret_cast<double*>(w + al256(km_bytes));
    const double* in = centers_in;
    for (int t = 0; t < T; ++t) {
        // rounds alternate between the two buffers so that the last one writes centers_out
        double* out = ((T - 1 - t) % 2 == 0) ? centers_out : tmp;
        e = pds::launch_kmeans_step(plan->prec, p, m, vals, idx, n, K, in, out, assign, objectives + t, w, km_bytes,
                                    dev, s, t > 0);
        if (e != hipSuccess) return hip_fail(e, "kmeans_run round");
        in = out;
    }
    return PDS_OK;
}

pds_status pds_kmeans_step_noalloc(pds_plan plan, const void* vals, const uint16_t* idx, int64_t n, int32_t K,
                                   const double* centers_in, double* centers_out, int32_t* assign,
                                   double* objective, void* stream)
{
    if (pds_status st = check_plan(plan)) return st;
    if (n < 0) return fail(PDS_E_ARG, "n < 0");
    if (K < 1 || K > 1024) return fail(PDS_E_ARG, "K = %d: must be in [1, 1024]", (int)K);
    if (n == 0) return PDS_OK;
    if (!vals || !idx || !centers_in || !centers_out || !assign || !objective)
        return fail(PDS_E_ARG, "vals, idx, centers_in, centers_out, assign and objective must be non-NULL");
    if (centers_in == centers_out) return fail(PDS_E_ARG, "centers_in and centers_out must not alias");
    pds::DeviceInfo dev;
    hipError_t e = pds::device_info(dev);
    if (e != hipSuccess) return hip_fail(e, "pds_kmeans_step_noalloc");
    const size_t need = pds::kmeans_workspace(plan->prec, (int)plan->p, (int)plan->m, n, K, dev);
    if (need > kNoAllocScratchBytes)
        return fail(PDS_E_WORKSPACE,
                    "kmeans_step_noalloc: this call needs %zu workspace bytes, more than the %zu bytes of the "
                    "library's scratch array; call pds_kmeans_step with a workspace instead",
                    need, kNoAllocScratchBytes);
    void* ws = nullptr;
    e = noalloc_scratch(dev.device, &ws);
    if (e != hipSuccess) return hip_fail(e, "kmeans_step_noalloc: address of the scratch array");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    e = pds::launch_kmeans_step(plan->prec, (int)plan->p, (int)plan->m, vals, idx, n, K, centers_in, centers_out,
                                assign, objective, ws, kNoAllocScratchBytes, dev, s);
    if (e != hipSuccess) return hip_fail(e, "kmeans_step_noalloc");
    return PDS_OK;
}

pds_status pds_kmeans_2pass(pds_plan plan, const void* X, int64_t n, int64_t ldx, int32_t K, const int32_t* c_hat,
                            const double* mu_hat, double* mu_out, int32_t* c_out, void* ws, size_t ws_bytes,
                            void* stream)
{
    if (pds_status st = check_plan(plan)) return st;
    if (n < 0) return fail(PDS_E_ARG, "n < 0");
    if (K < 1 || K > 1024) return fail(PDS_E_ARG, "K = %d: must be in [1, 1024]", (int)K);
    if (!pds::kmeans2_supported(K)) return fail(PDS_E_ARG, "K = %d: too many clusters for the second pass", (int)K);
    if (n == 0) return PDS_OK;
    if (!X || !c_hat || !mu_hat || !mu_out || !c_out)
        return fail(PDS_E_ARG, "X, c_hat, mu_hat, mu_out and c_out must be non-NULL");
    if (ldx < plan->p) return fail(PDS_E_ARG, "ldx = %lld < p = %lld", (long long)ldx, (long long)plan->p);
    if (mu_hat == mu_out) return fail(PDS_E_ARG, "mu_hat and mu_out must not alias");
    pds::DeviceInfo dev;
    hipError_t e = pds::device_info(dev);
    if (e != hipSuccess) return hip_fail(e, "pds_kmeans_2pass");
    const size_t need = pds::kmeans2_workspace(plan->prec, (int)plan->p, n, K, dev);
    if (!ws || ws_bytes < need)
        return fail(PDS_E_WORKSPACE, "kmeans_2pass needs %zu workspace bytes, got %zu", need, ws ? ws_bytes : (size_t)0);
    e = pds::launch_kmeans_2pass(plan->prec, (int)plan->p, X, n, ldx, K, c_hat, mu_hat, mu_out, c_out, ws, ws_bytes,
                                 dev, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kmeans_2pass");
    return PDS_OK;
}

pds_status pds_unmix(pds_plan plan, const double* centers_pre, int32_t K, double* centers_out, void* stream)
{
    if (pds_status st = check_plan(plan)) return st;
    if (K < 1) return fail(PDS_E_ARG, "K < 1");
    if (!centers_pre || !centers_out) return fail(PDS_E_ARG, "centers must be non-NULL");
    if (centers_pre == centers_out) return fail(PDS_E_ARG, "centers_pre and centers_out must not alias");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = plan->transform == PDS_TRANSFORM_DCT
                       ? pds::launch_dct_unmix(plan->seed, (int)plan->p, centers_pre, K, centers_out, s)
                       : pds::launch_unmix(plan->seed, (int)plan->p, centers_pre, K, centers_out, s);
    if (e != hipSuccess) return hip_fail(e, "unmix");
    return PDS_OK;
}

// ---- learned m-selector ------------------------------------------------------

pds_status pds_row_moments(const float* X, int64_t n, int64_t p, int64_t ldx, double* out, void* stream)
{
    if (n < 0 || p < 1 || p > (1 << 30)) return fail(PDS_E_ARG, "row_moments: n = %lld, p = %lld", (long long)n, (long long)p);
    if (ldx < p) return fail(PDS_E_ARG, "ldx = %lld < p = %lld", (long long)ldx, (long long)p);
    if (n == 0) return PDS_OK;
    if (!X || !out) return fail(PDS_E_ARG, "X and out must be non-NULL");
    pds::DeviceInfo dev;
    hipError_t e = pds::device_info(dev);
    if (e == hipSuccess) e = pds::launch_row_moments(X, n, (int)p, ldx, out, dev, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "row_moments");
    return PDS_OK;
}

pds_status pds_frob_diff(const double* A, const double* B, int64_t len, double* out2, void* ws, size_t ws_bytes,
                         void* stream)
{
    if (len < 1) return fail(PDS_E_ARG, "frob_diff: len = %lld < 1", (long long)len);
    if (!A || !B || !out2) return fail(PDS_E_ARG, "A, B and out2 must be non-NULL");
    if (!ws || ws_bytes < pds::frob_workspace())
        return fail(PDS_E_WORKSPACE, "frob_diff needs %zu workspace bytes", pds::frob_workspace());
    hipError_t e = pds::launch_frob_diff(A, B, len, out2, reinterpret_cast<double*>(ws),
                                         reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "frob_diff");
    return PDS_OK;
}

namespace {

// Workspace of the m-selector calls on n rows of a plan with m = p:
// idx (n x p u16) | Y (n x p f32) | moments raw, y (n x 3 f64 each) |
// acc, C (p x p f64 each) | covariance workspace | Frobenius partials | sums
struct MselLayout {
    size_t idx, y, mr, my, acc, c, cov, frob, sums, total;
};

size_t up256(size_t v) { return (v + 255) & ~(size_t)255; }

MselLayout msel_layout(int p, int64_t n, const pds::DeviceInfo& dev)
{
    MselLayout L;
    size_t o = 0;
    L.idx = o;
    o += up256((size_t)n * p * sizeof(uint16_t));
    L.y = o;
    o += up256((size_t)n * p * sizeof(float));
    L.mr = o;
    o += up256((size_t)n * 3 * sizeof(double));
    L.my = o;
    o += up256((size_t)n * 3 * sizeof(double));
    L.acc = o;
    o += up256((size_t)p * p * sizeof(double));
    L.c = o;
    o += up256((size_t)p * p * sizeof(double));
    L.cov = o;
    o += up256(pds::covariance_workspace(PDS_F32, p, p, n, dev, PDS_GRAM_DENSE) + pds::compress_workspace(PDS_F32, p, n, dev));
    L.frob = o;
    o += up256(pds::frob_workspace());
    L.sums = o;
    o += 256;
    L.total = o;
    return L;
}

pds_status msel_check_plan(pds_plan plan)
{
    if (pds_status st = check_plan(plan)) return st;
    if (plan->m != plan->p) return fail(PDS_E_M, "m-selector calls need a plan with m = p (got m = %lld, p = %lld)",
                                        (long long)plan->m, (long long)plan->p);
    if (plan->prec != PDS_F32) return fail(PDS_E_ARG, "m-selector calls need a PDS_F32 plan");
    if (plan->transform != PDS_TRANSFORM_HADAMARD)
        return fail(PDS_E_UNSUPPORTED, "m-selector calls need a Hadamard plan");
    return PDS_OK;
}

// y = H D x of rows 0..n-1, their moments and the raw rows' moments, then
// C = (1/n) sum y y^T into C and ||C||_F^2 into sums[1]
pds_status msel_exact(pds_plan plan, const float* X, int64_t n, int64_t ldx, unsigned char* w, const MselLayout& L,
                      double* C, const pds::DeviceInfo& dev, hipStream_t s)
{
    const int p = (int)plan->p;
    uint16_t* idx = reinterpret_cast<uint16_t*>(w + L.idx);
    float* Y = reinterpret_cast<float*>(w + L.y);
    double* acc = reinterpret_cast<double*>(w + L.acc);
    void* cws = w + L.cov;
    const size_t cws_bytes = L.frob - L.cov;
    hipError_t e = pds::launch_zero_f64(acc, (int64_t)p * p, dev, s);
    if (e == hipSuccess) e = pds::launch_sample_indices(plan->seed, p, p, n, 0, idx, dev, s);
    if (e == hipSuccess) e = pds::launch_compress(PDS_F32, plan->seed, p, p, X, n, ldx, idx, Y, cws, cws_bytes, dev, s);
    if (e == hipSuccess) e = pds::launch_row_moments(X, n, p, ldx, reinterpret_cast<double*>(w + L.mr), dev, s);
    if (e == hipSuccess) e = pds::launch_row_moments(Y, n, p, p, reinterpret_cast<double*>(w + L.my), dev, s);
    if (e == hipSuccess) e = pds::launch_covariance_accumulate(PDS_F32, p, p, Y, idx, n, acc, cws, cws_bytes, dev, s, PDS_GRAM_DENSE);
    if (e == hipSuccess) e = pds::launch_covariance_finalize(PDS_F32, p, p, p, n, acc, C, s);
    if (e == hipSuccess)
        e = pds::launch_frob_diff(C, C, (int64_t)p * p, reinterpret_cast<double*>(w + L.sums),
                                  reinterpret_cast<double*>(w + L.frob), s);
    if (e != hipSuccess) return hip_fail(e, "m-selector exact covariance");
    return PDS_OK;
}

}  // namespace

pds_status pds_msel_workspace_size(pds_plan plan, int64_t n, size_t* bytes)
{
    if (pds_status st = msel_check_plan(plan)) return st;
    if (!bytes) return fail(PDS_E_ARG, "bytes is NULL");
    if (n < 2) return fail(PDS_E_ARG, "n = %lld < 2", (long long)n);
    *bytes = msel_layout((int)plan->p, n, query_dev_or_default()).total;
    return PDS_OK;
}

pds_status pds_msel_label(pds_plan plan, const float* X, int64_t n, int64_t ldx, double target, int32_t* m_out,
                          double* C_out, void* ws, size_t ws_bytes, void* stream)
{
    if (pds_status st = msel_check_plan(plan)) return st;
    if (n < 2) return fail(PDS_E_ARG, "n = %lld < 2", (long long)n);
    if (ldx < plan->p) return fail(PDS_E_ARG, "ldx = %lld < p = %lld", (long long)ldx, (long long)plan->p);
    if (!X || !m_out) return fail(PDS_E_ARG, "X and m_out must be non-NULL");
    if (!(target > 0.0) || !isfinite(target)) return fail(PDS_E_ARG, "target must be positive and finite");
    pds::DeviceInfo dev;
    hipError_t e = pds::device_info(dev);
    if (e != hipSuccess) return hip_fail(e, "pds_msel_label");
    const MselLayout L = msel_layout((int)plan->p, n, dev);
    if (!ws || ws_bytes < L.total) return fail(PDS_E_WORKSPACE, "msel_label needs %zu workspace bytes", L.total);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double* C = C_out ? C_out : reinterpret_cast<double*>(w + L.c);
    if (pds_status st = msel_exact(plan, X, n, ldx, w, L, C, dev, s)) return st;
    e = pds::launch_msel_label(reinterpret_cast<double*>(w + L.my), n, (int)plan->p,
                               reinterpret_cast<double*>(w + L.sums) + 1, target, m_out, s);
    if (e != hipSuccess) return hip_fail(e, "msel_label");
    return PDS_OK;
}

pds_status pds_msel_features(pds_plan plan, const float* X, int64_t n, int64_t ldx, int64_t nsub, double target,
                             float* feats, void* ws, size_t ws_bytes, void* stream)
{
    if (pds_status st = msel_check_plan(plan)) return st;
    if (nsub < 2 || nsub > 1024 || nsub > n)
        return fail(PDS_E_ARG, "nsub = %lld: must satisfy 2 <= nsub <= min(n, 1024)", (long long)nsub);
    if (ldx < plan->p) return fail(PDS_E_ARG, "ldx = %lld < p = %lld", (long long)ldx, (long long)plan->p);
    if (!X || !feats) return fail(PDS_E_ARG, "X and feats must be non-NULL");
    if (!(target > 0.0) || !isfinite(target)) return fail(PDS_E_ARG, "target must be positive and finite");
    pds::DeviceInfo dev;
    hipError_t e = pds::device_info(dev);
    if (e != hipSuccess) return hip_fail(e, "pds_msel_features");
    const MselLayout L = msel_layout((int)plan->p, nsub, dev);
    if (!ws || ws_bytes < L.total) return fail(PDS_E_WORKSPACE, "msel_features needs %zu workspace bytes", L.total);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (pds_status st = msel_exact(plan, X, nsub, ldx, w, L, reinterpret_cast<double*>(w + L.c), dev, s)) return st;
    e = pds::launch_msel_features(reinterpret_cast<double*>(w + L.mr), reinterpret_cast<double*>(w + L.my), (int)nsub,
                                  n, (int)plan->p, reinterpret_cast<double*>(w + L.sums) + 1, target, feats, s);
    if (e != hipSuccess) return hip_fail(e, "msel_features");
    return PDS_OK;
}

int32_t pds_mlp_param_count(void) { return pds::mlp_param_count(); }

static pds_status mlp_check_B(int64_t B)
{
    if (B < 1 || B > (int64_t)1 << 26) return fail(PDS_E_ARG, "B = %lld: must be in [1, 2^26]", (long long)B);
    return PDS_OK;
}

pds_status pds_mlp_forward(const float* params, const float* feats, const float* mu, const float* sd, int64_t B,
                           float* acts, float* pred, void* stream)
{
    if (pds_status st = mlp_check_B(B)) return st;
    if (!params || !feats || !mu || !sd || !acts || !pred)
        return fail(PDS_E_ARG, "params, feats, mu, sd, acts and pred must be non-NULL");
    hipError_t e = pds::launch_mlp_forward(params, feats, mu, sd, (int)B, acts, pred,
                                           reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mlp_forward");
    return PDS_OK;
}

pds_status pds_mlp_backward(const float* params, const float* acts, const float* pred, const float* target, int64_t B,
                            float tau, float* ws, size_t ws_bytes, float* grad, float* loss, void* stream)
{
    if (pds_status st = mlp_check_B(B)) return st;
    if (!params || !acts || !pred || !target || !grad || !loss)
        return fail(PDS_E_ARG, "params, acts, pred, target, grad and loss must be non-NULL");
    if (!(tau > 0.0f && tau < 1.0f)) return fail(PDS_E_ARG, "tau must lie in (0, 1)");
    const size_t need = (size_t)B * 130 * sizeof(float);
    if (!ws || ws_bytes < need) return fail(PDS_E_WORKSPACE, "mlp_backward needs %zu workspace bytes", need);
    float* sig = ws;
    float* lossb = ws + (size_t)B * 129;
    hipError_t e = pds::launch_mlp_backward(params, acts, pred, target, (int)B, tau, sig, lossb, grad, loss,
                                            reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mlp_backward");
    return PDS_OK;
}

pds_status pds_mlp_adam(float* params, const float* grad, float* m1, float* m2, int32_t step, float lr, float beta1,
                        float beta2, float eps, void* stream)
{
    if (!params || !grad || !m1 || !m2) return fail(PDS_E_ARG, "params, grad, m1 and m2 must be non-NULL");
    if (step < 1) return fail(PDS_E_ARG, "step must be >= 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && lr >= 0.0f))
        return fail(PDS_E_ARG, "Adam needs 0 <= beta < 1, eps > 0, lr >= 0");
    hipError_t e = pds::launch_adam(params, grad, m1, m2, pds::mlp_param_count(), lr, beta1, beta2, eps, step,
                                    reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mlp_adam");
    return PDS_OK;
}

pds_status pds_mlp_pack_bf16(const float* params, uint16_t* params_bf16, void* stream)
{
    if (!params || !params_bf16) return fail(PDS_E_ARG, "params and params_bf16 must be non-NULL");
    hipError_t e = pds::launch_pack_bf16(params, pds::mlp_param_count(), params_bf16,
                                         reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mlp_pack_bf16");
    return PDS_OK;
}

pds_status pds_msel_predict(const uint16_t* params_bf16, const float* feats, const float* mu, const float* sd,
                            int64_t B, float gamma_min, float gamma_max, float gamma_fallback, float* gamma,
                            void* stream)
{
    if (pds_status st = mlp_check_B(B)) return st;
    if (!params_bf16 || !feats || !mu || !sd || !gamma)
        return fail(PDS_E_ARG, "params_bf16, feats, mu, sd and gamma must be non-NULL");
    if (!(gamma_min > 0.0f && gamma_min <= gamma_max && isfinite(gamma_max) && isfinite(gamma_fallback)))
        return fail(PDS_E_ARG, "need 0 < gamma_min <= gamma_max and a finite fallback");
    hipError_t e = pds::launch_mlp_predict_bf16(params_bf16, feats, mu, sd, (int)B, gamma_min, gamma_max,
                                                gamma_fallback, gamma, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "msel_predict");
    return PDS_OK;
}

// ---- batched form --------------------------------------------------------------

namespace {

constexpr int kBatchSpwCand[3] = {16, 32, 64};
constexpr int kBatchCchunkCand[3] = {4096, 16384, 65536};

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Workspace offsets (bytes) of the batch tables; sized for the smallest
// candidate chunks so that re-tuning never grows the workspace.
struct BatchOffsets {
    size_t sets, gp, ap, cp, up, tp, ct, cmax, vmax, pobj, psum, pcnt, vt, it, dist, rlist, rcount, total;
};

int accum_kg(int K, int p)
{
    int kg = pds::kBatchAccumEntries / p;
    if (kg < 1) kg = 1;
    if (kg > K) kg = K;
    return kg;
}

// Samples per accumulation chunk of a set: the tuned length, halved while an
// item (a chunk and a cluster group) would hold more than kAccItemEntries kept
// entries on average (large m with few cluster groups), so that no single item
// keeps its workgroup busy long after the others have finished.
constexpr double kAccItemEntries = 262144.0;

int accum_chunk(int64_t m, int K, int p, int tuned)
{
    const double per = (double)m * (double)accum_kg(K, p) / (double)K;  // entries per sample and item
    int c = tuned;
    while (c > 256 && (double)c * per > kAccItemEntries) c >>= 1;
    return c;
}

BatchOffsets batch_offsets(const pds_batch_s& b)
{
    const size_t ns = b.descs.size();
    size_t ct = 0, pobj = 0, part = 0, tiles = 0, nsamp = 0;
    for (const auto& d : b.descs) {
        const int64_t KP = (int64_t)d.K * d.p;
        ct += (size_t)KP;
        tiles += (size_t)cdiv(d.n, 64) * 64 * (size_t)((d.m + 7) & ~7);
        // the smallest candidate gives the most chunks (accum_chunk grows with it)
        const int64_t cmin = accum_chunk(d.m, d.K, d.p, kBatchCchunkCand[0]);
        pobj += (size_t)cdiv(d.n, cmin);  // one objective partial per accumulation chunk
        nsamp += (size_t)d.n;
        part += (size_t)cdiv(d.n, cmin) * (size_t)KP;
    }
    BatchOffsets o;
    size_t off = 0;
    o.sets = off;
    off += al256(ns * sizeof(pds::BatchSet));
    o.gp = off;
    off += al256((ns + 1) * 8);
    o.ap = off;
    off += al256((ns + 1) * 8);
    o.cp = off;
    off += al256((ns + 1) * 8);
    o.up = off;
    off += al256((ns + 1) * 8);
    o.tp = off;
    off += al256((ns + 1) * 8);
    o.ct = off;
    off += al256(ct * 4);
    o.cmax = off;
    off += al256(2 * ns * 4);
    o.vmax = off;
    off += al256(ns * 4);
    o.pobj = off;
    off += al256((pobj > 0 ? pobj : 1) * 8);
    o.psum = off;
    off += al256((part > 0 ? part : 1) * 8);
    o.pcnt = off;
    off += al256((part > 0 ? part : 1) * 4);
    o.vt = off;
    off += al256((tiles > 0 ? tiles : 1) * 4);
    o.it = off;
    off += al256((tiles > 0 ? tiles : 1) * 2);
    o.dist = off;
    off += al256((nsamp > 0 ? nsamp : 1) * 8);
    o.rlist = off;
    off += al256((nsamp > 0 ? nsamp : 1) * 8);
    o.rcount = off;
    off += 256;
    o.total = off;
    return o;
}

// Host image of the tables for a tuning; device pointers relative to ws.
void batch_build(const pds_batch_s& b, const pds::BatchTuning& tu, unsigned char* ws, std::vector<unsigned char>& img,
                 pds::BatchTables& t)
{
    const BatchOffsets o = batch_offsets(b);
    const int ns = (int)b.descs.size();
    img.assign(o.ct, 0);  // sets and prefix tables only
    pds::BatchSet* sets = reinterpret_cast<pds::BatchSet*>(img.data() + o.sets);
    int64_t* gp = reinterpret_cast<int64_t*>(img.data() + o.gp);
    int64_t* ap = reinterpret_cast<int64_t*>(img.data() + o.ap);
    int64_t* cp = reinterpret_cast<int64_t*>(img.data() + o.cp);
    int64_t* up = reinterpret_cast<int64_t*>(img.data() + o.up);
    int64_t* tp = reinterpret_cast<int64_t*>(img.data() + o.tp);
    int64_t g = 0, a = 0, c = 0, u = 0, ct = 0, part = 0, tl = 0, telem = 0, dsum = 0, pch = 0;
    for (int i = 0; i < ns; ++i) {
        const pds_batch_desc& d = b.descs[i];
        pds::BatchSet& S = sets[i];
        S.X = d.X;
        S.vals = d.vals;
        S.idx = d.idx;
        S.c_a = d.centers;
        S.c_b = d.centers_alt;
        S.assign = d.assign;
        S.objective = d.objective;
        S.n = d.n;
        S.ldx = d.ldx;
        S.p = d.p;
        S.m = d.m;
        S.K = d.K;
        int L = 0;
        while ((1 << L) < d.p) ++L;
        S.L = L;
        S.seed = d.seed;
        const int64_t KP = (int64_t)d.K * d.p;
        S.aitem0 = a;
        S.naitems = cdiv(d.n, pds::kBatchAssignSamples);
        S.ct_off = ct;
        S.part_off = part;
        S.cchunk = accum_chunk(d.m, d.K, d.p, tu.cchunk);
        S.nacc = cdiv(d.n, S.cchunk);
        S.kg = accum_kg(d.K, d.p);
        S.ngk = (int)cdiv(d.K, S.kg);
        S.ntiles = cdiv(d.n, 64);
        S.tile_off = telem;
        S.dist_off = dsum;
        dsum += d.n;
        S.pchunk0 = pch;
        pch += S.nacc;
        tp[i] = tl;
        tl += S.ntiles;
        telem += S.ntiles * 64 * (int64_t)((d.m + 7) & ~7);
        gp[i] = g;
        ap[i] = a;
        cp[i] = c;
        up[i] = u;
        g += cdiv(d.n, tu.spw);
        a += S.naitems;
        c += S.nacc * S.ngk;
        u += cdiv(KP, 256);
        ct += KP;
        part += S.nacc * KP;
    }
    gp[ns] = g;
    tp[ns] = tl;
    ap[ns] = a;
    cp[ns] = c;
    up[ns] = u;
    t.gprefix = reinterpret_cast<const int64_t*>(ws + o.gp);
    t.aprefix = reinterpret_cast<const int64_t*>(ws + o.ap);
    t.cprefix = reinterpret_cast<const int64_t*>(ws + o.cp);
    t.uprefix = reinterpret_cast<const int64_t*>(ws + o.up);
    t.ngroups = g;
    t.naitems = a;
    t.ncitems = c;
    t.nuitems = u;
    t.ct = reinterpret_cast<float*>(ws + o.ct);
    t.cmax = reinterpret_cast<uint32_t*>(ws + o.cmax);
    t.pobj = reinterpret_cast<double*>(ws + o.pobj);
    t.psum = reinterpret_cast<int64_t*>(ws + o.psum);
    t.vmax = reinterpret_cast<uint32_t*>(ws + o.vmax);
    t.pcnt = reinterpret_cast<uint32_t*>(ws + o.pcnt);
    t.tprefix = reinterpret_cast<const int64_t*>(ws + o.tp);
    t.ntiles = tl;
    t.vt = reinterpret_cast<float*>(ws + o.vt);
    t.it = reinterpret_cast<uint16_t*>(ws + o.it);
    t.dist = reinterpret_cast<double*>(ws + o.dist);
    t.rlist = reinterpret_cast<int64_t*>(ws + o.rlist);
    t.rcount = reinterpret_cast<uint32_t*>(ws + o.rcount);
    t.recheck_grid = (int64_t)b.tune.update_grid;
}

const pds::BatchSet* batch_sets(const pds_batch_s& b) { return reinterpret_cast<const pds::BatchSet*>(b.ws); }

void batch_set_grids(pds_batch_s& b, const pds::DeviceInfo& dev)
{
    b.tune.compress_grid = (int64_t)dev.cus * pds::batch_compress_occupancy(b.tune.spw, b.pmax);
    b.tune.assign_grid = (int64_t)dev.cus * 2;
    b.tune.accum_grid = (int64_t)dev.cus * 2;
    b.tune.update_grid = (int64_t)dev.cus * 8;
}

hipError_t batch_upload(pds_batch_s& b, hipStream_t s)
{
    batch_build(b, b.tune, b.ws, b.host_tables, b.tables);
    return hipMemcpyAsync(b.ws, b.host_tables.data(), b.host_tables.size(), hipMemcpyHostToDevice, s);
}

void batch_drop_graph(pds_batch_s& b)
{
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
}

// the T rounds (and their prep) on stream s
hipError_t batch_enqueue_rounds(pds_batch_s& b, hipStream_t s, int T)
{
    const int ns = (int)b.descs.size();
    const pds::BatchSet* sets = batch_sets(b);
    hipError_t e = pds::launch_batch_round_prep(sets, ns, b.tables, (T & 1) ? 1 : 0, s);
    if (e == hipSuccess) e = pds::launch_batch_tile(sets, ns, b.tables, b.tune.update_grid, s);
    for (int r = 0; r < T && e == hipSuccess; ++r)
        e = pds::launch_batch_round(sets, ns, b.tables, b.tune, (T - 1 - r) & 1, r, s);
    return e;
}

hipError_t batch_capture(pds_batch_s& b)
{
    batch_drop_graph(b);
    if (b.T == 0) return hipSuccess;
    if (!b.cap) {
        hipError_t e = hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = batch_enqueue_rounds(b, b.cap, b.T);
    e = hipStreamEndCapture(b.cap, &b.graph);
    if (le != hipSuccess) return le;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0);
    size_t nodes = 0;
    if (e == hipSuccess) e = hipGraphGetNodes(b.graph, nullptr, &nodes);
    b.kernels_per_kmeans = (int)nodes;
    return e;
}

pds_status check_batch(pds_batch b, bool bound)
{
    if (!b) return fail(PDS_E_ARG, "batch is NULL");
    if (bound && !b->ws) return fail(PDS_E_ARG, "batch has no workspace bound (pds_batch_bind)");
    return PDS_OK;
}

}  // namespace

pds_status pds_batch_create(pds_batch* out, const pds_batch_desc* descs, int32_t count, int32_t T)
{
    if (!out) return fail(PDS_E_ARG, "out is NULL");
    *out = nullptr;
    if (!descs || count < 1) return fail(PDS_E_ARG, "need count >= 1 descriptors");
    if (T < 0 || T > 100000) return fail(PDS_E_ARG, "T = %d: must be in [0, 100000]", (int)T);
    int pmax = 128;
    for (int i = 0; i < count; ++i) {
        const pds_batch_desc& d = descs[i];
        if (d.p < 128 || d.p > 2048 || !is_pow2(d.p))
            return fail(PDS_E_UNSUPPORTED, "set %d: p = %d must be a power of two in [128, 2048]", i, (int)d.p);
        if (d.m < 1 || d.m > d.p) return fail(PDS_E_M, "set %d: m = %d must satisfy 1 <= m <= p", i, (int)d.m);
        if (d.K < 1 || d.K > 1024) return fail(PDS_E_ARG, "set %d: K = %d must be in [1, 1024]", i, (int)d.K);
        if (d.n < 0 || d.n > ((int64_t)1 << 40)) return fail(PDS_E_ARG, "set %d: n out of range", i);
        if (d.reserved != 0) return fail(PDS_E_ARG, "set %d: reserved must be 0", i);
        if (d.ldx < d.p) return fail(PDS_E_ARG, "set %d: ldx < p", i);
        if (!d.centers || !d.centers_alt || d.centers == d.centers_alt)
            return fail(PDS_E_ARG, "set %d: centers and centers_alt must be distinct non-NULL buffers", i);
        if (T > 0 && !d.objective) return fail(PDS_E_ARG, "set %d: objective is NULL", i);
        if (d.n > 0) {
            if (!d.X || !d.vals || !d.idx || !d.assign)
                return fail(PDS_E_ARG, "set %d: X, vals, idx and assign must be non-NULL", i);
            if (d.p >= 256 && (((uintptr_t)d.X) % 16 != 0 || (d.ldx * 4) % 16 != 0))
                return fail(PDS_E_ARG, "set %d: rows must be 16-byte aligned for p >= 256", i);
        }
        if (d.p > pmax) pmax = d.p;
    }
    pds_batch b = new (std::nothrow) pds_batch_s;
    if (!b) return fail(PDS_E_ARG, "out of host memory");
    b->descs.assign(descs, descs + count);
    b->T = T;
    b->pmax = pmax;
    b->tune.spw = 64;
    b->tune.cchunk = 16384;
    b->ws_bytes = batch_offsets(*b).total;
    *out = b;
    return PDS_OK;
}

pds_status pds_batch_destroy(pds_batch b)
{
    if (!b) return PDS_OK;
    batch_drop_graph(*b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return PDS_OK;
}

pds_status pds_batch_workspace_size(pds_batch b, size_t* bytes)
{
    if (pds_status st = check_batch(b, false)) return st;
    if (!bytes) return fail(PDS_E_ARG, "bytes is NULL");
    *bytes = b->ws_bytes;
    return PDS_OK;
}

pds_status pds_batch_bind(pds_batch b, void* ws, size_t ws_bytes, void* stream)
{
    if (pds_status st = check_batch(b, false)) return st;
    if (!ws || ws_bytes < b->ws_bytes)
        return fail(PDS_E_WORKSPACE, "batch needs %zu workspace bytes, got %zu", b->ws_bytes, ws ? ws_bytes : (size_t)0);
    if (((uintptr_t)ws) % 256 != 0) return fail(PDS_E_ARG, "workspace must be 256-byte aligned");
    pds::DeviceInfo dev;
    hipError_t e = pds::device_info(dev);
    if (e != hipSuccess) return hip_fail(e, "pds_batch_bind");
    e = pds::batch_init_attributes();
    if (e != hipSuccess) return hip_fail(e, "pds_batch_bind");
    b->ws = reinterpret_cast<unsigned char*>(ws);
    batch_set_grids(*b, dev);
    e = batch_upload(*b, reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = batch_capture(*b);
    if (e != hipSuccess) {
        b->ws = nullptr;
        return hip_fail(e, "pds_batch_bind");
    }
    return PDS_OK;
}

pds_status pds_batch_compress(pds_batch b, void* stream)
{
    if (pds_status st = check_batch(b, true)) return st;
    hipError_t e = pds::launch_batch_compress(batch_sets(*b), (int)b->descs.size(), b->tables.gprefix,
                                              b->tables.ngroups, b->tune.spw, b->pmax, b->tune.compress_grid,
                                              reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "pds_batch_compress");
    return PDS_OK;
}

pds_status pds_batch_init_centers(pds_batch b, void* stream)
{
    if (pds_status st = check_batch(b, true)) return st;
    hipError_t e = pds::launch_batch_init(batch_sets(*b), (int)b->descs.size(), b->tables.uprefix, b->tables.nuitems,
                                          b->tune.update_grid, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "pds_batch_init_centers");
    return PDS_OK;
}

pds_status pds_batch_kmeans(pds_batch b, void* stream)
{
    if (pds_status st = check_batch(b, true)) return st;
    if (b->T == 0) return PDS_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e;
    {
        pds::ProfScope ps_("batch_kmeans_graph", s);
        e = hipGraphLaunch(b->exec, s);
    }
    if (e != hipSuccess) return hip_fail(e, "pds_batch_kmeans");
    return PDS_OK;
}

pds_status pds_batch_autotune(pds_batch b, void* stream)
{
    if (pds_status st = check_batch(b, true)) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    pds::DeviceInfo dev;
    hipError_t e = pds::device_info(dev);
    if (e != hipSuccess) return hip_fail(e, "pds_batch_autotune");
    hipEvent_t t0, t1;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
        return fail(PDS_E_HIP, "pds_batch_autotune: event creation failed");
    auto timed = [&](auto&& work, float& ms) -> hipError_t {
        hipError_t r = work();  // warm-up
        if (r == hipSuccess) r = hipEventRecord(t0, s);
        for (int rep = 0; rep < 3 && r == hipSuccess; ++rep) r = work();
        if (r == hipSuccess) r = hipEventRecord(t1, s);
        if (r == hipSuccess) r = hipEventSynchronize(t1);
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, t0, t1);
        return r;
    };
    const int ns = (int)b->descs.size();
    // compression: samples per group
    float best = 1e30f;
    int best_spw = b->tune.spw;
    for (int spw : kBatchSpwCand) {
        if (e != hipSuccess) break;
        b->tune.spw = spw;
        batch_set_grids(*b, dev);
        e = batch_upload(*b, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        float ms = 0.0f;
        if (e == hipSuccess)
            e = timed([&]() {
                return pds::launch_batch_compress(batch_sets(*b), ns, b->tables.gprefix, b->tables.ngroups, spw,
                                                  b->pmax, b->tune.compress_grid, s);
            }, ms);
        if (e == hipSuccess && ms < best) {
            best = ms;
            best_spw = spw;
        }
    }
    b->tune.spw = best_spw;
    // K-means round: accumulation chunk length
    best = 1e30f;
    int best_c = b->tune.cchunk;
    {
        for (int cc : kBatchCchunkCand) {
            if (e != hipSuccess || b->T == 0) break;
            b->tune.cchunk = cc;
            batch_set_grids(*b, dev);
            e = batch_upload(*b, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e == hipSuccess) e = pds::launch_batch_round_prep(batch_sets(*b), ns, b->tables, 0, s);
            if (e == hipSuccess) e = pds::launch_batch_tile(batch_sets(*b), ns, b->tables, b->tune.update_grid, s);
            float ms = 0.0f;
            if (e == hipSuccess)
                e = timed([&]() { return pds::launch_batch_round(batch_sets(*b), ns, b->tables, b->tune, 1, 0, s); }, ms);
            if (e == hipSuccess && ms < best) {
                best = ms;
                best_c = cc;
            }
        }
    }
    b->tune.cchunk = best_c;
    batch_set_grids(*b, dev);
    if (e == hipSuccess) e = batch_upload(*b, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = batch_capture(*b);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (e != hipSuccess) return hip_fail(e, "pds_batch_autotune");
    return PDS_OK;
}

pds_status pds_batch_info(pds_batch b, char* buf, size_t len)
{
    if (pds_status st = check_batch(b, false)) return st;
    if (!buf || len == 0) return fail(PDS_E_ARG, "buf is NULL");
    int64_t n = 0;
    for (const auto& d : b->descs) n += d.n;
    snprintf(buf, len,
             "sets=%d samples=%lld T=%d spw=%d cchunk=%d groups=%lld assign_items=%lld accum_items=%lld "
             "update_items=%lld compress_grid=%lld graph_kernels=%d ws_bytes=%zu",
             (int)b->descs.size(), (long long)n, b->T, b->tune.spw, b->tune.cchunk,
             (long long)b->tables.ngroups, (long long)b->tables.naitems, (long long)b->tables.ncitems,
             (long long)b->tables.nuitems, (long long)b->tune.compress_grid, b->kernels_per_kmeans, b->ws_bytes);
    return PDS_OK;
}

pds_status pds_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(pds::g_prof_mu);
    if (on) {
        for (auto& r : pds::g_prof) {
            (void)hipEventDestroy(r.start);
            (void)hipEventDestroy(r.stop);
        }
        pds::g_prof.clear();
    }
    pds::g_prof_on = on != 0;
    return PDS_OK;
}

pds_status pds_profile_report(char* buf, size_t len, size_t* needed)
{
    if (!buf && len > 0) return fail(PDS_E_ARG, "buf is NULL");
    struct Agg {
        int count = 0;
        double total = 0, mn = 1e300, mx = 0;
    };
    std::map<std::string, Agg> agg;
    std::vector<std::string> order;
    pds_status st = PDS_OK;
    {
        std::lock_guard<std::mutex> lk(pds::g_prof_mu);
        for (auto& r : pds::g_prof) {
            float ms = 0.0f;
            hipError_t e = hipEventSynchronize(r.stop);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
            if (e != hipSuccess) st = hip_fail(e, "pds_profile_report");
            if (!agg.count(r.name)) order.push_back(r.name);
            Agg& a = agg[r.name];
            a.count += 1;
            a.total += ms;
            a.mn = ms < a.mn ? ms : a.mn;
            a.mx = ms > a.mx ? ms : a.mx;
            (void)hipEventDestroy(r.start);
            (void)hipEventDestroy(r.stop);
        }
        pds::g_prof.clear();
    }
    std::string out;
    char line[256];
    for (auto& nm : order) {
        const Agg& a = agg[nm];
        snprintf(line, sizeof(line), "%s %d %.6f %.6f %.6f\n", nm.c_str(), a.count, a.total, a.mn, a.mx);
        out += line;
    }
    if (needed) *needed = out.size() + 1;
    if (len > 0) {
        size_t c = out.size() < len - 1 ? out.size() : len - 1;
        memcpy(buf, out.data(), c);
        buf[c] = 0;
    }
    return st;
}

const char* pds_last_error(void) { return g_err; }

const char* pds_version(void) { return "pds 0.1.0 (gfx950)"; }

}  // extern "C"
