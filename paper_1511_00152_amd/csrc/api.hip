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
#include <vector>

#include "../../include/pds.h"
#include "pds_device.hpp"
#include "pds_internal.hpp"

struct pds_plan_s {
    int64_t p;
    int64_t m;
    uint64_t seed;
    int32_t prec;
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
    *out = pl;
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

pds_status pds_workspace_size(pds_plan plan, int32_t op, int64_t n, int32_t K, size_t* bytes)
{
    if (pds_status st = check_plan(plan)) return st;
    if (!bytes) return fail(PDS_E_ARG, "bytes is NULL");
    if (n < 0) return fail(PDS_E_ARG, "n < 0");
    pds::DeviceInfo dev = query_dev_or_default();
    const int p = (int)plan->p, m = (int)plan->m;
    switch (op) {
        case PDS_OP_COMPRESS:
            *bytes = pds::compress_workspace(plan->prec, p, n, dev);
            return PDS_OK;
        case PDS_OP_COVARIANCE:
            *bytes = pds::covariance_workspace(plan->prec, p, m, n, dev);
            return PDS_OK;
        case PDS_OP_KMEANS:
            if (K < 1 || K > 1024) return fail(PDS_E_ARG, "K = %d: must be in [1, 1024]", (int)K);
            *bytes = pds::kmeans_workspace(plan->prec, p, m, n, K, dev);
            return PDS_OK;
        default:
            return fail(PDS_E_ARG, "unknown op %d", (int)op);
    }
}

pds_status pds_covariance_acc_size(pds_plan plan, size_t* bytes)
{
    if (pds_status st = check_plan(plan)) return st;
    if (!bytes) return fail(PDS_E_ARG, "bytes is NULL");
    *bytes = (size_t)plan->p * (size_t)plan->p * sizeof(double);
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
    const size_t need = pds::compress_workspace(plan->prec, (int)plan->p, n, dev);
    if (need > 0 && (!ws || ws_bytes < need))
        return fail(PDS_E_WORKSPACE, "compress needs %zu workspace bytes, got %zu", need, ws ? ws_bytes : (size_t)0);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    e = pds::launch_sample_indices(plan->seed, (int)plan->p, (int)plan->m, n, i0, idx, dev, s);
    if (e != hipSuccess) return hip_fail(e, "sample_indices");
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
    const size_t need = pds::covariance_workspace(plan->prec, (int)plan->p, (int)plan->m, n, dev);
    if (need > 0 && (!ws || ws_bytes < need))
        return fail(PDS_E_WORKSPACE, "covariance needs %zu workspace bytes, got %zu", need, ws ? ws_bytes : (size_t)0);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (n > 0) {
        e = pds::launch_covariance_accumulate(plan->prec, (int)plan->p, (int)plan->m, vals, idx, n, acc, ws, ws_bytes,
                                              dev, s);
        if (e != hipSuccess) return hip_fail(e, "covariance accumulate");
    }
    if (finalize) {
        e = pds::launch_covariance_finalize(plan->prec, (int)plan->p, (int)plan->m, n_total, acc, C_out, s);
        if (e != hipSuccess) return hip_fail(e, "covariance finalize");
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

pds_status pds_unmix(pds_plan plan, const double* centers_pre, int32_t K, double* centers_out, void* stream)
{
    if (pds_status st = check_plan(plan)) return st;
    if (K < 1) return fail(PDS_E_ARG, "K < 1");
    if (!centers_pre || !centers_out) return fail(PDS_E_ARG, "centers must be non-NULL");
    if (centers_pre == centers_out) return fail(PDS_E_ARG, "centers_pre and centers_out must not alias");
    hipError_t e = pds::launch_unmix(plan->seed, (int)plan->p, centers_pre, K, centers_out,
                                     reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "unmix");
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
