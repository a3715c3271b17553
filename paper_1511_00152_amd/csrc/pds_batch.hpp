// Batched form: per-set device descriptors, the work tables of the persistent
// launches, and the launch interface used by the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pds {

constexpr int kBatchAccumLds = 65536;               // LDS of one accumulation workgroup
constexpr int kBatchAccumEntries = kBatchAccumLds / 8;  // FP32 sum + u32 count per entry

// One data set as the kernels see it (device copy).
struct BatchSet {
    const float* X;
    float* vals;
    uint16_t* idx;
    double* c_a;  // the caller's centers
    double* c_b;  // the caller's second center buffer
    int32_t* assign;
    double* objective;
    int64_t n, ldx;
    int p, m, K, L;
    uint64_t seed;
    int64_t aitem0, naitems;  // assignment items of the set
    int64_t part_off;         // first element of the set's chunk partials
    int64_t ct_off;           // first element of the set's transposed FP32 centers
    int64_t nacc, cchunk;     // accumulation chunks and their length (samples)
    int ngk, kg;              // cluster groups, clusters per group
};

// Device tables in the workspace (pointers) and their sizes.
struct BatchTables {
    const int64_t* gprefix;  // compression groups, per set, prefix (nsets + 1)
    const int64_t* aprefix;  // assignment items
    const int64_t* cprefix;  // accumulation items
    const int64_t* uprefix;  // update items (256 center entries each)
    int64_t ngroups, naitems, ncitems, nuitems;
    float* ct;
    uint32_t* cmax;  // 2 x nsets (float bits)
    double* pobj;
    float* psum;
    uint32_t* pcnt;
};

struct BatchTuning {
    int spw;     // samples per compression group
    int achunk;  // samples per assignment item
    int cchunk;  // samples per accumulation chunk
    int64_t compress_grid, assign_grid, accum_grid, update_grid;
};

// dynamic-LDS limits of the batch kernels (call once before launching or capturing)
hipError_t batch_init_attributes();
size_t batch_compress_lds(int spw, int pmax);
int batch_compress_occupancy(int spw, int pmax);
hipError_t launch_batch_compress(const BatchSet* sets, int nsets, const int64_t* gprefix, int64_t ngroups, int spw,
                                 int pmax, int64_t grid, hipStream_t s);
hipError_t launch_batch_init(const BatchSet* sets, int nsets, const int64_t* uprefix, int64_t nitems, int64_t grid,
                             hipStream_t s);
hipError_t launch_batch_round_prep(const BatchSet* sets, int nsets, float* ct, uint32_t* cmax0, int copy_to_b,
                                   hipStream_t s);
// dir = 1: round reads c_a, writes c_b; dir = 0: reads c_b, writes c_a
hipError_t launch_batch_round(const BatchSet* sets, int nsets, const BatchTables& t, const BatchTuning& tu, int dir,
                              int round, hipStream_t s);

}  // namespace pds
