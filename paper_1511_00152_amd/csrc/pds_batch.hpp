// Batched form: per-set device descriptors, the work tables of the persistent
// launches, and the launch interface used by the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pds {

constexpr int kBatchAssignSamples = 512;           // samples per assignment item (one per thread)
constexpr int kBatchAccumLds = 65536;               // LDS of one accumulation workgroup
constexpr int kBatchAccumEntries = kBatchAccumLds / 12;  // 64-bit fixed-point sum + u32 count per entry

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
    int64_t tile_off;         // first element of the set's 64-sample tiles (vt, it)
    int64_t ntiles;           // ceil(n / 64)
    int64_t dist_off;         // first element of the set's per-sample distances
    int64_t pchunk0;          // first objective partial (one per accumulation chunk)
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
    int64_t* psum;           // fixed-point partial sums (scale 2^F of the set, see batch_fx_exp)
    uint32_t* pcnt;
    uint32_t* vmax;          // nsets: largest |compressed value| of the set (float bits), per K-means call
    const int64_t* tprefix;  // tiles (nsets + 1)
    int64_t ntiles;
    float* vt;               // compressed values tiled by 64 samples: [tile][entry][lane]
    uint16_t* it;            // kept coordinates, same tiling
    double* dist;            // distance of each sample to its center (FP32 value, FP64 after a recheck)
    int64_t* rlist;          // samples to recheck in FP64: set << 40 | sample
    uint32_t* rcount;        // number of entries in rlist
    int64_t recheck_grid;
};

struct BatchTuning {
    int spw;     // samples per compression group
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
hipError_t launch_batch_round_prep(const BatchSet* sets, int nsets, const BatchTables& t, int copy_to_b,
                                   hipStream_t s);
// row-major compressed data -> 64-sample tiles (once per K-means call)
hipError_t launch_batch_tile(const BatchSet* sets, int nsets, const BatchTables& t, int64_t grid, hipStream_t s);
// dir = 1: round reads c_a, writes c_b; dir = 0: reads c_b, writes c_a
hipError_t launch_batch_round(const BatchSet* sets, int nsets, const BatchTables& t, const BatchTuning& tu, int dir,
                              int round, hipStream_t s);

}  // namespace pds
