// Internal interfaces between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "agis.h"
#include "agis_common.h"

struct agis_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int num_cus = 256;
    // reusable device buffers
    agis::DevPlan* d_plan = nullptr;
    agis::Partial* d_partials = nullptr;
    size_t partials_cap = 0;
    void* d_scratch = nullptr;
    size_t scratch_bytes = 0;
    void* d_small = nullptr;  // 4 KiB of flags / reduction cells
    uint64_t* d_blocksums = nullptr;
    size_t blocksums_cap = 0;
    double* d_xout = nullptr;  // per-sample weights of the current launch
    uint64_t xout_cap = 0;
    int sample_blocks_per_cu = 0;
    hipEvent_t ev_start = nullptr;  // brackets each sampling launch
    hipEvent_t ev_stop = nullptr;
};

struct agis_graph {
    agis_ctx* ctx = nullptr;
    agis::DevGraph g{};
    uint32_t max_deg = 0;
};

struct agis_tables {
    agis_ctx* ctx = nullptr;
    const agis_graph* graph = nullptr;
    uint4* rec = nullptr;      // {deg, LA, LC, 0}
    uint64_t* s2 = nullptr;
    uint64_t* hits = nullptr;
    uint64_t* trials = nullptr;
};

namespace agis {

int compile_plan(const agis_pattern* p, const uint8_t* order, int mode, int beta_num, int beta_den,
                 agis_plan* out, std::string* err);

// Host copies of the Q16 tables (generated on first use) and their upload
// into the device constant tables of this library.
const int32_t* host_logtab();
const uint32_t* host_exp2tab();
hipError_t upload_fixed_point_tables(hipStream_t stream);

// Kernels launchers (all asynchronous on `stream`).
// Row checks (offsets monotone and within nnz) must pass before the edge
// checks run: the edge checks index rows through the offsets.
hipError_t launch_validate_rows(const DevGraph& g, uint32_t* d_flags, hipStream_t stream);
hipError_t launch_validate_edges(const DevGraph& g, uint32_t* d_flags, hipStream_t stream);
hipError_t launch_max_degree(const DevGraph& g, uint32_t* d_max, hipStream_t stream);
hipError_t launch_build_tables(const DevGraph& g, uint4* rec, uint64_t* s2, uint64_t* hits, uint64_t* trials,
                               uint32_t k0, uint32_t k1, int32_t lc_min, int exact, hipStream_t stream);
hipError_t launch_export_tables(const agis_tables& t, uint64_t n, uint32_t* deg, int32_t* la, int32_t* lc,
                                hipStream_t stream);

// First-step table for step 0 of `plan` (host copy `hp`): q1, inclusive
// prefix pre, total copied into *total (synchronises the stream).
hipError_t build_step1(agis_ctx* ctx, const agis_graph& g, const agis_tables& t, const DevPlan& hp,
                       uint32_t* q1, uint64_t* pre, uint64_t* total);

// Per-row pick table (one inclusive u64 prefix over all CSR slots, read per row
// relative to the entry before the row) of a weighted
// step with one backward vertex and signature (b, f1, ie, f2) or learned
// log weights lt.
// rowmax: n int32 of scratch for the row maxima.
hipError_t launch_rowtab(agis_ctx* ctx, const DevGraph& g, const uint4* rec, uint32_t b, uint32_t f1, uint32_t ie,
                         uint32_t f2, const int32_t* lt, uint64_t* pre, int32_t* rowmax);

struct SampleLaunch {
    int blocks = 0;
    int threads = 256;
    uint64_t cap = 0;    // scratch entries per wave
    uint32_t grab = 1;   // sample slots a wave takes per queue access
    uint64_t tiles = 0;  // reduction tiles of the weight buffer
};

// Sizes the persistent grid (resident waves only) and the buffers for a
// launch of `count` samples.
SampleLaunch plan_sample_launch(agis_ctx* ctx, const agis_graph& g, uint64_t count, std::string* err, int* rc);

// Samples slots [0, count) (sample index start + slot, or idx[slot]) into
// ctx->d_xout; dump != nullptr also writes one record per slot.
// `before`/`after` (may be null) are recorded around the sampling kernel alone.
hipError_t launch_sample(agis_ctx* ctx, const SampleLaunch& L, const DevGraph& g, const DevTables& t,
                         const Step1& s1, uint32_t k0, uint32_t k1, uint64_t start, uint64_t count,
                         const uint64_t* idx, Record* dump, hipEvent_t before, hipEvent_t after);

// Per-tile (n, mean, M2, nonzero) of ctx->d_xout[0, count) into ctx->d_partials,
// one tile per kReduceTileSamples consecutive weights.
constexpr uint64_t kReduceTileSamples = 2048;
hipError_t launch_reduce(agis_ctx* ctx, const SampleLaunch& L, uint64_t count);

}  // namespace agis
