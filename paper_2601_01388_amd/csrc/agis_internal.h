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
    agis::Partial* d_partials = nullptr;
    size_t partials_cap = 0;
    void* d_scratch = nullptr;
    size_t scratch_bytes = 0;
    void* d_small = nullptr;  // 4 KiB of flags / reduction cells
    uint64_t* d_blocksums = nullptr;
    size_t blocksums_cap = 0;
    double* d_xout = nullptr;  // per-sample weights of the current round
    uint64_t xout_cap = 0;
    agis::DevPlan* d_plans = nullptr;    // kMaxSegs plans
    agis::LaunchDesc* d_launch = nullptr;  // the current round
    int sample_blocks_per_cu[6] = {0, 0, 0, 0, 0, 0};  // resident blocks per CU of each kernel (variant, pairs)
    int lanes_blocks_per_cu = 0;                       // the same for the lane sampler
    // launch tuning (0 = default): resident blocks per CU, slots per grab
    int tune_blocks_per_cu = 0;
    uint32_t tune_grab = 0;
    int use_graphs = 1;
    int tune_variant = 0;  // sampling-kernel register budget (see sample_kernel)
    uint32_t tune_hub_window = 0;  // see LaunchDesc::hub_window
    // captured round (k_zero, k_sample, k_reduce_x) replayed on graph_stream;
    // valid while the key below matches
    hipStream_t graph_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    uint64_t graph_key[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    hipEvent_t ev_in = nullptr;
    hipEvent_t ev_out = nullptr;
    hipEvent_t ev_start = nullptr;  // brackets each sampling launch
    hipEvent_t ev_stop = nullptr;
    // device address of this device's fixed workspace (agis_estimate_noalloc)
    void* noalloc_scratch = nullptr;
    // buffers of runs to epsilon in one launch (pattern states, rings, tiles)
    void* d_eps = nullptr;
    size_t eps_bytes = 0;
    // pinned, device-mapped host flag: the cancel request of a run to
    // epsilon in one launch, read by the kernel while it runs
    volatile uint32_t* h_cancel = nullptr;
    const volatile uint32_t* d_cancel = nullptr;
    int wall_clock_khz = 100000;
};

struct agis_graph {
    agis_ctx* ctx = nullptr;
    agis::DevGraph g{};
    uint32_t max_deg = 0;
    // a degree-oriented graph (agis_orient) owns its CSR and keeps the
    // undirected graph it came from (adjacency tests of its tables)
    const agis_graph* parent = nullptr;
    uint64_t* own_off = nullptr;
    uint32_t* own_nbr = nullptr;
};

struct TableCache;  // proposal tables of f_approx kept across calls (csrc/api.hip)

struct agis_tables {
    agis_ctx* ctx = nullptr;
    TableCache* cache = nullptr;
    const agis_graph* graph = nullptr;
    uint4* rec = nullptr;      // {deg, LA, LC, 0}
    uint64_t* s2 = nullptr;
    uint64_t* hits = nullptr;
    uint64_t* trials = nullptr;
    // hub neighbourhood bitmaps (see DevTables)
    uint32_t* hub_bits = nullptr;
    int32_t* hub_slot = nullptr;
    uint64_t hub_words = 0;
    uint64_t hubs = 0;
    uint32_t hub_min_degree = 0;
    // common-neighbour counts of the pair hubs (see DevTables)
    int32_t* pair_slot = nullptr;
    uint32_t* pair_count = nullptr;
    uint32_t* pair_quart = nullptr;
    uint64_t pairs = 0;
    uint32_t pair_min_degree = 0;
    // common-neighbour lists of the core pairs (see DevTables)
    int32_t* core_slot = nullptr;
    uint64_t* core_start = nullptr;
    uint32_t* core_len = nullptr;
    uint32_t* core_nbr = nullptr;
    uint64_t cores = 0;
    uint64_t core_entries = 0;  // entries of core_nbr (lists padded to kCoreBlock)
};

namespace agis {

int compile_plan(const agis_pattern* p, const uint8_t* order, int mode, int beta_num, int beta_den,
                 agis_plan* out, std::string* err);

// Every connected graph on k vertices up to isomorphism (see
// agis_connected_patterns).
int connected_patterns(uint32_t k, agis_pattern* out, uint32_t cap, uint32_t* count, std::string* err);

// Edge-induced and vertex-induced concentrations from copy counts of every
// connected k-pattern (see agis_concentrations).
int concentrations(uint32_t n, const agis_pattern* patterns, const double* copies, double* conc_edge, double* induced,
                   double* conc_induced, std::string* err);

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
// adj: the graph whose lists decide whether two neighbours are adjacent (g
// itself, or the undirected graph of an oriented g)
hipError_t launch_build_tables(const DevGraph& g, const DevGraph& adj, uint4* rec, uint64_t* s2, uint64_t* hits,
                               uint64_t* trials, uint32_t k0, uint32_t k1, int32_t lc_min, int exact,
                               hipStream_t stream);
// Hub bitmaps: log2-degree histogram (64 buckets) of g; then, for vertices
// of degree >= min_deg, their slots (hub_slot, -1 elsewhere; flags is n
// entries of scratch), the count into *hubs; then the bits.
hipError_t launch_degree_histogram(const DevGraph& g, uint32_t* hist, hipStream_t stream);
hipError_t launch_hub_slots(agis_ctx* ctx, const DevGraph& g, uint32_t min_deg, uint32_t* flags, int32_t* hub_slot,
                            uint64_t* d_count);
// pair_count[a * H + b] = |N(u_a) cap N(u_b)| for the H vertices with
// pair_slot >= 0 (all of them hubs with bitmaps); the diagonal is 0.
// pair_quart[(a * H + b) * (kPairParts - 1) + j - 1] = common neighbours
// before position j d / kPairParts of the walked list (the shorter of the
// two by (degree, id)).
hipError_t launch_pair_counts(agis_ctx* ctx, const DevGraph& g, const int32_t* hub_slot, const uint32_t* hub_bits,
                              uint64_t hub_words, const int32_t* pair_slot, uint64_t H, uint32_t* pair_hub,
                              uint32_t* pair_count, uint32_t* pair_quart);
hipError_t launch_hub_bits(const DevGraph& g, const int32_t* hub_slot, uint64_t words, uint32_t* bits,
                           hipStream_t stream);
// Degree orientation: out-degrees into outdeg (n entries of scratch), the
// offsets into off_out (n + 1), then the neighbours into nbr_out.
hipError_t launch_orient_offsets(agis_ctx* ctx, const DevGraph& g, uint32_t* outdeg, uint64_t* off_out);
hipError_t launch_orient_fill(const DevGraph& g, const uint64_t* off_out, uint32_t* nbr_out, hipStream_t stream);
// out[v] = certain-zero marker if d(v) < b + f1, else lt[v] (lt given) or the
// f_approx log weight of signature (b, f1, ie, f2).
hipError_t launch_step_log_weights(const agis_tables& t, uint64_t n, uint32_t b, uint32_t f1, uint32_t ie, uint32_t f2,
                                   const int32_t* lt, int32_t* out, hipStream_t stream);
hipError_t launch_export_tables(const agis_tables& t, uint64_t n, uint32_t* deg, int32_t* la, int32_t* lc,
                                hipStream_t stream);

// A bump allocator over a fixed device buffer, for calls that allocate
// nothing: take() returns the next `bytes` (aligned to 256) or nullptr when
// they do not fit.
struct Arena {
    char* base = nullptr;
    uint64_t cap = 0;
    uint64_t used = 0;
    void* take(uint64_t bytes) {
        const uint64_t at = (used + 255) / 256 * 256;
        if (at > cap || bytes > cap - at) return nullptr;
        used = at + bytes;
        return base + at;
    }
    uint64_t left() const {
        const uint64_t at = (used + 255) / 256 * 256;
        return at < cap ? cap - at : 0;
    }
};

// Tile sums of the first-step scan (one per kScanTile vertices).
uint64_t step1_scan_tiles(uint64_t n);

// First-step table for step 0 of the plan `hp`: q1, inclusive prefix pre,
// total copied into *total (synchronises the stream).  blocksums: device
// uint64[step1_scan_tiles(n)] of scratch, or nullptr for the context's own.
hipError_t build_step1(agis_ctx* ctx, const agis_graph& g, const agis_tables& t, const DevPlan& hp,
                       uint32_t* q1, uint64_t* pre, uint64_t* total, uint64_t* blocksums = nullptr);

// Blocked first-step table for step 0 of `hp`: blk (device uint64[nblk + 1],
// nblk = ceil(n / kStep1Block)) receives 0 and then the inclusive prefix of
// the blocks' weight sums (so blk + 1 is the table and blk[0] its "before
// block 0"); *lmax_out the largest log weight, *total the sum (synchronises
// the stream).
hipError_t build_step1_blocks(agis_ctx* ctx, const agis_graph& g, const agis_tables& t, const DevPlan& hp,
                              uint64_t* blk, int32_t* lmax_out, uint64_t* total);

// Guide of an inclusive prefix pre[0..n) with total = pre[n - 1] > 0:
// guide[b] = first v with pre[v] > b << shift for b < buckets =
// ((total - 1) >> shift) + 1 <= 2^kGuideBits, guide[buckets] = n - 1.
constexpr uint32_t kGuideBits = 16;
uint32_t guide_shift(uint64_t total);
hipError_t launch_prefix_guide(const uint64_t* pre, uint64_t n, uint64_t total, uint32_t shift, uint32_t* guide,
                               hipStream_t stream);

// a[0 .. n) = v (a kernel, so that a captured sequence holds no memset).
hipError_t launch_fill_u32(uint32_t* a, uint64_t n, uint32_t v, hipStream_t stream);

// Per-row pick table (per CSR slot, the inclusive u64 prefix of the integer
// weights within the slot's row) of a weighted step with one backward vertex
// whose per-vertex log weights (launch_step_log_weights) are sw.
// lists: 2 n + 2 uint32 of scratch (the lists of longer rows and their lengths).
hipError_t launch_rowtab(agis_ctx* ctx, const DevGraph& g, const int32_t* sw, uint64_t* pre, uint32_t* lists);

struct SampleLaunch {
    int blocks = 0;
    int threads = 256;
    uint64_t cap = 0;        // scratch entries per wave
    uint32_t grab = 1;       // sample slots a wave takes per queue access
    uint64_t max_slots = 0;  // largest round
    uint64_t max_tiles = 0;  // reduction tiles of the largest round
    bool dump = false;       // launch the record-writing variant
    bool meter = false;      // launch the request-metering variant (needs idx)
    int variant = 0;         // register-budget variant
    uint32_t hub_window = 0; // see LaunchDesc::hub_window
    // the kernel with the pair-hub paths (set by the caller before
    // plan_sample_launch: some plan has an unweighted step over exactly two
    // backward lists and the tables hold the pair-hub table)
    bool pairs = false;
    // the lane sampler (one sample per lane; set by the caller before
    // plan_sample_launch when every plan of the launch is a lane plan)
    bool lanes = false;
    // buffers of the launch (set by plan_sample_launch): the waves' scratch,
    // the per-slot weights and the reduction tiles
    void* scratch = nullptr;
    double* xout = nullptr;
    Partial* partials = nullptr;
};

// The sampling kernel for (record-writing?, register-budget variant 0..2,
// pair-hub paths?).
const void* sample_kernel(bool dump, int variant, bool pairs, bool meter);
// Degrees of the pair hubs (deg[i] of pair_hub[i]).
hipError_t launch_pair_hub_degrees(agis_ctx* ctx, const DevGraph& g, const uint32_t* pair_hub, uint64_t H,
                                   uint32_t* deg);
// Core-pair lists: core_slot[core_vertex[c]] = c, and for every pair a < b
// of core slots the common neighbours of the two vertices, ascending, at
// core_nbr + core_start[a * C + b] (walking the shorter list and probing the
// other's hub bitmap).
hipError_t launch_core_pairs(agis_ctx* ctx, const DevGraph& g, const int32_t* hub_slot, const uint32_t* hub_bits,
                             uint64_t hub_words, const uint32_t* core_vertex, uint64_t C, int32_t* core_slot,
                             const uint64_t* core_start, const uint32_t* core_len, uint32_t* core_nbr);

// The pick table of one step signature (per-vertex log weights sw, certain
// zeros folded in) over the core-pair lists: clm[pair] (indexed like
// core_len), cbp[entry / kCoreBlock].
hipError_t launch_core_pick(agis_ctx* ctx, const agis_tables& t, const int32_t* sw, int32_t* clm, uint64_t* cbp);

// The lane sampler for (record-writing?, metering?).
const void* sample_lanes_kernel(bool dump, bool meter);
// Whether the lane sampler serves a plan: every step after the first is a
// uniform draw from the row of one backward vertex, and a weighted first
// step is held in the full table (not blocked).
bool lane_plan(const DevPlan& hp);
// The persistent run-to-epsilon sampler for (register-budget variant, pair-hub paths?).
const void* sample_eps_kernel(int variant, bool pairs);

// Sizes the persistent grid (resident waves only) and the buffers for
// rounds of at most max_slots samples over at most max_segs segments.  With
// an arena the buffers are taken from it (no allocation; the grid shrinks to
// the waves whose scratch fits, AGIS_E_UNSUPPORTED below one workgroup),
// else they are the context's, grown as needed.
int plan_sample_launch(agis_ctx* ctx, const agis_graph& g, uint64_t max_slots, uint32_t max_segs, SampleLaunch* L,
                       std::string* err, Arena* arena = nullptr);

// One round as described by ctx->d_launch (plans in ctx->d_plans): clears
// the work queue (a kernel, so the sequence can be captured in a graph),
// samples every slot into ctx->d_xout (slot weights), reduces each
// segment's weights into tiles of kReduceTileSamples in ctx->d_partials.
// With D.idx the single segment's samples are idx[0..count); with D.dump
// one record per slot.  `before`/`after` (may be null) are recorded
// around the sampling kernel alone.
constexpr uint64_t kReduceTileSamples = 2048;
hipError_t launch_round(agis_ctx* ctx, hipStream_t stream, const SampleLaunch& L, hipEvent_t before,
                        hipEvent_t after);

// Host-side fill of the launch descriptor's buffers and shape (the round
// part is filled by the caller); upload it to ctx->d_launch before a round.
void fill_launch(agis_ctx* ctx, const SampleLaunch& L, const DevGraph& g, const DevTables& t, const uint64_t* idx,
                 Record* dump, LaunchDesc* D, uint64_t* meter = nullptr);

}  // namespace agis
