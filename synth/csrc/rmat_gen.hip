// R-MAT graph generator on the GPU, for graphs too large for host
// generation or for deduplication by a global sort: input generation only
// (it draws nothing for the estimator and shares no code with it).
//
// Recipe (the recursive-quadrant R-MAT of Chakrabarti, Zhan and Faloutsos,
// SDM 2004, without noise): edge e of n_edges = edge_factor * 2^scale picks,
// at each of `scale` levels, the quadrant (0,0), (0,1), (1,0), (1,1) with
// probabilities a, b, c, 1 - a - b - c from one uniform double r of the
// stream below: the row bit is r >= a + b, the column bit is
// (a <= r < a + b) or r >= a + b + c.  Self-loops are dropped; the graph is
// symmetrised and deduplicated into CSR with ascending rows.
//
// Random stream: counter-based SplitMix64 (Steele, Lea and Flood, OOPSLA
// 2014): draw i of seed s is mix(s + (i + 1) * 0x9E3779B97F4A7C15), and the
// uniform of level l of edge e is draw (e * 32 + l), top 53 bits over 2^53.
// synth/graphs.py holds a numpy twin of the same stream for small scales.
//
// Passes (all in place on caller buffers): count the two endpoint degrees
// of every edge; scatter both directions into their rows at offsets the
// caller derived from the counts; sort each row (hipCUB segmented sort over
// batches of consecutive rows) and keep its distinct values; move the rows
// left onto the offsets of the deduplicated degrees, a batch of rows at a
// time through a staging buffer.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cstdint>
#include <cstring>
#include <vector>

namespace {

__device__ __forceinline__ uint64_t splitmix_draw(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct RmatParams {
    uint64_t n_edges;
    uint64_t seed;
    double a, ab, abc;
    uint32_t scale;
};

__device__ __forceinline__ void rmat_edge(const RmatParams& P, uint64_t e, uint32_t& u, uint32_t& v) {
    uint32_t x = 0, y = 0;
    for (uint32_t l = 0; l < P.scale; ++l) {
        const double r = (double)(splitmix_draw(P.seed, e * 32 + l) >> 11) * 0x1.0p-53;
        x = (x << 1) | (r >= P.ab ? 1u : 0u);
        y = (y << 1) | (((r >= P.a && r < P.ab) || r >= P.abc) ? 1u : 0u);
    }
    u = x;
    v = y;
}

constexpr unsigned kThreads = 256;
constexpr uint64_t kMaxBlocks = 1ull << 20;

unsigned grid(uint64_t items) {
    const uint64_t b = (items + kThreads - 1) / kThreads;
    return (unsigned)(b < kMaxBlocks ? b : kMaxBlocks);
}

__global__ void k_count(RmatParams P, uint32_t* deg) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < P.n_edges; e += stride) {
        uint32_t u, v;
        rmat_edge(P, e, u, v);
        if (u == v) continue;
        atomicAdd(&deg[u], 1u);
        atomicAdd(&deg[v], 1u);
    }
}

__global__ void k_fill(RmatParams P, const uint64_t* off, uint32_t* cursor, uint32_t* nbr) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < P.n_edges; e += stride) {
        uint32_t u, v;
        rmat_edge(P, e, u, v);
        if (u == v) continue;
        nbr[off[u] + atomicAdd(&cursor[u], 1u)] = v;
        nbr[off[v] + atomicAdd(&cursor[v], 1u)] = u;
    }
}

// Batch offsets relative to the batch start, as the segmented sort takes
// them (int: a batch holds fewer than 2^31 slots).
__global__ void k_rel_offsets(const uint64_t* off, uint64_t r0, uint64_t rows, int* rel) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= rows; i += stride)
        rel[i] = (int)(off[r0 + i] - off[r0]);
}

// Distinct values of every sorted row to the row's front; the count into
// newdeg.  One thread per row up to kThreadRow entries; longer rows are
// left to k_dedup_long (one wave each).
constexpr uint64_t kThreadRow = 1024;

__global__ void k_dedup_short(const uint64_t* off, uint32_t* nbr, uint64_t n, uint32_t* newdeg) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        const uint64_t o = off[u], d = off[u + 1] - o;
        if (d > kThreadRow) continue;
        uint32_t* row = nbr + o;
        uint32_t cnt = 0;
        uint32_t last = 0;
        for (uint64_t i = 0; i < d; ++i) {
            const uint32_t x = row[i];
            if ((cnt > 0 && x == last) || (uint64_t)x == u) continue;
            row[cnt++] = x;
            last = x;
        }
        newdeg[u] = cnt;
    }
}

__global__ void k_dedup_long(const uint64_t* off, uint32_t* nbr, uint64_t n, uint32_t* newdeg) {
    const int lane = (int)__lane_id();
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    const uint64_t w0 = (uint64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    for (uint64_t u = w0; u < n; u += waves) {
        const uint64_t o = off[u], d = off[u + 1] - o;
        if (d <= kThreadRow) continue;
        uint32_t* row = nbr + o;
        uint64_t cnt = 0;
        for (uint64_t c = 0; c < d; c += 64) {
            const uint64_t i = c + (uint64_t)lane;
            const bool valid = i < d;
            const uint32_t x = valid ? row[i] : 0u;
            // the value before this one in the row (the previous chunk's last for lane 0)
            uint32_t before = __shfl_up(x, 1, 64);
            const uint32_t chunk_prev = c > 0 ? row[c - 1] : 0u;
            if (lane == 0) before = chunk_prev;
            const bool first = (i == 0) || x != before;
            const bool keep = valid && first && (uint64_t)x != u;
            const uint64_t m = __ballot(keep);
            const uint64_t below = m & ((1ull << lane) - 1ull);
            // the chunk's values are in registers before any write; a write
            // lands at or below its own lane's position (cnt <= c), and
            // position c + 63, read as the next chunk's predecessor, is only
            // ever rewritten with its own value
            if (keep) row[cnt + (uint64_t)__popcll(below)] = x;
            cnt += (uint64_t)__popcll(m);
        }
        if (lane == 0) newdeg[u] = (uint32_t)cnt;
    }
}

// Rows [r0, r1) from the staging copy of their old span (starting at
// old_off[r0]) onto their new offsets: one thread per short row, one wave
// per long row.
__global__ void k_move_short(const uint64_t* old_off, const uint64_t* new_off, uint64_t r0, uint64_t r1,
                             const uint32_t* stage, uint32_t* nbr) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t base = old_off[r0];
    for (uint64_t u = r0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < r1; u += stride) {
        const uint64_t d = new_off[u + 1] - new_off[u];
        if (d > kThreadRow) continue;
        const uint32_t* src = stage + (old_off[u] - base);
        uint32_t* dst = nbr + new_off[u];
        for (uint64_t i = 0; i < d; ++i) dst[i] = src[i];
    }
}

__global__ void k_move_long(const uint64_t* old_off, const uint64_t* new_off, uint64_t r0, uint64_t r1,
                            const uint32_t* stage, uint32_t* nbr) {
    const int lane = (int)__lane_id();
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    const uint64_t base = old_off[r0];
    for (uint64_t u = r0 + (uint64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; u < r1; u += waves) {
        const uint64_t d = new_off[u + 1] - new_off[u];
        if (d <= kThreadRow) continue;
        const uint32_t* src = stage + (old_off[u] - base);
        uint32_t* dst = nbr + new_off[u];
        for (uint64_t i = (uint64_t)lane; i < d; i += 64) dst[i] = src[i];
    }
}

}  // namespace

extern "C" {

// Degrees of the multigraph (both endpoints of every non-loop edge) added
// into deg (device uint32[2^scale], zeroed by the caller).
int synth_rmat_count(uint32_t* deg, uint64_t n_edges, uint32_t scale, double a, double b, double c, uint64_t seed,
                     void* stream) {
    if (scale == 0 || scale > 32) return -1;
    RmatParams P{n_edges, seed, a, a + b, a + b + c, scale};
    hipLaunchKernelGGL(k_count, dim3(grid(n_edges)), dim3(kThreads), 0, (hipStream_t)stream, P, deg);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Both directions of every non-loop edge into its rows: off (device
// uint64[n + 1]) from the counts, cursor (device uint32[n], zeroed), nbr
// (device uint32[off[n]]).
int synth_rmat_fill(const uint64_t* off, uint32_t* cursor, uint32_t* nbr, uint64_t n_edges, uint32_t scale, double a,
                    double b, double c, uint64_t seed, void* stream) {
    if (scale == 0 || scale > 32) return -1;
    RmatParams P{n_edges, seed, a, a + b, a + b + c, scale};
    hipLaunchKernelGGL(k_fill, dim3(grid(n_edges)), dim3(kThreads), 0, (hipStream_t)stream, P, off, cursor, nbr);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Sorts every row of (off, nbr) and keeps its distinct values (no value
// equal to the row id), front-packed; newdeg (device uint32[n]) receives
// their counts.  stage: device scratch of stage_bytes (a quarter for the
// sort's output, a quarter for the batch offsets, a half for its temporary
// storage); batches of consecutive rows whose slots fit in a quarter of it
// (below 2^30 slots and 2^22 rows) are sorted at a time.
int synth_sort_dedup_rows(const uint64_t* off, uint32_t* nbr, uint64_t n, uint32_t* newdeg, void* stage,
                          uint64_t stage_bytes, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    std::vector<uint64_t> h_off(n + 1);
    if (hipMemcpyAsync(h_off.data(), off, (n + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, st) != hipSuccess)
        return -2;
    if (hipStreamSynchronize(st) != hipSuccess) return -2;
    uint64_t cap = stage_bytes / 4 / sizeof(uint32_t);
    if (cap > (1ull << 30)) cap = 1ull << 30;
    char* base = (char*)stage;
    uint32_t* out = (uint32_t*)base;                         // a quarter: sorted keys
    int* rel = (int*)(base + stage_bytes / 4);                // a quarter: batch offsets
    char* temp = base + stage_bytes / 2;                      // a half: the sort's temporary storage
    const uint64_t temp_bytes = stage_bytes - stage_bytes / 2;
    // at most 2^22 segments per sort: the segmented sort's launches grow
    // with the segment count, and batches of many more short rows (the high
    // ids of an R-MAT graph) were left unsorted without an error
    uint64_t max_rows = stage_bytes / 4 / sizeof(int) - 1;
    if (max_rows > (1ull << 22)) max_rows = 1ull << 22;
    uint64_t r0 = 0;
    uint64_t batch_cap = cap;
    while (r0 < n) {
        // the longest run of rows from r0 whose slots fit (at least one row)
        uint64_t lo = r0 + 1, hi = n;
        while (lo < hi) {
            const uint64_t mid = (lo + hi + 1) / 2;
            if (h_off[mid] - h_off[r0] <= batch_cap && mid - r0 <= max_rows)
                lo = mid;
            else
                hi = mid - 1;
        }
        const uint64_t r1 = lo;
        const uint64_t items = h_off[r1] - h_off[r0];
        if (items > cap) return -3;  // one row longer than the staging buffer allows
        if (items > 0) {
            size_t need = 0;
            if (hipcub::DeviceSegmentedSort::SortKeys(nullptr, need, nbr + h_off[r0], out, (int)items, (int)(r1 - r0),
                                                      rel, rel + 1, st) != hipSuccess)
                return -2;
            if (need > temp_bytes) {
                // the sort's temporary storage outgrows its half: a smaller batch
                if (r1 - r0 == 1 || batch_cap < 2) return -4;
                batch_cap = items / 2;
                continue;
            }
            hipLaunchKernelGGL(k_rel_offsets, dim3(grid(r1 - r0 + 1)), dim3(kThreads), 0, st, off, r0, r1 - r0, rel);
            if (hipcub::DeviceSegmentedSort::SortKeys(temp, need, nbr + h_off[r0], out, (int)items, (int)(r1 - r0),
                                                      rel, rel + 1, st) != hipSuccess)
                return -2;
            if (hipMemcpyAsync(nbr + h_off[r0], out, items * sizeof(uint32_t), hipMemcpyDeviceToDevice, st) !=
                hipSuccess)
                return -2;
        }
        r0 = r1;
        batch_cap = cap;
    }
    hipLaunchKernelGGL(k_dedup_short, dim3(grid(n)), dim3(kThreads), 0, st, off, nbr, n, newdeg);
    hipLaunchKernelGGL(k_dedup_long, dim3(2048), dim3(kThreads), 0, st, off, nbr, n, newdeg);
    if (hipGetLastError() != hipSuccess) return -2;
    return hipStreamSynchronize(st) == hipSuccess ? 0 : -2;
}

// Moves every row's first new_off[u + 1] - new_off[u] values from old_off[u]
// to new_off[u] (new_off[u] <= old_off[u] for every u), batches of
// consecutive rows at a time through stage (device, stage_bytes): a batch's
// old span is copied to the stage before its rows are written, and every
// earlier batch is already in place, so no value is overwritten before it
// is read.
int synth_compact_rows(const uint64_t* old_off, const uint64_t* new_off, uint32_t* nbr, uint64_t n, void* stage,
                       uint64_t stage_bytes, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    std::vector<uint64_t> h_off(n + 1);
    if (hipMemcpyAsync(h_off.data(), old_off, (n + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, st) != hipSuccess)
        return -2;
    if (hipStreamSynchronize(st) != hipSuccess) return -2;
    const uint64_t cap = stage_bytes / sizeof(uint32_t);
    uint32_t* sbuf = (uint32_t*)stage;
    uint64_t r0 = 0;
    while (r0 < n) {
        uint64_t lo = r0 + 1, hi = n;
        while (lo < hi) {
            const uint64_t mid = (lo + hi + 1) / 2;
            if (h_off[mid] - h_off[r0] <= cap)
                lo = mid;
            else
                hi = mid - 1;
        }
        const uint64_t r1 = lo;
        const uint64_t items = h_off[r1] - h_off[r0];
        if (items > cap) return -3;
        if (items > 0 &&
            hipMemcpyAsync(sbuf, nbr + h_off[r0], items * sizeof(uint32_t), hipMemcpyDeviceToDevice, st) != hipSuccess)
            return -2;
        hipLaunchKernelGGL(k_move_short, dim3(grid(r1 - r0)), dim3(kThreads), 0, st, old_off, new_off, r0, r1, sbuf,
                           nbr);
        hipLaunchKernelGGL(k_move_long, dim3(1024), dim3(kThreads), 0, st, old_off, new_off, r0, r1, sbuf, nbr);
        if (hipGetLastError() != hipSuccess) return -2;
        r0 = r1;
    }
    return hipStreamSynchronize(st) == hipSuccess ? 0 : -2;
}

}  // extern "C"
