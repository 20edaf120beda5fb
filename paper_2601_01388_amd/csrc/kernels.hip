// gfx950 kernels of the AGIS library: CSR validation, per-vertex proposal
// tables (Sec. 4.4), the first-step proposal over all vertices, and the
// sampling kernel (Algorithm 3) with its estimator partials (Algorithm 1).
//
// Execution model of the sampler: one 64-lane wavefront owns one sample at
// a time.  Control flow is wave-uniform (every lane holds the same matched
// prefix, factors and weight); the lanes cooperate on the data-parallel
// parts of a step: the 64-ary searches of the first step, the probes of
// already-matched vertices, and the chunked walk over the shortest
// backward neighbour list that builds the candidate set, its integer
// weights and the prefix pick.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "agis_internal.h"

namespace agis {

__constant__ int32_t c_logtab[4096];
__constant__ uint32_t c_exp2tab[4096];
// the same table staged in LDS by the sampling kernel (each block fills its
// copy once), for the weighted picks
__shared__ uint32_t s_exp2tab[4096];

namespace {
std::vector<int32_t> g_logtab;
std::vector<uint32_t> g_exp2tab;

void ensure_host_tables() {
    if (!g_logtab.empty()) return;
    g_logtab.resize(4096);
    g_exp2tab.resize(4096);
    for (int j = 0; j < 4096; ++j) {
        const double frac = (double)j / 4096.0;
        g_logtab[j] = (int32_t)std::llround(65536.0 * std::log2(1.0 + frac));
        g_exp2tab[j] = (uint32_t)std::llround(2147483648.0 * std::exp2(-frac));
    }
}
}  // namespace

const int32_t* host_logtab() {
    ensure_host_tables();
    return g_logtab.data();
}

const uint32_t* host_exp2tab() {
    ensure_host_tables();
    return g_exp2tab.data();
}

hipError_t upload_fixed_point_tables(hipStream_t stream) {
    ensure_host_tables();
    hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_logtab), g_logtab.data(), 4096 * sizeof(int32_t), 0,
                                          hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return e;
    e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_exp2tab), g_exp2tab.data(), 4096 * sizeof(uint32_t), 0,
                               hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(stream);
}

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
namespace {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint32_t readlane_u32(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
    uint32_t lo = readlane_u32((uint32_t)v, l);
    uint32_t hi = readlane_u32((uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// A wave-uniform value moved to a scalar register (the compiler cannot
// always prove uniformity, and a uniform value in a vector register costs
// 64 lanes of register file).
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    return ((uint64_t)uniform_u32((uint32_t)(v >> 32)) << 32) | uniform_u32((uint32_t)v);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        int32_t w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint64_t w = __shfl_up(v, d, kWave);
        if (lane >= d) v += w;
    }
    return v;
}

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// Segments of equal keys in a wave whose keys do not decrease across lanes:
// head = first lane of this lane's segment, tail = this lane ends it.
__device__ __forceinline__ void wave_segments(uint32_t key, int& head, bool& tail) {
    const int lane = lane_id();
    const uint32_t prev = __shfl_up(key, 1, kWave);
    const uint64_t heads = __ballot(lane == 0 || prev != key);
    head = 63 - __clzll(heads & ((2ull << lane) - 1ull));
    const uint32_t next = __shfl_down(key, 1, kWave);
    tail = lane == kWave - 1 || next != key;
}

// Memory-request accounting of the sampler.  The production kernel carries
// NoMeter (every call compiles to nothing); the metering kernel carries a
// Meter, which counts for one sample the bytes its global loads (reads) and
// stores (writes) ask for, the 64-byte segments each wave-level access
// touches (an access's segments, less the first one when it is the previous
// lane's last), and the wave-level requests.  Every method is called by the
// whole wave with wave-uniform counters; LDS traffic is not counted.
struct NoMeter {
    static constexpr bool kOn = false;
    __device__ __forceinline__ void vec(const void*, uint32_t, bool, bool = false) {}
    __device__ __forceinline__ void uni(const void*, uint32_t, bool = false) {}
    __device__ __forceinline__ void lanes(uint32_t, uint32_t) {}
    __device__ __forceinline__ void span(const void*, uint64_t, uint32_t) {}
};

struct Meter {
    static constexpr bool kOn = true;
    uint64_t rbytes = 0, wbytes = 0, segs = 0, reqs = 0;
    // one access of `width` bytes (per lane) at p by every lane with `active`
    __device__ __forceinline__ void vec(const void* p, uint32_t width, bool active, bool write = false) {
        const uint64_t am = __ballot(active);
        if (am == 0) return;
        const int lane = lane_id();
        const uint64_t a = (uint64_t)(uintptr_t)p;
        const uint64_t s0 = a >> 6, s1 = (a + width - 1) >> 6;
        const uint64_t prev = __shfl_up(s1, 1, kWave);
        const bool pact = lane > 0 && ((am >> (lane - 1)) & 1ull);
        const uint64_t mine = active ? (s1 - s0 + 1 - ((pact && prev == s0) ? 1 : 0)) : 0;
        const uint64_t b = wave_sum_u64(active ? (uint64_t)width : 0ull);
        if (write)
            wbytes += b;
        else
            rbytes += b;
        segs += wave_sum_u64(mine);
        reqs += 1;
    }
    // one wave-uniform access of `width` bytes at p
    __device__ __forceinline__ void uni(const void* p, uint32_t width, bool write = false) {
        const uint64_t a = (uint64_t)(uintptr_t)p;
        if (write)
            wbytes += width;
        else
            rbytes += width;
        segs += ((a + width - 1) >> 6) - (a >> 6) + 1;
        reqs += 1;
    }
    // independent per-lane loops of `loads` accesses of `width` bytes each
    // at scattered addresses (binary searches): one segment per access, as
    // many wave-level requests as the longest loop
    __device__ __forceinline__ void lanes(uint32_t loads, uint32_t width) {
        uint64_t v = loads;
        const uint64_t tot = wave_sum_u64(v);
        uint32_t mx = loads;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t w = (uint32_t)__shfl_xor((int)mx, o, kWave);
            mx = w > mx ? w : mx;
        }
        rbytes += tot * width;
        segs += tot;
        reqs += mx;
    }
    // a contiguous read of `bytes` bytes at p in wave-level requests of
    // `per_req` bytes
    __device__ __forceinline__ void span(const void* p, uint64_t bytes, uint32_t per_req) {
        if (bytes == 0) return;
        const uint64_t a = (uint64_t)(uintptr_t)p;
        rbytes += bytes;
        segs += ((a + bytes - 1) >> 6) - (a >> 6) + 1;
        reqs += (bytes + per_req - 1) / per_req;
    }
};

// Inclusive sum of v over this lane's segment so far.
__device__ __forceinline__ uint64_t wave_segmented_sum_u64(uint64_t v, int head) {
    const uint64_t incl = wave_incl_scan_u64(v);
    const uint64_t before = __shfl(incl, head > 0 ? head - 1 : 0, kWave);
    return head > 0 ? incl - before : incl;
}

// lower bound of x in a sorted list: first position with list[pos] >= x
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* __restrict__ list, uint32_t len, uint32_t x) {
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (list[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool contains_u32(const uint32_t* __restrict__ list, uint32_t len, uint32_t x) {
    uint32_t p = lower_bound_u32(list, len, x);
    return p < len && list[p] == x;
}

// contains_u32 that also adds its element reads to `loads`
__device__ __forceinline__ bool contains_u32_counted(const uint32_t* __restrict__ list, uint32_t len, uint32_t x,
                                                     uint32_t& loads) {
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        ++loads;
        if (list[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo < len) ++loads;
    return lo < len && list[lo] == x;
}

// Row of edge slot e: the vertex v with off[v] <= e < off[v + 1].
__device__ __forceinline__ uint32_t row_of_slot(const uint64_t* __restrict__ off, uint64_t n, uint64_t e) {
    uint64_t lo = 0, hi = n;  // first v with off[v + 1] > e
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        if (off[mid + 1] > e)
            hi = mid;
        else
            lo = mid + 1;
    }
    return (uint32_t)lo;
}

// Wave-cooperative 64-ary search: first index p in [0, n) with a[p] > r,
// given a non-decreasing and a[n - 1] > r.  Every lane returns the answer.
template <class MT = NoMeter>
__device__ __forceinline__ uint64_t wave_first_greater(const uint64_t* __restrict__ a, uint64_t n, uint64_t r,
                                                       MT&& mt = MT()) {
    const int lane = lane_id();
    uint64_t lo = 0, hi = n - 1;  // answer in [lo, hi], a[hi] > r
    while (hi - lo + 1 > (uint64_t)kWave) {
        const uint64_t step = (hi - lo + kWave) >> 6;
        const uint64_t p = lo + (uint64_t)lane * step;
        const bool valid = p <= hi;
        mt.vec(a + p, 8, valid);
        const bool pred = valid && a[p] > r;
        const uint64_t m = __ballot(pred);
        if (m == 0) {
            const uint64_t vm = __ballot(valid);
            const int last = 63 - __clzll(vm);
            lo = lo + (uint64_t)last * step + 1;
        } else {
            const int f = __ffsll((unsigned long long)m) - 1;
            const uint64_t nh = lo + (uint64_t)f * step;
            if (f > 0) lo = lo + (uint64_t)(f - 1) * step + 1;
            hi = nh;
        }
    }
    const uint64_t p = lo + (uint64_t)lane;
    mt.vec(a + p, 8, p <= hi);
    const bool pred = p <= hi && a[p] > r;
    const uint64_t m = __ballot(pred);
    return lo + (uint64_t)(__ffsll((unsigned long long)m) - 1);
}

// Wave-cooperative: first position p in [lo, hi) with list[p] > key, or hi
// when there is none (list ascending).
template <class MT = NoMeter>
__device__ __forceinline__ uint32_t wave_first_greater_u32(const uint32_t* __restrict__ list, uint32_t lo, uint32_t hi,
                                                           uint32_t key, MT&& mt = MT()) {
    const int lane = lane_id();
    while (hi - lo > (uint32_t)kWave) {  // answer in [lo, hi]
        const uint32_t step = (hi - lo + kWave - 1) >> 6;
        const uint32_t p = lo + (uint32_t)lane * step;
        const bool valid = p < hi;
        mt.vec(list + p, 4, valid);
        const uint64_t m = __ballot(valid && list[p] > key);
        if (m == 0) {
            const int last = 63 - __clzll(__ballot(valid));
            lo = lo + (uint32_t)last * step + 1;
        } else {
            const int f = __ffsll((unsigned long long)m) - 1;
            const uint32_t nh = lo + (uint32_t)f * step;
            if (f > 0) lo = lo + (uint32_t)(f - 1) * step + 1;
            hi = nh;
        }
    }
    const uint32_t p = lo + (uint32_t)lane;
    mt.vec(list + p, 4, p < hi);
    const uint64_t m = __ballot(p < hi && list[p] > key);
    return m ? lo + (uint32_t)(__ffsll((unsigned long long)m) - 1) : hi;
}

// One backward list co-iterated with a chunk of ascending base elements
// (this lane's element xv, the chunk's largest xlast).  Elements of `list`
// before `pos` are below every element of the chunk, so membership of xv
// is decided inside the window [pos, end) of elements <= xlast.  The window
// is streamed in coalesced 256-element blocks, each searched for every
// lane's xv with register shuffles, until a block holds an element above
// xlast: the bytes read are the window itself, as in a merge.  When the
// window is expected to be far longer than the chunk (the list is much
// longer than what is left of the base: left = base elements from this
// chunk on), it is bounded by a 64-ary wave search instead and searched
// per lane.  Clears `member` when xv is absent; returns end, the window
// start of the next chunk.
constexpr uint32_t kStreamMaxWindow = 2048;

// The value `v` held by lane `src` (0..63), as seen by this lane: one
// ds_bpermute.  Every lane of the wave must execute it.
__device__ __forceinline__ uint32_t bperm(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}

// Whether this lane's xv occurs among the 64 ascending values held one per
// lane (val): a binary search by shuffles.  Every lane must take part (a
// lane outside the exec mask would not supply its value to the others).
__device__ __forceinline__ bool piece_contains(uint32_t val, uint32_t xv) {
    int lo = 0;
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) {
        const uint32_t pv = bperm(val, lo + s - 1);
        lo += pv < xv ? s : 0;
    }
    const uint32_t cand = bperm(val, lo);
    return cand == xv;
}

// Lower bounds of up to eight keys in one ascending list, searched
// together: the wave splits into groups of G lanes (G = 16 for up to four
// keys, else 8), group q searching for the key of lane q (if `need` there)
// with G probes per level, each level cutting the interval (G + 1)-fold.
// Lane q receives the first position whose element is not below its key
// (d when there is none) and, in `found`, whether that element is the key.
// Every lane must call it; nq (<= 8, wave-uniform) bounds the query lanes.
template <class MT>
__device__ __forceinline__ uint32_t wave_lower_bound_keys(const uint32_t* __restrict__ list, uint32_t d, uint32_t key,
                                                          bool need, uint32_t nq, bool& found, MT& mt) {
    const int lane = lane_id();
    const int sh = nq <= 4 ? 4 : 3;
    const uint32_t G = 1u << sh;
    // x / (G + 1) for any 32-bit x as a multiply-high and a shift
    // (multipliers ceil(2^36 / 17) and ceil(2^33 / 9))
    const uint32_t mg = nq <= 4 ? 0xF0F0F0F1u : 0x38E38E39u;
    const uint32_t ms = nq <= 4 ? 4u : 1u;
    auto div = [&](uint32_t x) { return __umulhi(x, mg) >> ms; };
    const int q = lane >> sh;
    const uint32_t s = (uint32_t)lane & (G - 1u);
    const uint32_t qkey = bperm(key, q);
    const bool qneed = bperm(need ? 1u : 0u, q) != 0u;
    const uint64_t gmask = ((G == 16u) ? 0xFFFFull : 0xFFull) << ((uint32_t)q * G);
    uint32_t lo = 0, hi = qneed ? d : 0u;  // answer in [lo, hi]
    uint32_t hival = 0;                    // the element at hi, once a probe has set hi
    bool hset = false;
    while (__ballot(lo < hi)) {
        const bool active = lo < hi;  // uniform within a group
        // probe t (1..G) at lo + floor(t span / (G + 1)), in 32 bits:
        // span = a (G + 1) + b gives t a + floor(t b / (G + 1))
        const uint32_t span = hi - lo;
        const uint32_t a = div(span), b = span - a * (G + 1u);
        auto at = [&](uint32_t t) { return lo + t * a + div(t * b); };
        const uint32_t p = at(s + 1u);
        mt.vec(list + p, 4, active);
        const uint32_t val = active ? list[p] : 0u;
        // probes below the key form a prefix of the group's probes
        const uint32_t c = (uint32_t)__popcll(__ballot(active && val < qkey) & gmask);
        const uint32_t vc = bperm(val, (int)((uint32_t)q * G + (c < G ? c : G - 1u)));
        if (active) {
            const uint32_t nlo = c > 0u ? at(c) + 1u : lo;
            if (c < G) {
                hi = at(c + 1u);
                hival = vc;
                hset = true;
            }
            lo = nlo;
        }
    }
    // lane j < 64 / G takes the answer of group j (from its first lane)
    const int src = (lane * (int)G) & (kWave - 1);
    found = bperm((hset && lo < d && hival == qkey) ? 1u : 0u, src) != 0u;
    return bperm(lo, src);
}

template <class MT>
__device__ __forceinline__ uint32_t co_iterate_member(const uint32_t* __restrict__ list, uint32_t pos, uint32_t len,
                                                      uint32_t xv, uint32_t xlast, uint32_t left, bool& member,
                                                      MT& mt) {
    const int lane = lane_id();
    // expected window (len - pos) * 64 / left <= kStreamMaxWindow, without a
    // division; the streaming path takes positions as 32-bit signed values
    if (len < 0x7FFFFF00u && (uint64_t)(len - pos) * kWave <= (uint64_t)kStreamMaxWindow * (left ? left : 1u)) {
        // Blocks of 256 elements, 4 consecutive ones per lane from one
        // 16-byte load (blocks are aligned to 16 bytes in memory, so the
        // first may start up to 3 elements before pos; elements before pos
        // are below the chunk and never match).  A lane finds the lane whose
        // quad may hold its xv by a shuffle search over the quads' first
        // elements, then compares with that quad: 10 shuffles per 256
        // elements.  Reads stay inside [0, len) of the list.
        constexpr uint32_t kNone = 0xFFFFFFFFu;  // ids are < n <= 2^32 - 1
        // positions as 32-bit signed values (the caller keeps len < 2^31)
        const int32_t mis = (int32_t)(((uintptr_t)list >> 2) & 3u);
        const int32_t ilen = (int32_t)len;
        const int32_t ipos = (int32_t)pos;
        int32_t qs = ((ipos + mis) & ~3) - mis;  // block start, >= pos - 3
        bool hit = false;
        for (;;) {
            const int32_t e = qs + 4 * lane;
            // The block read as one ascending sequence: zero fill before the
            // list's start, the list, none after its end.  Its elements
            // before pos are at most the previous chunk's largest element,
            // so below every xv of this chunk: they never match xv and never
            // end the window.
            uint32_t v0, v1, v2, v3;
            if (qs >= 0 && qs + 4 * kWave <= ilen) {  // the whole block is in the list
                mt.vec(list + e, 16, true);
                const uint4 q = *reinterpret_cast<const uint4*>(list + e);
                v0 = q.x;
                v1 = q.y;
                v2 = q.z;
                v3 = q.w;
            } else {
                if constexpr (MT::kOn) {
                    // the elements of the block inside the list
                    const int32_t ea = e < 0 ? 0 : e, eb = e + 4 < ilen ? e + 4 : ilen;
                    mt.vec(list + ea, eb > ea ? 4u * (uint32_t)(eb - ea) : 4u, eb > ea);
                }
                v0 = e < 0 ? 0u : (e < ilen ? list[e] : kNone);
                v1 = e + 1 < 0 ? 0u : (e + 1 < ilen ? list[e + 1] : kNone);
                v2 = e + 2 < 0 ? 0u : (e + 2 < ilen ? list[e + 2] : kNone);
                v3 = e + 3 < ilen ? list[e + 3] : kNone;
            }
            // the elements <= xlast form a prefix of the block
            const uint64_t m0 = __ballot(v0 > xlast);
            const uint64_t m1 = __ballot(v1 > xlast);
            const uint64_t m2 = __ballot(v2 > xlast);
            const uint64_t m3 = __ballot(v3 > xlast);
            // membership of xv: the lane whose quad may hold it, then its quad
            int lo = 0;
#pragma unroll
            for (int s = 32; s > 0; s >>= 1) {
                const uint32_t pv = bperm(v0, lo + s);
                lo += pv <= xv ? s : 0;
            }
            const uint32_t a0 = bperm(v0, lo);
            const uint32_t a1 = bperm(v1, lo);
            const uint32_t a2 = bperm(v2, lo);
            const uint32_t a3 = bperm(v3, lo);
            // the zero fill before the list's start (at most the first 3
            // elements of the block) may equal xv = 0
            const int32_t fill = -(qs + 4 * lo);
            hit = hit | ((a0 == xv) & (fill <= 0)) | ((a1 == xv) & (fill <= 1)) | ((a2 == xv) & (fill <= 2)) |
                  (a3 == xv);
            if ((m0 | m1 | m2 | m3) != 0) {
                member = member && hit;
                return (uint32_t)(qs + __popcll(~m0) + __popcll(~m1) + __popcll(~m2) + __popcll(~m3));
            }
            qs += 4 * kWave;
        }
    }
    const uint32_t p = pos + (uint32_t)lane;
    mt.vec(list + p, 4, p < len);
    const uint32_t val = p < len ? list[p] : 0xFFFFFFFFu;
    const uint64_t gt = __ballot(val > xlast);
    if (gt != 0) {
        const bool in = piece_contains(val, xv);
        member = member && in;
        return pos + (uint32_t)(__ffsll((unsigned long long)gt) - 1);
    }
    const uint32_t end = wave_first_greater_u32(list, pos + kWave, len, xlast, mt);
    if constexpr (MT::kOn) {
        uint32_t loads = 0;
        if (member) member = contains_u32_counted(list + pos, end - pos, xv, loads);
        mt.lanes(loads, 4);
    } else {
        if (member) member = contains_u32(list + pos, end - pos, xv);
    }
    return end;
}

__device__ __forceinline__ int32_t approx_log_weight(uint4 rec, uint32_t b, uint32_t f1, uint32_t ie, uint32_t f2) {
    const uint32_t d = rec.x;
    if (d < b + f1) return kCertainZero;
    int32_t l = 0;
    for (uint32_t t = 0; t < f1; ++t) l += log2fx((uint64_t)(d - b - t), c_logtab);
    l += (int32_t)ie * (int32_t)rec.z;
    l += (int32_t)f2 * (int32_t)rec.y;
    return l;
}

}  // namespace

// ---------------------------------------------------------------------------
// CSR validation and max degree
// ---------------------------------------------------------------------------
__global__ void k_validate_rows(DevGraph g, uint32_t* flags) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    if (g.off[v + 1] < g.off[v] || g.off[v + 1] > g.nnz) atomicOr(flags, 1u);
}

// Per-slot kernels run a grid-stride loop over 64-bit slot indices on a
// capped grid (a dispatch holds at most 2^32 work-items, fewer than the
// slots of the largest graphs).
__global__ void k_validate_edges(DevGraph g, uint32_t* flags) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < g.nnz; e += stride) {
        const uint32_t v = row_of_slot(g.off, g.n, e);
        if (v >= g.n) {
            atomicOr(flags, 1u);
            continue;
        }
        // offsets were checked (monotone, within nnz) by k_validate_rows first
        const uint32_t x = g.nbr[e];
        uint32_t f = 0;
        if ((uint64_t)x >= g.n) {
            atomicOr(flags, 2u);
            continue;
        }
        if (x == v) f |= 4u;
        if (e + 1 < g.off[v + 1] && g.nbr[e + 1] <= x) f |= 8u;
        const uint64_t o = g.off[x];
        const uint64_t d = g.off[x + 1] - o;
        if (d > 0xFFFFFFFFull || !contains_u32(g.nbr + o, (uint32_t)d, v)) f |= 16u;
        if (f) atomicOr(flags, f);
    }
}

__global__ void k_max_degree(DevGraph g, uint32_t* out) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t d = v < g.n ? (uint32_t)(g.off[v + 1] - g.off[v]) : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t w = __shfl_xor(d, o, kWave);
        d = w > d ? w : d;
    }
    if (lane_id() == 0 && d) atomicMax(out, d);
}

static unsigned grid_for(uint64_t n, unsigned threads) { return (unsigned)((n + threads - 1) / threads); }

// Workgroups of a grid-stride launch over n items: enough to cover them up
// to kStrideBlocks (2^20 workgroups of 256 = 2^28 work-items per pass).
constexpr uint64_t kStrideBlocks = 1ull << 20;
static unsigned stride_grid(uint64_t n, unsigned threads) {
    const uint64_t b = (n + threads - 1) / threads;
    return (unsigned)(b < kStrideBlocks ? b : kStrideBlocks);
}

hipError_t launch_validate_rows(const DevGraph& g, uint32_t* d_flags, hipStream_t stream) {
    if (g.n) hipLaunchKernelGGL(k_validate_rows, dim3(grid_for(g.n, 256)), dim3(256), 0, stream, g, d_flags);
    return hipGetLastError();
}

hipError_t launch_validate_edges(const DevGraph& g, uint32_t* d_flags, hipStream_t stream) {
    if (g.nnz) hipLaunchKernelGGL(k_validate_edges, dim3(stride_grid(g.nnz, 256)), dim3(256), 0, stream, g, d_flags);
    return hipGetLastError();
}

hipError_t launch_max_degree(const DevGraph& g, uint32_t* d_max, hipStream_t stream) {
    if (g.n) hipLaunchKernelGGL(k_max_degree, dim3(grid_for(g.n, 256)), dim3(256), 0, stream, g, d_max);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-vertex proposal tables (Sec. 4.4)
// ---------------------------------------------------------------------------
__global__ void k_tables_init(DevGraph g, uint4* rec, uint64_t* s2, uint64_t* hits) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    rec[v] = make_uint4((uint32_t)(g.off[v + 1] - g.off[v]), 0u, 0u, 0u);
    s2[v] = 0;
    hits[v] = 0;
}

// One thread per edge slot (v, x): adds d(x) to S2(v) and, for the sampled
// clustering coefficient, runs trial t = slot - off[v] of vertex v: an
// ordered pair (a, b) of distinct neighbour positions from Philox key
// cv_seed, counter (v, t, 0, tag 0 / tag 1), a hit when the two neighbours
// are adjacent.  For the exact coefficient, counts the neighbours z > x of v
// that are adjacent to x (each edge among N(v) once).
__global__ __launch_bounds__(256) void k_tables_edges(DevGraph g, DevGraph adj, const uint4* rec, uint64_t* s2,
                                                       uint64_t* hits, uint32_t k0, uint32_t k1, int exact) {
    // grid-stride over slots; the loop bound is uniform in a workgroup, so
    // every lane of a wave takes part in the wave-wide sums below
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < g.nnz; base += stride) {
    const uint64_t e = base + threadIdx.x;
    const bool active = e < g.nnz;
    uint32_t v = 0xFFFFFFFFu;
    uint64_t dx = 0, h = 0;
    if (active) {
        v = row_of_slot(g.off, g.n, e);
        const uint32_t x = g.nbr[e];
        const uint64_t ov = g.off[v];
        const uint32_t d = rec[v].x;
        dx = rec[x].x;
        const uint32_t* row = g.nbr + ov;
        if (d >= 2 && !exact) {
            const uint32_t t = (uint32_t)(e - ov);
            const uint64_t a = bounded_draw(k0, k1, v, t, 0, 0, d);
            uint64_t b = bounded_draw(k0, k1, v, t, 0, 1, d - 1);
            if (b >= a) ++b;
            const uint32_t y = row[a], z = row[b];
            const uint64_t oy = adj.off[y];
            h = contains_u32(adj.nbr + oy, (uint32_t)(adj.off[y + 1] - oy), z) ? 1u : 0u;
        } else if (d >= 2) {
            const uint64_t ox = adj.off[x];
            const uint32_t dxx = (uint32_t)(adj.off[x + 1] - ox);
            for (uint32_t p = lower_bound_u32(row, d, x + 1); p < d; ++p)
                if (contains_u32(adj.nbr + ox, dxx, row[p])) ++h;
        }
    }
    // consecutive slots mostly share a row: one atomic per row segment of the wave
    int head;
    bool tail;
    wave_segments(v, head, tail);
    const uint64_t sdx = wave_segmented_sum_u64(dx, head);
    const uint64_t sh = wave_segmented_sum_u64(h, head);
    if (active && tail) {
        atomicAdd((unsigned long long*)&s2[v], (unsigned long long)sdx);
        if (sh) atomicAdd((unsigned long long*)&hits[v], (unsigned long long)sh);
    }
    }
}

__global__ void k_tables_finalize(DevGraph g, uint4* rec, const uint64_t* s2, const uint64_t* hits, uint64_t* trials,
                                  int32_t lc_min, int exact) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    uint4 r = rec[v];
    const uint64_t d = r.x;
    const uint64_t t = d < 2 ? 0 : (exact ? d * (d - 1) / 2 : d);
    trials[v] = t;
    // S2 = 0 happens only on an oriented graph (out-neighbours without
    // out-neighbours); LA is then 0, as for d = 0 (cliques never use it)
    const int32_t la = (d >= 1 && s2[v] > 0) ? log2fx(s2[v], c_logtab) - log2fx(d, c_logtab) : 0;
    int32_t lc = lc_min;
    const uint64_t h = hits[v];
    if (d >= 2 && h > 0) {
        const int32_t c = log2fx(h, c_logtab) - log2fx(t, c_logtab);
        lc = c > lc_min ? c : lc_min;
    }
    r.y = (uint32_t)la;
    r.z = (uint32_t)lc;
    rec[v] = r;
}

hipError_t launch_build_tables(const DevGraph& g, const DevGraph& adj, uint4* rec, uint64_t* s2, uint64_t* hits,
                               uint64_t* trials, uint32_t k0, uint32_t k1, int32_t lc_min, int exact,
                               hipStream_t stream) {
    if (!g.n) return hipSuccess;
    hipLaunchKernelGGL(k_tables_init, dim3(grid_for(g.n, 256)), dim3(256), 0, stream, g, rec, s2, hits);
    if (g.nnz)
        hipLaunchKernelGGL(k_tables_edges, dim3(stride_grid(g.nnz, 256)), dim3(256), 0, stream, g, adj, rec, s2, hits,
                           k0, k1, exact);
    hipLaunchKernelGGL(k_tables_finalize, dim3(grid_for(g.n, 256)), dim3(256), 0, stream, g, rec, s2, hits, trials,
                       lc_min, exact);
    return hipGetLastError();
}

__global__ void k_tables_export(const uint4* rec, uint64_t n, uint32_t* deg, int32_t* la, int32_t* lc) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const uint4 r = rec[v];
    if (deg) deg[v] = r.x;
    if (la) la[v] = (int32_t)r.y;
    if (lc) lc[v] = (int32_t)r.z;
}

hipError_t launch_export_tables(const agis_tables& t, uint64_t n, uint32_t* deg, int32_t* la, int32_t* lc,
                                hipStream_t stream) {
    if (n && (deg || la || lc))
        hipLaunchKernelGGL(k_tables_export, dim3(grid_for(n, 256)), dim3(256), 0, stream, t.rec, n, deg, la, lc);
    return hipGetLastError();
}

// Log weight (Q16) of every vertex for one step signature: the certain-zero
// marker where d(v) - b < f1, else the learned value lt[v] or the f_approx
// value.
__global__ void k_step_log_weights(const uint4* rec, uint64_t n, uint32_t b, uint32_t f1, uint32_t ie, uint32_t f2,
                                   const int32_t* lt, int32_t* out) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const uint4 r = rec[v];
    out[v] = r.x < b + f1 ? kCertainZero : (lt ? lt[v] : approx_log_weight(r, b, f1, ie, f2));
}

hipError_t launch_step_log_weights(const agis_tables& t, uint64_t n, uint32_t b, uint32_t f1, uint32_t ie, uint32_t f2,
                                   const int32_t* lt, int32_t* out, hipStream_t stream) {
    if (n)
        hipLaunchKernelGGL(k_step_log_weights, dim3(grid_for(n, 256)), dim3(256), 0, stream, t.rec, n, b, f1, ie, f2,
                           lt, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// First-step proposal over all vertices (the step-1 "cumulative
// distribution" of the paper): log weights, their maximum, integer weights
// and an inclusive 64-bit prefix, in three passes.
// ---------------------------------------------------------------------------
namespace {
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ int32_t step0_log(const uint4* rec, const DevPlan& P, uint64_t v) {
    const uint4 r = rec[v];
    if (r.x < (uint32_t)P.f1[0]) return kCertainZero;
    if (P.lt[0]) return P.lt[0][v];
    return approx_log_weight(r, 0, P.f1[0], P.ie[0], P.f2[0]);
}
}  // namespace

__global__ void k_step1_max(const uint4* rec, DevPlan P, uint64_t n, int32_t* lmax) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t l = kCertainZero;
    if (v < n) l = step0_log(rec, P, v);
    l = wave_max_i32(l);
    if (lane_id() == 0 && l != kCertainZero) atomicMax(lmax, l);
}

__device__ __forceinline__ uint32_t step0_weight(const uint4* rec, const DevPlan& P, uint64_t v, int32_t lmax) {
    const int32_t l = step0_log(rec, P, v);
    return l == kCertainZero ? 0u : weight_from_log(lmax, l, c_exp2tab);
}

__global__ __launch_bounds__(kScanThreads) void k_step1_tilesum(const uint4* rec, DevPlan P, uint64_t n,
                                                                 const int32_t* lmax_p, uint64_t* tile_sums) {
    const int32_t lmax = *lmax_p;
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint64_t s = 0;
    for (int j = 0; j < kScanItems; ++j) {
        const uint64_t v = base + (uint64_t)j * kScanThreads + threadIdx.x;
        if (v < n) s += step0_weight(rec, P, v, lmax);
    }
    s = wave_sum_u64(s);
    __shared__ uint64_t ws[kScanThreads / kWave];
    if (lane_id() == 0) ws[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < kScanThreads / kWave; ++w) t += ws[w];
        tile_sums[blockIdx.x] = t;
    }
}

// Exclusive scan of the tile sums in place by one workgroup.
__global__ __launch_bounds__(1024) void k_scan_tiles(uint64_t* tile_sums, uint64_t ntiles) {
    __shared__ uint64_t part[1024];
    const uint64_t per = (ntiles + 1023) / 1024;
    const uint64_t b = threadIdx.x * per;
    uint64_t s = 0;
    for (uint64_t j = 0; j < per && b + j < ntiles; ++j) s += tile_sums[b + j];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t run = 0;
        for (int j = 0; j < 1024; ++j) {
            uint64_t t = part[j];
            part[j] = run;
            run += t;
        }
    }
    __syncthreads();
    uint64_t run = part[threadIdx.x];
    for (uint64_t j = 0; j < per && b + j < ntiles; ++j) {
        uint64_t t = tile_sums[b + j];
        tile_sums[b + j] = run;
        run += t;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_step1_final(const uint4* rec, DevPlan P, uint64_t n,
                                                               const int32_t* lmax_p, const uint64_t* tile_offs,
                                                               uint32_t* q1, uint64_t* pre) {
    const int32_t lmax = *lmax_p;
    // thread t owns items [t*kScanItems, (t+1)*kScanItems) of the tile
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t q[kScanItems];
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint64_t v = base + j;
        q[j] = v < n ? step0_weight(rec, P, v, lmax) : 0u;
        s += q[j];
    }
    // exclusive scan of thread sums across the workgroup
    uint64_t incl = wave_incl_scan_u64(s);
    __shared__ uint64_t wsum[kScanThreads / kWave];
    const int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint64_t wbase = 0;
    for (int j = 0; j < w; ++j) wbase += wsum[j];
    uint64_t run = tile_offs[blockIdx.x] + wbase + incl - s;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint64_t v = base + j;
        if (v < n) {
            run += q[j];
            q1[v] = q[j];
            pre[v] = run;
        }
    }
}

// Weight sums of blocks of kStep1Block vertices (one wave per block, lane j
// summing vertices 4j .. 4j + 3 of it) into sums[b]; sums[nblk] = 0.
__global__ __launch_bounds__(256) void k_step1_blocksum(const uint4* rec, DevPlan P, uint64_t n,
                                                         const int32_t* lmax_p, uint64_t* sums) {
    const int32_t lmax = *lmax_p;
    const uint64_t nblk = (n + kStep1Block - 1) / kStep1Block;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / kWave);
    for (uint64_t b = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; b < nblk; b += waves) {
        const uint64_t v0 = b * kStep1Block + 4ull * (uint64_t)lane_id();
        uint64_t s = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (v0 + e < n) s += step0_weight(rec, P, v0 + e, lmax);
        s = wave_sum_u64(s);
        if (lane_id() == 0) sums[b] = s;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) sums[nblk] = 0;
}

// ---------------------------------------------------------------------------
// Degree orientation (the DAG the paper uses for clique patterns): the edge
// {v, w} is kept as v -> w iff (d(v), v) < (d(w), w), i.e. edges from the
// higher-degree end are dropped.  Rows stay in ascending id order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t orient_key(const DevGraph& g, uint32_t v) {
    return ((g.off[v + 1] - g.off[v]) << 32) | (uint64_t)v;
}

__global__ void k_orient_count(DevGraph g, uint32_t* outdeg) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    const uint64_t kv = orient_key(g, (uint32_t)v);
    uint32_t c = 0;
    for (uint64_t e = g.off[v]; e < g.off[v + 1]; ++e) c += orient_key(g, g.nbr[e]) > kv ? 1u : 0u;
    outdeg[v] = c;
}

__global__ __launch_bounds__(kScanThreads) void k_u32_tilesum(const uint32_t* in, uint64_t n, uint64_t* tile_sums) {
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint64_t s = 0;
    for (int j = 0; j < kScanItems; ++j) {
        const uint64_t v = base + (uint64_t)j * kScanThreads + threadIdx.x;
        if (v < n) s += in[v];
    }
    s = wave_sum_u64(s);
    __shared__ uint64_t ws[kScanThreads / kWave];
    if (lane_id() == 0) ws[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < kScanThreads / kWave; ++w) t += ws[w];
        tile_sums[blockIdx.x] = t;
    }
}

// out[v + 1] = in[0] + ... + in[v] (out[0] is set by the caller)
__global__ __launch_bounds__(kScanThreads) void k_u32_final(const uint32_t* in, uint64_t n, const uint64_t* tile_offs,
                                                             uint64_t* out) {
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t q[kScanItems];
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint64_t v = base + j;
        q[j] = v < n ? in[v] : 0u;
        s += q[j];
    }
    const uint64_t incl = wave_incl_scan_u64(s);
    __shared__ uint64_t wsum[kScanThreads / kWave];
    const int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint64_t wbase = 0;
    for (int j = 0; j < w; ++j) wbase += wsum[j];
    uint64_t run = tile_offs[blockIdx.x] + wbase + incl - s;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint64_t v = base + j;
        if (v < n) {
            run += q[j];
            out[v + 1] = run;
        }
    }
}

__global__ void k_orient_fill(DevGraph g, const uint64_t* off_out, uint32_t* nbr_out) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    const uint64_t kv = orient_key(g, (uint32_t)v);
    uint64_t p = off_out[v];
    for (uint64_t e = g.off[v]; e < g.off[v + 1]; ++e) {
        const uint32_t w = g.nbr[e];
        if (orient_key(g, w) > kv) nbr_out[p++] = w;
    }
}

hipError_t launch_orient_offsets(agis_ctx* ctx, const DevGraph& g, uint32_t* outdeg, uint64_t* off_out) {
    hipStream_t st = ctx->stream;
    const uint64_t n = g.n;
    const uint64_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (ctx->blocksums_cap < ntiles) {
        if (ctx->d_blocksums) (void)hipFree(ctx->d_blocksums);
        ctx->d_blocksums = nullptr;
        ctx->blocksums_cap = 0;
        hipError_t e = hipMalloc(&ctx->d_blocksums, ntiles * sizeof(uint64_t));
        if (e != hipSuccess) return e;
        ctx->blocksums_cap = ntiles;
    }
    hipError_t e = hipMemsetAsync(off_out, 0, sizeof(uint64_t), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_orient_count, dim3(grid_for(n, 256)), dim3(256), 0, st, g, outdeg);
    hipLaunchKernelGGL(k_u32_tilesum, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, outdeg, n, ctx->d_blocksums);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, ctx->d_blocksums, ntiles);
    hipLaunchKernelGGL(k_u32_final, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, outdeg, n, ctx->d_blocksums,
                       off_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Hub neighbourhood bitmaps
// ---------------------------------------------------------------------------
// per-block histogram in LDS, then one global atomic per nonzero bucket
__global__ __launch_bounds__(256) void k_degree_histogram(DevGraph g, uint32_t* hist) {
    __shared__ uint32_t h[64];
    if (threadIdx.x < 64) h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < g.n) {
        const uint64_t d = g.off[v + 1] - g.off[v];
        if (d) atomicAdd(&h[63 - __builtin_clzll(d)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 64 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

hipError_t launch_degree_histogram(const DevGraph& g, uint32_t* hist, hipStream_t stream) {
    hipError_t e = hipMemsetAsync(hist, 0, 64 * sizeof(uint32_t), stream);
    if (e != hipSuccess) return e;
    if (g.n) hipLaunchKernelGGL(k_degree_histogram, dim3(grid_for(g.n, 256)), dim3(256), 0, stream, g, hist);
    return hipGetLastError();
}

__global__ void k_hub_flags(DevGraph g, uint32_t min_deg, uint32_t* flags) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < g.n) flags[v] = (g.off[v + 1] - g.off[v]) >= min_deg ? 1u : 0u;
}

// hub_slot[v] = number of hubs before v for a hub, -1 otherwise; prefix[v + 1]
// = inclusive count (from the scan)
__global__ void k_hub_slot(const uint32_t* flags, const uint64_t* prefix, uint64_t n, int32_t* hub_slot) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) hub_slot[v] = flags[v] ? (int32_t)(prefix[v + 1] - 1) : -1;
}

hipError_t launch_hub_slots(agis_ctx* ctx, const DevGraph& g, uint32_t min_deg, uint32_t* flags, int32_t* hub_slot,
                            uint64_t* d_count) {
    hipStream_t st = ctx->stream;
    const uint64_t n = g.n;
    const uint64_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (ctx->blocksums_cap < ntiles) {
        if (ctx->d_blocksums) (void)hipFree(ctx->d_blocksums);
        ctx->d_blocksums = nullptr;
        ctx->blocksums_cap = 0;
        hipError_t e = hipMalloc(&ctx->d_blocksums, ntiles * sizeof(uint64_t));
        if (e != hipSuccess) return e;
        ctx->blocksums_cap = ntiles;
    }
    // the inclusive prefix goes to d_count[0..n] (n + 1 entries of scratch)
    hipError_t e = hipMemsetAsync(d_count, 0, sizeof(uint64_t), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hub_flags, dim3(grid_for(n, 256)), dim3(256), 0, st, g, min_deg, flags);
    hipLaunchKernelGGL(k_u32_tilesum, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, flags, n, ctx->d_blocksums);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, ctx->d_blocksums, ntiles);
    hipLaunchKernelGGL(k_u32_final, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, flags, n, ctx->d_blocksums,
                       d_count);
    hipLaunchKernelGGL(k_hub_slot, dim3(grid_for(n, 256)), dim3(256), 0, st, flags, d_count, n, hub_slot);
    return hipGetLastError();
}

__global__ void k_hub_bits(DevGraph g, const int32_t* hub_slot, uint64_t words, uint32_t* bits) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < g.nnz; e += stride) {
        const uint32_t v = row_of_slot(g.off, g.n, e);
        const int32_t slot = hub_slot[v];
        if (slot < 0) continue;
        const uint32_t x = g.nbr[e];
        atomicOr(&bits[(uint64_t)slot * words + (x >> 5)], 1u << (x & 31u));
    }
}

hipError_t launch_hub_bits(const DevGraph& g, const int32_t* hub_slot, uint64_t words, uint32_t* bits,
                           hipStream_t stream) {
    if (g.nnz) hipLaunchKernelGGL(k_hub_bits, dim3(stride_grid(g.nnz, 256)), dim3(256), 0, stream, g, hub_slot, words, bits);
    return hipGetLastError();
}

// Pair hubs in slot order, then one wave per pair (a, b), a < b: the
// shorter of the two lists is walked and each element probed in the other
// vertex's bitmap (every pair hub has one); both orders of the pair get
// the count, the diagonal 0.
__global__ void k_pair_hubs(const int32_t* __restrict__ pair_slot, uint64_t n, uint32_t* __restrict__ pair_hub) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && pair_slot[v] >= 0) pair_hub[pair_slot[v]] = (uint32_t)v;
}

__global__ __launch_bounds__(256) void k_pair_counts(DevGraph g, const int32_t* __restrict__ hub_slot,
                                                      const uint32_t* __restrict__ hub_bits, uint64_t hub_words,
                                                      const uint32_t* __restrict__ pair_hub, uint64_t H,
                                                      uint32_t* __restrict__ pair_count,
                                                      uint32_t* __restrict__ pair_quart) {
    const int lane = lane_id();
    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x / kWave);
    for (uint64_t pr = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; pr < H * H; pr += nw) {
        const uint64_t a = pr / H, b = pr % H;
        if (a > b) continue;  // wave-uniform
        if (a == b) {
            if (lane == 0) {
                pair_count[pr] = 0u;
                for (int j = 0; j < kPairParts - 1; ++j) pair_quart[pr * (kPairParts - 1) + j] = 0u;
            }
            continue;
        }
        const uint32_t va = pair_hub[a], vb = pair_hub[b];
        const uint64_t oa = g.off[va], ob = g.off[vb];
        const uint64_t da = g.off[va + 1] - oa, db = g.off[vb + 1] - ob;
        // walk the shorter list (by (degree, id)), probe the other's bitmap
        const bool walk_a = da < db || (da == db && va < vb);
        const uint64_t o = walk_a ? oa : ob, d = walk_a ? da : db;
        const uint32_t* bits = hub_bits + (uint64_t)hub_slot[walk_a ? vb : va] * hub_words;
        // members per part: part j holds positions [j d / P, (j + 1) d / P)
        uint32_t cp[kPairParts];
#pragma unroll
        for (int j = 0; j < kPairParts; ++j) cp[j] = 0u;
        for (uint64_t e = (uint64_t)lane; e < d; e += kWave) {
            const uint32_t x = g.nbr[o + e];
            const uint32_t m = (bits[x >> 5] >> (x & 31u)) & 1u;
            // the part of position e: the largest j with j d / P <= e
            int part = (int)((e * kPairParts) / d);
            while (part + 1 < kPairParts && (uint64_t)(part + 1) * d / kPairParts <= e) ++part;
            while (part > 0 && (uint64_t)part * d / kPairParts > e) --part;
#pragma unroll
            for (int j = 0; j < kPairParts; ++j) cp[j] += j == part ? m : 0u;
        }
        uint32_t run = 0;
        for (int j = 0; j < kPairParts; ++j) {
            const uint32_t sj = (uint32_t)wave_sum_u64(cp[j]);
            if (lane == 0 && j > 0) {
                pair_quart[(a * H + b) * (kPairParts - 1) + j - 1] = run;
                pair_quart[(b * H + a) * (kPairParts - 1) + j - 1] = run;
            }
            run += sj;
        }
        if (lane == 0) {
            pair_count[a * H + b] = run;
            pair_count[b * H + a] = run;
        }
    }
}

hipError_t launch_pair_counts(agis_ctx* ctx, const DevGraph& g, const int32_t* hub_slot, const uint32_t* hub_bits,
                              uint64_t hub_words, const int32_t* pair_slot, uint64_t H, uint32_t* pair_hub,
                              uint32_t* pair_count, uint32_t* pair_quart) {
    hipLaunchKernelGGL(k_pair_hubs, dim3(grid_for(g.n, 256)), dim3(256), 0, ctx->stream, pair_slot, g.n, pair_hub);
    const uint64_t waves = H * H;
    const uint64_t blocks = std::min<uint64_t>((waves + 3) / 4, (uint64_t)ctx->num_cus * 8);
    hipLaunchKernelGGL(k_pair_counts, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, g, hub_slot, hub_bits,
                       hub_words, pair_hub, H, pair_count, pair_quart);
    return hipGetLastError();
}

__global__ void k_pair_hub_degrees(DevGraph g, const uint32_t* __restrict__ pair_hub, uint64_t H,
                                   uint32_t* __restrict__ deg) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < H) deg[i] = (uint32_t)(g.off[pair_hub[i] + 1] - g.off[pair_hub[i]]);
}

__global__ void k_core_slots(const uint32_t* __restrict__ core_vertex, uint64_t C, int32_t* __restrict__ core_slot) {
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < C) core_slot[core_vertex[c]] = (int32_t)c;
}

// One wave per pair a < b of core slots: the shorter list (by (degree, id))
// is walked in order and its members of the other list (one bit probe of
// that vertex's hub bitmap each) are appended by ballot, so the list comes
// out ascending.
__global__ __launch_bounds__(256) void k_core_fill(DevGraph g, const int32_t* __restrict__ hub_slot,
                                                    const uint32_t* __restrict__ hub_bits, uint64_t hub_words,
                                                    const uint32_t* __restrict__ core_vertex, uint64_t C,
                                                    const uint64_t* __restrict__ core_start,
                                                    const uint32_t* __restrict__ core_len,
                                                    uint32_t* __restrict__ core_nbr) {
    const int lane = lane_id();
    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x / kWave);
    for (uint64_t pr = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; pr < C * C; pr += nw) {
        const uint64_t a = pr / C, b = pr % C;
        if (a >= b) continue;  // wave-uniform
        const uint32_t va = core_vertex[a], vb = core_vertex[b];
        const uint64_t oa = g.off[va], ob = g.off[vb];
        const uint64_t da = g.off[va + 1] - oa, db = g.off[vb + 1] - ob;
        const bool walk_a = da < db || (da == db && va < vb);
        const uint64_t o = walk_a ? oa : ob, d = walk_a ? da : db;
        const uint32_t* bits = hub_bits + (uint64_t)hub_slot[walk_a ? vb : va] * hub_words;
        uint32_t* out = core_nbr + core_start[pr];
        const uint64_t len = core_len[pr];  // the pair's range: no write beyond it
        uint64_t at = 0;
        for (uint64_t e0 = 0; e0 < d; e0 += kWave) {
            const uint64_t e = e0 + (uint64_t)lane;
            bool m = false;
            uint32_t x = 0;
            if (e < d) {
                x = g.nbr[o + e];
                m = ((bits[x >> 5] >> (x & 31u)) & 1u) != 0u;
            }
            const uint64_t bm = __ballot(m);
            const uint64_t w = at + (uint64_t)__popcll(bm & lanemask_lt());
            if (m && w < len) out[w] = x;
            at += (uint64_t)__popcll(bm);
        }
    }
}

// The pick table of one step signature over the core-pair lists, one wave
// per pair: the list's largest non-certain log weight (the normalising
// maximum over the intersection of the two backward lists), and per block
// the inclusive prefix within the list of the entries' integer weights
// against it (0 for certain zeros).  The weights themselves are not kept:
// a draw recomputes the 64 of its block from the step's weight table.
__global__ __launch_bounds__(256) void k_core_pick(const uint32_t* __restrict__ core_nbr,
                                                    const uint64_t* __restrict__ core_start,
                                                    const uint32_t* __restrict__ core_len, uint64_t C,
                                                    const int32_t* __restrict__ sw, int32_t* __restrict__ clm,
                                                    uint64_t* __restrict__ cbp) {
    const int lane = lane_id();
    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x / kWave);
    for (uint64_t pr = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; pr < C * C; pr += nw) {
        const uint64_t a = pr / C, b = pr % C;
        if (a > b) continue;  // wave-uniform; (b, a) shares the list
        const uint64_t st = core_start[pr];
        const uint64_t len = core_len[pr];
        int32_t lm = kCertainZero;
        for (uint64_t e = (uint64_t)lane; e < len; e += kWave) {
            const int32_t l = sw[core_nbr[st + e]];
            lm = l > lm ? l : lm;
        }
        lm = wave_max_i32(lm);
        if (lane == 0) {
            clm[pr] = lm;
            clm[b * C + a] = lm;
        }
        uint64_t run = 0;
        for (uint64_t e0 = 0; e0 < len; e0 += kWave) {
            const uint64_t e = e0 + (uint64_t)lane;
            uint32_t q = 0;
            if (e < len) {
                const int32_t l = sw[core_nbr[st + e]];
                q = l == kCertainZero ? 0u : weight_from_log(lm, l, c_exp2tab);
            }
            run += wave_sum_u64(q);
            if (lane == 0) cbp[(st + e0) / kCoreBlock] = run;
        }
    }
}

hipError_t launch_core_pick(agis_ctx* ctx, const agis_tables& t, const int32_t* sw, int32_t* clm, uint64_t* cbp) {
    const uint64_t C = t.cores;
    const uint64_t waves = C * C;
    const uint64_t blocks = std::min<uint64_t>((waves + 3) / 4, (uint64_t)ctx->num_cus * 8);
    hipLaunchKernelGGL(k_core_pick, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, t.core_nbr, t.core_start,
                       t.core_len, C, sw, clm, cbp);
    return hipGetLastError();
}

hipError_t launch_pair_hub_degrees(agis_ctx* ctx, const DevGraph& g, const uint32_t* pair_hub, uint64_t H,
                                   uint32_t* deg) {
    hipLaunchKernelGGL(k_pair_hub_degrees, dim3(grid_for(H, 256)), dim3(256), 0, ctx->stream, g, pair_hub, H, deg);
    return hipGetLastError();
}

hipError_t launch_core_pairs(agis_ctx* ctx, const DevGraph& g, const int32_t* hub_slot, const uint32_t* hub_bits,
                             uint64_t hub_words, const uint32_t* core_vertex, uint64_t C, int32_t* core_slot,
                             const uint64_t* core_start, const uint32_t* core_len, uint32_t* core_nbr) {
    hipLaunchKernelGGL(k_core_slots, dim3(grid_for(C, 256)), dim3(256), 0, ctx->stream, core_vertex, C, core_slot);
    const uint64_t waves = C * C;
    const uint64_t blocks = std::min<uint64_t>((waves + 3) / 4, (uint64_t)ctx->num_cus * 8);
    hipLaunchKernelGGL(k_core_fill, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, g, hub_slot, hub_bits,
                       hub_words, core_vertex, C, core_start, core_len, core_nbr);
    return hipGetLastError();
}

hipError_t launch_orient_fill(const DevGraph& g, const uint64_t* off_out, uint32_t* nbr_out, hipStream_t stream) {
    hipLaunchKernelGGL(k_orient_fill, dim3(grid_for(g.n, 256)), dim3(256), 0, stream, g, off_out, nbr_out);
    return hipGetLastError();
}

uint64_t step1_scan_tiles(uint64_t n) { return (n + kScanTile - 1) / kScanTile; }

// The block sums with a trailing 0, scanned exclusively in place: blk[b] is
// then the total of the blocks before b, so blk[0] = 0, blk[1 + b] is the
// inclusive prefix of block b and blk[nblk] the total.
hipError_t build_step1_blocks(agis_ctx* ctx, const agis_graph& g, const agis_tables& t, const DevPlan& hp,
                              uint64_t* blk, int32_t* lmax_out, uint64_t* total) {
    const uint64_t n = g.g.n;
    hipStream_t st = ctx->stream;
    int32_t* d_lmax = (int32_t*)ctx->d_small;
    const int32_t init = kCertainZero;
    hipError_t e = hipMemcpyAsync(d_lmax, &init, sizeof(init), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    const uint64_t nblk = (n + kStep1Block - 1) / kStep1Block;
    hipLaunchKernelGGL(k_step1_max, dim3(grid_for(n, 256)), dim3(256), 0, st, t.rec, hp, n, d_lmax);
    const uint64_t wg = (nblk + 3) / 4;
    hipLaunchKernelGGL(k_step1_blocksum, dim3((unsigned)(wg < kStrideBlocks ? wg : kStrideBlocks)), dim3(256), 0, st,
                       t.rec, hp, n, d_lmax, blk);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, blk, nblk + 1);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    int32_t lm = 0;
    e = hipMemcpyAsync(&lm, d_lmax, sizeof(lm), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(total, blk + nblk, sizeof(uint64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    *lmax_out = lm;
    return e;
}

hipError_t build_step1(agis_ctx* ctx, const agis_graph& g, const agis_tables& t, const DevPlan& hp, uint32_t* q1,
                       uint64_t* pre, uint64_t* total, uint64_t* blocksums) {
    const uint64_t n = g.g.n;
    hipStream_t st = ctx->stream;
    int32_t* d_lmax = (int32_t*)ctx->d_small;
    const int32_t init = kCertainZero;
    hipError_t e = hipMemcpyAsync(d_lmax, &init, sizeof(init), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    const uint64_t ntiles = step1_scan_tiles(n);
    if (!blocksums) {
        if (ctx->blocksums_cap < ntiles) {
            if (ctx->d_blocksums) (void)hipFree(ctx->d_blocksums);
            ctx->d_blocksums = nullptr;
            e = hipMalloc(&ctx->d_blocksums, ntiles * sizeof(uint64_t));
            if (e != hipSuccess) return e;
            ctx->blocksums_cap = ntiles;
        }
        blocksums = ctx->d_blocksums;
    }
    hipLaunchKernelGGL(k_step1_max, dim3(grid_for(n, 256)), dim3(256), 0, st, t.rec, hp, n, d_lmax);
    hipLaunchKernelGGL(k_step1_tilesum, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, t.rec, hp, n, d_lmax,
                       blocksums);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, blocksums, ntiles);
    hipLaunchKernelGGL(k_step1_final, dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, t.rec, hp, n, d_lmax,
                       blocksums, q1, pre);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(total, pre + (n - 1), sizeof(uint64_t), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

// Entry v owns the buckets b with pre[v - 1] <= b << shift < pre[v]
// (pre[-1] = 0): it is the first entry above each of their lower bounds.
__global__ void k_prefix_guide(const uint64_t* __restrict__ pre, uint64_t n, uint64_t buckets, uint32_t shift,
                               uint32_t* __restrict__ guide) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const uint64_t lo = v ? pre[v - 1] : 0ull, hi = pre[v];
    const uint64_t unit = 1ull << shift;
    uint64_t b = (lo + unit - 1) >> shift;      // first b with b << shift >= lo
    const uint64_t e = (hi + unit - 1) >> shift;  // first b with b << shift >= hi
    for (; b < e && b < buckets; ++b) guide[b] = (uint32_t)v;
    if (v == n - 1) guide[buckets] = (uint32_t)v;
}

uint32_t guide_shift(uint64_t total) {
    const int bits = 64 - __builtin_clzll(total);
    return bits > (int)kGuideBits ? (uint32_t)(bits - (int)kGuideBits) : 0u;
}

hipError_t launch_prefix_guide(const uint64_t* pre, uint64_t n, uint64_t total, uint32_t shift, uint32_t* guide,
                               hipStream_t stream) {
    const uint64_t buckets = ((total - 1) >> shift) + 1;
    hipLaunchKernelGGL(k_prefix_guide, dim3(grid_for(n, 256)), dim3(256), 0, stream, pre, n, buckets, shift, guide);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-row pick tables of a weighted step with one backward vertex w: its
// candidates are N(w) minus matched vertices, and the normalising maximum is
// taken over N(w), so every slot's integer weight depends on its row alone.
// The table holds, per CSR slot, the inclusive prefix of these weights
// within the slot's row (64-bit).  The log weights come from the step's
// per-vertex table sw (4 bytes per neighbour instead of its 16-byte record);
// these gathers, one cache line per slot, dominate the traffic.  Three
// kernels by row length, none with workgroup barriers on the common path:
//  - k_rowtab_short: one lane per row of degree <= kRowtabLane, the row's
//    log weights held in registers; longer rows are listed;
//  - k_rowtab_mid: one wave per listed row of degree <= kRowtabWaveRow, the
//    row's log weights in registers (slot u * 64 + lane in lane's entry u),
//    a wave scan per 64 slots;
//  - k_rowtab_long: one workgroup per longer row, which parks each slot's
//    log weight in the low half of its table entry, takes the row maximum,
//    then overwrites the entries with the prefix, 4096 slots per piece.
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t* a, uint64_t n, int32_t v) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

constexpr uint32_t kRowtabLane = 16;
constexpr uint32_t kRowtabPerLane = 16;
constexpr uint32_t kRowtabWaveRow = kWave * kRowtabPerLane;
constexpr int kRowtabThreads = 256;
constexpr int kRowtabWaves = kRowtabThreads / kWave;
constexpr int kRowtabBigItems = 16;
constexpr int kRowtabUnroll = 8;

__device__ __forceinline__ uint32_t rowtab_q(int32_t lmax, int32_t l) {
    return l == kCertainZero ? 0u : weight_from_log(lmax, l, c_exp2tab);
}

// Appends the rows of this wave whose `take` is set to list (length in *len).
__device__ __forceinline__ void wave_append(bool take, uint32_t v, uint32_t* __restrict__ list,
                                            uint32_t* __restrict__ len) {
    const uint64_t bm = __ballot(take);
    if (!bm) return;
    uint32_t at = 0;
    if (lane_id() == 0) at = atomicAdd(len, (uint32_t)__popcll(bm));
    at = (uint32_t)__shfl((int)at, 0, kWave);
    if (take) list[at + (uint32_t)__popcll(bm & lanemask_lt())] = v;
}

__global__ __launch_bounds__(kRowtabThreads) void k_rowtab_short(DevGraph g, const int32_t* __restrict__ sw,
                                                                  uint64_t* __restrict__ pre,
                                                                  uint32_t* __restrict__ mid,
                                                                  uint32_t* __restrict__ long_rows,
                                                                  uint32_t* __restrict__ counts) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // whole waves iterate together (the lists are appended wave by wave)
    const uint64_t n_up = (g.n + kWave - 1) / kWave * kWave;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n_up; v += stride) {
        const bool have = v < g.n;
        uint64_t o = 0;
        uint32_t d = 0;
        if (have) {
            o = g.off[v];
            d = (uint32_t)(g.off[v + 1] - o);
        }
        if (have && d <= kRowtabLane) {
            uint32_t x[kRowtabLane];
            int32_t l[kRowtabLane];
#pragma unroll
            for (uint32_t j = 0; j < kRowtabLane; ++j) x[j] = j < d ? g.nbr[o + j] : 0u;
            int32_t lmax = kCertainZero;
#pragma unroll
            for (uint32_t j = 0; j < kRowtabLane; ++j) {
                l[j] = j < d ? sw[x[j]] : kCertainZero;
                lmax = l[j] > lmax ? l[j] : lmax;
            }
            uint64_t run = 0;
#pragma unroll
            for (uint32_t j = 0; j < kRowtabLane; ++j)
                if (j < d) {
                    run += rowtab_q(lmax, l[j]);
                    pre[o + j] = run;
                }
        }
        wave_append(have && d > kRowtabLane && d <= kRowtabWaveRow, (uint32_t)v, mid, counts);
        wave_append(have && d > kRowtabWaveRow, (uint32_t)v, long_rows, counts + 1);
    }
}

__global__ __launch_bounds__(kRowtabThreads) void k_rowtab_mid(DevGraph g, const int32_t* __restrict__ sw,
                                                                uint64_t* __restrict__ pre,
                                                                const uint32_t* __restrict__ mid,
                                                                const uint32_t* __restrict__ counts) {
    const int lane = lane_id();
    const uint32_t m = counts[0];
    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x / kWave);
    for (uint64_t i = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; i < m; i += nw) {
        const uint64_t v = mid[i];
        const uint64_t o = g.off[v];
        const uint32_t d = (uint32_t)(g.off[v + 1] - o);
        // slot u * 64 + lane of the row in x[u], l[u]
        uint32_t x[kRowtabPerLane];
        int32_t l[kRowtabPerLane];
#pragma unroll
        for (uint32_t u = 0; u < kRowtabPerLane; ++u) {
            const uint32_t e = u * kWave + (uint32_t)lane;
            x[u] = e < d ? g.nbr[o + e] : 0u;
        }
        int32_t lm = kCertainZero;
#pragma unroll
        for (uint32_t u = 0; u < kRowtabPerLane; ++u) {
            l[u] = u * kWave + (uint32_t)lane < d ? sw[x[u]] : kCertainZero;
            lm = l[u] > lm ? l[u] : lm;
        }
        const int32_t lmax = wave_max_i32(lm);
        uint64_t carry = 0;
#pragma unroll
        for (uint32_t u = 0; u < kRowtabPerLane; ++u) {
            if (u * kWave >= d) break;
            const uint32_t e = u * kWave + (uint32_t)lane;
            const uint64_t q = e < d ? (uint64_t)rowtab_q(lmax, l[u]) : 0ull;
            const uint64_t inc = wave_incl_scan_u64(q);
            if (e < d) pre[o + e] = carry + inc;
            carry += __shfl(inc, kWave - 1, kWave);
        }
    }
}

__global__ __launch_bounds__(kRowtabThreads) void k_rowtab_long(DevGraph g, const int32_t* __restrict__ sw,
                                                                 uint64_t* __restrict__ pre,
                                                                 const uint32_t* __restrict__ long_rows,
                                                                 const uint32_t* __restrict__ counts) {
    __shared__ int32_t s_wmax[kRowtabWaves];
    __shared__ uint64_t s_wsum[kRowtabWaves];
    int32_t* park = reinterpret_cast<int32_t*>(pre);  // low half of entry e: park[2 e]
    const uint32_t m = counts[1];
    const int t = (int)threadIdx.x;
    const int lane = lane_id();
    const int wib = t / kWave;
    constexpr uint32_t kPiece = kRowtabThreads * kRowtabBigItems;
    for (uint32_t i = blockIdx.x; i < m; i += gridDim.x) {
        const uint64_t v = long_rows[i];
        const uint64_t o = g.off[v];
        const uint32_t d = (uint32_t)(g.off[v + 1] - o);
        int32_t lm = kCertainZero;
        for (uint32_t e0 = 0; e0 < d; e0 += kRowtabThreads * kRowtabUnroll) {
            uint32_t x[kRowtabUnroll];
            int32_t l[kRowtabUnroll];
#pragma unroll
            for (int u = 0; u < kRowtabUnroll; ++u) {
                const uint32_t e = e0 + (uint32_t)(u * kRowtabThreads + t);
                x[u] = e < d ? g.nbr[o + e] : 0u;
            }
#pragma unroll
            for (int u = 0; u < kRowtabUnroll; ++u)
                l[u] = e0 + (uint32_t)(u * kRowtabThreads + t) < d ? sw[x[u]] : kCertainZero;
#pragma unroll
            for (int u = 0; u < kRowtabUnroll; ++u) {
                const uint32_t e = e0 + (uint32_t)(u * kRowtabThreads + t);
                if (e < d) park[2 * (o + e)] = l[u];
                lm = l[u] > lm ? l[u] : lm;
            }
        }
        lm = wave_max_i32(lm);
        if (lane == 0) s_wmax[wib] = lm;
        __syncthreads();
        int32_t lmax = s_wmax[0];
        for (int w = 1; w < kRowtabWaves; ++w) lmax = s_wmax[w] > lmax ? s_wmax[w] : lmax;
        // pieces of kPiece slots, kRowtabBigItems consecutive ones per thread
        uint64_t carry = 0;
        for (uint32_t p0 = 0; p0 < d; p0 += kPiece) {
            const uint32_t e0 = p0 + (uint32_t)t * kRowtabBigItems;
            uint64_t q[kRowtabBigItems];
            uint64_t s = 0;
#pragma unroll
            for (int j = 0; j < kRowtabBigItems; ++j) {
                q[j] = e0 + j < d ? rowtab_q(lmax, park[2 * (o + e0 + j)]) : 0ull;
                s += q[j];
            }
            const uint64_t inc = wave_incl_scan_u64(s);
            if (lane == kWave - 1) s_wsum[wib] = inc;
            __syncthreads();
            uint64_t run = carry + inc - s;
            uint64_t piece = 0;
            for (int w = 0; w < kRowtabWaves; ++w) {
                if (w < wib) run += s_wsum[w];
                piece += s_wsum[w];
            }
#pragma unroll
            for (int j = 0; j < kRowtabBigItems; ++j) {
                run += q[j];
                if (e0 + j < d) pre[o + e0 + j] = run;
            }
            carry += piece;
            __syncthreads();  // s_wsum (and s_wmax) are rewritten next
        }
    }
}

__global__ void k_fill_u32(uint32_t* a, uint64_t n, uint32_t v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = v;
}

hipError_t launch_fill_u32(uint32_t* a, uint64_t n, uint32_t v, hipStream_t stream) {
    if (n) hipLaunchKernelGGL(k_fill_u32, dim3(stride_grid(n, 256)), dim3(256), 0, stream, a, n, v);
    return hipGetLastError();
}

hipError_t launch_rowtab(agis_ctx* ctx, const DevGraph& g, const int32_t* sw, uint64_t* pre, uint32_t* lists) {
    if (!g.n || !g.nnz) return hipSuccess;
    hipStream_t st = ctx->stream;
    // lists: the mid-length rows from the front, the long rows from n on
    // (a row is in at most one), their two lengths at 2 n
    uint32_t* mid = lists;
    uint32_t* long_rows = lists + g.n;
    uint32_t* counts = lists + 2 * g.n;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, reinterpret_cast<int32_t*>(counts), 2, 0);
    const uint64_t waves = (g.n + kWave - 1) / kWave;
    const uint64_t blocks = std::min<uint64_t>((waves + kRowtabWaves - 1) / kRowtabWaves, (uint64_t)ctx->num_cus * 8);
    hipLaunchKernelGGL(k_rowtab_short, dim3((unsigned)blocks), dim3(kRowtabThreads), 0, st, g, sw, pre, mid,
                       long_rows, counts);
    hipLaunchKernelGGL(k_rowtab_mid, dim3((unsigned)ctx->num_cus * 8), dim3(kRowtabThreads), 0, st, g, sw, pre, mid,
                       counts);
    hipLaunchKernelGGL(k_rowtab_long, dim3((unsigned)ctx->num_cus * 8), dim3(kRowtabThreads), 0, st, g, sw, pre,
                       long_rows, counts);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sampling kernel
// ---------------------------------------------------------------------------
namespace {

// |S| of a last step whose candidates are the common neighbours of the two
// matched vertices a and b (bm) minus the matched vertices, when a and b
// are both pair hubs: the table's |N(a) cap N(b)| less the other matched
// vertices found in both bitmaps (a and b lie in neither of their own
// lists).  Returns false, and leaves `out`, when either is not a pair hub.
template <class MT>
__device__ __forceinline__ bool pair_hub_count(const DevTables& t, uint32_t my_tau, uint32_t bm, uint32_t i,
                                               uint64_t& out, MT& mt) {
    const int lane = lane_id();
    const uint32_t a = readlane_u32(my_tau, __builtin_ctz(bm));
    const uint32_t b = readlane_u32(my_tau, 31 - __builtin_clz(bm));
    mt.uni(t.pair_slot + a, 4);
    mt.uni(t.pair_slot + b, 4);
    const int32_t sa = t.pair_slot[a], sb = t.pair_slot[b];
    if (sa < 0 || sb < 0) return false;
    mt.uni(t.pair_count + (uint64_t)sa * t.pairs + (uint64_t)sb, 4);
    const uint32_t c = t.pair_count[(uint64_t)sa * t.pairs + (uint64_t)sb];
    bool both = false;
    const bool probe = (uint32_t)lane < i && my_tau != a && my_tau != b;
    if constexpr (MT::kOn) {
        if (__ballot(probe)) {
            mt.uni(t.hub_slot + a, 4);
            mt.uni(t.hub_slot + b, 4);
            mt.vec(t.hub_bits + (uint64_t)t.hub_slot[a] * t.hub_words + (my_tau >> 5), 4, probe);
            mt.vec(t.hub_bits + (uint64_t)t.hub_slot[b] * t.hub_words + (my_tau >> 5), 4, probe);
        }
    }
    if (probe) {
        const auto ba = t.hub_bits + (uint64_t)t.hub_slot[a] * t.hub_words;
        const auto bb = t.hub_bits + (uint64_t)t.hub_slot[b] * t.hub_words;
        const uint32_t w = my_tau >> 5, m = 1u << (my_tau & 31u);
        both = (ba[w] & m) != 0 && (bb[w] & m) != 0;
    }
    out = (uint64_t)c - (uint64_t)__popcll(__ballot(both));
    return true;
}

// The element of rank r (ascending, 0-based) of S = (N(a) cap N(b)) minus
// the matched vertices, |S| = m, for two pair hubs a and b (bm).  The
// shorter list (by (degree, id)) is cut into kPairParts parts at positions
// j d / kPairParts; the table holds how many common neighbours lie before
// each cut, less here the matched ones (their ids are compared with the
// elements at the cuts).  The part holding rank r is walked 64 elements at
// a time, each probed in the other hub's bitmap, from its nearer end (ranks
// then counted from that end).
template <class MT>
__device__ __forceinline__ uint32_t pair_hub_select(const DevGraph& g, const DevTables& t, uint32_t my_tau, uint32_t bm,
                                                    uint32_t i, uint64_t r, uint64_t m, MT& mt) {
    const int lane = lane_id();
    const uint32_t a = readlane_u32(my_tau, __builtin_ctz(bm));
    const uint32_t b = readlane_u32(my_tau, 31 - __builtin_clz(bm));
    mt.uni(g.off + a, 16);
    mt.uni(g.off + b, 16);
    const uint64_t oa = g.off[a], ob = g.off[b];
    const uint64_t da = g.off[a + 1] - oa, db = g.off[b + 1] - ob;
    const bool walk_a = da < db || (da == db && a < b);
    const uint32_t* list = g.nbr + (walk_a ? oa : ob);
    const uint64_t d = walk_a ? da : db;
    const auto row = t.hub_bits + (uint64_t)t.hub_slot[walk_a ? b : a] * t.hub_words;
    // matched vertices (other than a and b) that lie in both lists
    bool both = false;
    const bool probe = (uint32_t)lane < i && my_tau != a && my_tau != b;
    if constexpr (MT::kOn) {
        if (__ballot(probe)) {
            mt.uni(t.hub_slot + a, 4);
            mt.uni(t.hub_slot + b, 4);
            mt.vec(t.hub_bits + (uint64_t)t.hub_slot[a] * t.hub_words + (my_tau >> 5), 4, probe);
            mt.vec(t.hub_bits + (uint64_t)t.hub_slot[b] * t.hub_words + (my_tau >> 5), 4, probe);
        }
    }
    if (probe) {
        const auto ra = t.hub_bits + (uint64_t)t.hub_slot[a] * t.hub_words;
        const auto rb = t.hub_bits + (uint64_t)t.hub_slot[b] * t.hub_words;
        const uint32_t w = my_tau >> 5, mk = 1u << (my_tau & 31u);
        both = (ra[w] & mk) != 0 && (rb[w] & mk) != 0;
    }
    // the cuts j d / P: members of S before each (the part holding rank r
    // lies between the last cut at or below r and the next)
    const auto q = t.pair_quart + ((uint64_t)t.pair_slot[a] * t.pairs + (uint64_t)t.pair_slot[b]) * (kPairParts - 1);
    uint32_t cutv[kPairParts - 1], qv[kPairParts - 1];
    mt.uni(t.pair_slot + a, 4);
    mt.uni(t.pair_slot + b, 4);
    mt.uni(q, 4 * (kPairParts - 1));
#pragma unroll
    for (int j = 1; j < kPairParts; ++j) {
        mt.uni(list + (uint64_t)j * d / kPairParts, 4);
        cutv[j - 1] = list[(uint64_t)j * d / kPairParts];
        qv[j - 1] = q[j - 1];
    }
    int s = 0;
    uint64_t lo_cnt = 0, hi_cnt = m;
#pragma unroll
    for (int j = 1; j < kPairParts; ++j) {
        const uint64_t cj = (uint64_t)qv[j - 1] - (uint64_t)__popcll(__ballot(both && my_tau < cutv[j - 1]));
        if (cj <= r) {
            s = j;
            lo_cnt = cj;
        } else {
            hi_cnt = cj;
            break;
        }
    }
    const bool forward = r - lo_cnt <= hi_cnt - 1 - r;
    const uint64_t target = forward ? r - lo_cnt : hi_cnt - 1 - r;
    const uint64_t from = (uint64_t)s * d / kPairParts, len = (uint64_t)(s + 1) * d / kPairParts - from;
    uint64_t seen = 0;
    for (uint64_t c = 0; c < len; c += kWave) {
        const uint64_t e = c + (uint64_t)lane;
        const bool valid = e < len;
        mt.vec(list + (forward ? from + e : from + len - 1 - e), 4, valid);
        const uint32_t x = valid ? list[forward ? from + e : from + len - 1 - e] : 0u;
        mt.vec(row + (x >> 5), 4, valid);
        bool keep = valid && ((row[x >> 5] >> (x & 31u)) & 1u) != 0;
        for (uint32_t j = 0; j < i; ++j) keep = keep && x != readlane_u32(my_tau, (int)j);
        uint64_t bal = __ballot(keep);
        const uint64_t n = (uint64_t)__popcll(bal);
        if (seen + n > target) {
            for (uint64_t k = target - seen; k > 0; --k) bal &= bal - 1;
            return readlane_u32(x, __builtin_ctzll(bal));
        }
        seen += n;
    }
    return 0u;  // not reached: the part holds the rank
}

// Log weight of candidate v at a weighted step: one 4-byte read of the
// step's table when it was built, else from the 16-byte vertex record.
__device__ __forceinline__ int32_t step_log_weight(const DevTables& t, const int32_t* sw, const int32_t* lt, uint32_t v,
                                                   uint32_t b, uint32_t f1, uint32_t ie, uint32_t f2) {
    if (sw) return sw[v];
    const uint4 r = t.rec[v];
    if (r.x < b + f1) return kCertainZero;
    return lt ? lt[v] : approx_log_weight(r, b, f1, ie, f2);
}

// The reads step_log_weight makes for the lanes with `active` (called by
// the whole wave).
template <class MT>
__device__ __forceinline__ void meter_step_log_weight(const DevTables& t, const int32_t* sw, const int32_t* lt,
                                                      uint32_t v, uint32_t b, uint32_t f1, bool active, MT& mt) {
    if constexpr (MT::kOn) {
        if (sw) {
            mt.vec(sw + v, 4, active);
            return;
        }
        mt.vec(t.rec + v, 16, active);
        if (lt) mt.vec(lt + v, 4, active && t.rec[active ? v : 0].x >= b + f1);
    }
}

// In-order sample: returns its weight X; lane 0 writes the record when
// rec != nullptr.  `my_tau` of lane j holds the data vertex matched at step
// j (wave-uniform by construction).  sv/sl: this wave's scratch for the
// candidate vertices and their log weights (capacity >= max degree).
// candidates per lane up to which a weighted pick keeps them in registers
constexpr int kPickBlock = 8;

// Whether the two vertices matched at the positions of bm's bits are both
// in the core; pr = their pair's index.
template <class MT>
__device__ __forceinline__ bool core_pair_of(const DevTables& t, uint32_t my_tau, uint32_t bm, uint64_t& pr, MT& mt) {
    const int lane = lane_id();
    const int ja = __builtin_ctz(bm), jb = __builtin_ctz(bm & (bm - 1u));
    const bool mine = lane == ja || lane == jb;
    mt.vec(t.core_slot + my_tau, 4, mine);
    const int32_t c = mine ? t.core_slot[my_tau] : -1;
    const int32_t ca = (int32_t)readlane_u32((uint32_t)c, ja), cb = (int32_t)readlane_u32((uint32_t)c, jb);
    if (ca < 0 || cb < 0) return false;
    pr = (uint64_t)ca * t.cores + (uint64_t)cb;
    return true;
}

// This lane's entry of block kb of a core-pair list (x; 0 past the list)
// and its integer weight against the list's largest log weight lm.
template <class MT>
__device__ __forceinline__ uint32_t core_block_q(const uint32_t* list, uint32_t len, const AGIS_GMEM int32_t* sw,
                                                 int32_t lm, uint64_t kb, uint32_t& x, MT& mt) {
    const uint64_t e = kb * kCoreBlock + (uint64_t)lane_id();
    mt.vec(list + e, 4, e < len);
    x = e < len ? list[e] : 0u;
    mt.vec(sw + x, 4, e < len);
    const int32_t l = e < len ? sw[x] : kCertainZero;
    return l == kCertainZero ? 0u : weight_from_log(lm, l, s_exp2tab);
}

// The vertices matched at step i but not backward there that lie in a
// core-pair list: lane j (one of them) gets its position, its weight and
// the list's weight before it (from the block prefixes bp).
struct CoreMatched {
    uint64_t qx, px;
    uint32_t pos, found;
};

template <class MT>
__device__ __forceinline__ CoreMatched core_matched(const uint32_t* list, uint32_t len, const AGIS_GMEM int32_t* sw,
                                                 int32_t lm, const AGIS_GMEM uint64_t* bp, uint32_t my_tau,
                                                 uint32_t bm, uint32_t i, MT& mt) {
    const int lane = lane_id();
    CoreMatched m{0, 0, 0, 0};
    const bool need = (uint32_t)lane < i && !(bm >> lane & 1u);
    bool f;
    const uint32_t pq = wave_lower_bound_keys(list, len, my_tau, need, i, f, mt);
    if (need && f) {
        m.pos = pq;
        m.found = 1;
    }
    for (uint64_t fl = __ballot(m.found != 0); fl; fl &= fl - 1) {
        const int j = __builtin_ctzll(fl);
        const uint32_t pj = readlane_u32(m.pos, j);
        const uint64_t kj = pj / kCoreBlock;
        const int o = (int)(pj % kCoreBlock);
        uint32_t xj;
        const uint32_t qj = core_block_q(list, len, sw, lm, kj, xj, mt);
        const uint64_t inc = wave_incl_scan_u64((uint64_t)qj);
        if (kj > 0) mt.uni(bp + kj - 1, 8);
        const uint64_t b0 = kj > 0 ? bp[kj - 1] : 0ull;
        const uint64_t q0 = (uint64_t)readlane_u32(qj, o);
        const uint64_t p0 = b0 + readlane_u64(inc, o) - q0;
        if (lane == j) {
            m.qx = q0;
            m.px = p0;
        }
    }
    return m;
}

template <bool kDump, bool kPairs, class MT>
__device__ __forceinline__ double sample_one(const DevGraph& g, const DevTables& t, const DevPlan* __restrict__ P,
                             uint32_t k0, uint32_t k1, uint64_t s, uint32_t* __restrict__ sv,
                             int32_t* __restrict__ sl, Record* __restrict__ rec, uint32_t hub_window, MT& mt) {
    const int lane = lane_id();
    const uint32_t c0 = (uint32_t)s, c1 = (uint32_t)(s >> 32), c2 = P->pattern_id;
    const uint32_t k = P->k;
    uint32_t my_tau = 0;
    // lane j: the row its vertex was drawn from at a single-backward step and
    // its position there (a later probe of the same row needs no search)
    uint32_t my_row = 0xFFFFFFFFu, my_rpos = 0;
    uint64_t scnt = 0;  // size of the candidate set the scratch holds
    // the previous step's candidate set when it was a core-pair list drawn
    // through its pick table (the next step starts from that list), and
    // whether that list may hold matched vertices (drawn at step 3 or later)
    const uint32_t* core_set = nullptr;
    bool core_loose = false;
    double x = 1.0;
    int fail = -1;
    uint32_t i = 0;
    for (; i < k; ++i) {
        uint64_t num, den;
        uint32_t v;
        uint32_t drawn_row = 0xFFFFFFFFu, drawn_pos = 0;
        if (i == 0) {
            if (P->weighted[0]) {
                if (P->s1_total == 0) {
                    fail = 0;
                    break;
                }
                const uint64_t r = bounded_draw(k0, k1, c0, c1, c2, 0, P->s1_total);
                if (P->s1_blk) {
                    // Blocked table: the block holding r from the block
                    // prefix (narrowed by the guide), then the block's
                    // weights recomputed from the vertex records exactly as
                    // the table was built (lane j: vertices 4j .. 4j + 3),
                    // once for the lane sums and once more for the chosen
                    // lane (no weights held across the scan).
                    const AGIS_GMEM uint64_t* blk = P->s1_blk;
                    uint64_t bk;
                    if (P->s1_guide) {
                        const uint64_t bkt = r >> P->s1_shift;
                        mt.uni(P->s1_guide + bkt, 8);
                        const uint32_t lo = P->s1_guide[bkt], hi = P->s1_guide[bkt + 1];
                        bk = lo + wave_first_greater(blk + lo, (uint64_t)(hi - lo) + 1, r, mt);
                    } else {
                        bk = wave_first_greater(blk, (g.n + kStep1Block - 1) / kStep1Block, r, mt);
                    }
                    mt.uni(blk + bk - 1, 8);
                    const uint64_t rr = r - blk[(int64_t)bk - 1];
                    const uint64_t v0 = bk * kStep1Block + 4ull * (uint64_t)lane;
                    const AGIS_GMEM int32_t* lt0 = P->lt[0];
                    mt.vec(t.rec + v0, 64, v0 < g.n);
                    if (lt0) mt.vec(lt0 + v0, 16, v0 < g.n);
                    auto q_of = [&](uint64_t vv) -> uint32_t {
                        if (vv >= g.n) return 0u;
                        const uint4 rc = t.rec[vv];
                        const uint32_t f1 = P->f1[0];
                        if (rc.x < f1) return 0u;
                        const int32_t l = lt0 ? lt0[vv] : approx_log_weight(rc, 0, f1, P->ie[0], P->f2[0]);
                        return l == kCertainZero ? 0u : weight_from_log(P->s1_lmax, l, s_exp2tab);
                    };
                    uint64_t qs = 0;
#pragma unroll
                    for (int e = 0; e < 4; ++e) qs += q_of(v0 + (uint64_t)e);
                    const uint64_t incl = wave_incl_scan_u64(qs);
                    const int L = __ffsll((unsigned long long)__ballot(incl > rr)) - 1;
                    uint64_t run = readlane_u64(incl - qs, L);
                    const uint64_t vL = bk * kStep1Block + 4ull * (uint64_t)L;
                    v = 0;
                    den = 0;
                    for (uint32_t e = 0; e < 4; ++e) {
                        const uint32_t w = q_of(vL + e);  // the same for every lane
                        if (run + w > rr) {
                            v = (uint32_t)(vL + e);
                            den = w;
                            break;
                        }
                        run += w;
                    }
                    num = P->s1_total;
                } else {
                    if (P->s1_guide) {
                        // the answer lies between the guides of r's bucket and the next
                        const uint64_t bkt = r >> P->s1_shift;
                        mt.uni(P->s1_guide + bkt, 8);
                        const uint32_t lo = P->s1_guide[bkt], hi = P->s1_guide[bkt + 1];
                        v = lo + (uint32_t)wave_first_greater(P->s1_pre + lo, (uint64_t)(hi - lo) + 1, r, mt);
                    } else {
                        v = (uint32_t)wave_first_greater(P->s1_pre, g.n, r, mt);
                    }
                    num = P->s1_total;
                    mt.uni(P->s1_q + v, 4);
                    den = P->s1_q[v];
                }
            } else {
                if (g.nnz == 0) {
                    fail = 0;
                    break;
                }
                const uint64_t r = bounded_draw(k0, k1, c0, c1, c2, 0, g.nnz);
                v = (uint32_t)wave_first_greater(g.off + 1, g.n, r, mt);
                num = g.nnz;
                mt.uni(g.off + v, 16);
                den = g.off[v + 1] - g.off[v];
            }
            x = (double)num / (double)den;
        } else {
            const uint32_t bm = P->bmask[i];
            const bool weighted = P->weighted[i] != 0;
            // At the last step only the size of a uniform draw's candidate
            // set enters X (no later step reads the vertex): the production
            // kernel counts the set and skips the draw; the record-writing
            // variant still picks the vertex.
            const bool count_only = !kDump && !weighted && i + 1 == k;
            const uint32_t* prev_core = core_set;
            const bool prev_loose = core_loose;
            core_set = nullptr;
            core_loose = false;
            uint64_t cpr = 0;
            if (weighted && P->rowpre[i] != nullptr) {
                // Weighted draw from S = N(w) minus the matched vertices
                // through the row's prefix of integer weights: subtract the
                // weights of matched vertices found in N(w), then search the
                // prefix segment by segment between their positions.
                const uint32_t w = readlane_u32(my_tau, __builtin_ctz(bm));
                mt.uni(g.off + w, 16);
                const uint64_t o = g.off[w];
                const uint32_t d = (uint32_t)(g.off[w + 1] - o);
                const uint32_t* list = g.nbr + o;
                const uint64_t* pre = P->rowpre[i] + o;  // the row's own inclusive prefix
                uint32_t pos = 0xFFFFFFFFu;
                bool found = false;
                uint64_t qx = 0;
                // w itself is matched but never in its own list (no loops);
                // a vertex drawn from this row has its position already
                const bool mine = (uint32_t)lane < i && my_tau != w;
                const bool need = mine && my_row != w;
                if (__ballot(need)) {
                    bool f;
                    const uint32_t pq = wave_lower_bound_keys(list, d, my_tau, need, i, f, mt);
                    if (need) {
                        pos = pq;
                        found = f;
                    }
                }
                if (mine && my_row == w) {
                    pos = my_rpos;
                    found = true;
                }
                if constexpr (MT::kOn) {
                    mt.vec(pre + (found && pos > 0 ? pos - 1 : pos), found && pos > 0 ? 16u : 8u, found);
                    if (d) mt.uni(pre + d - 1, 8);
                }
                if (found) qx = pre[pos] - (pos > 0 ? pre[pos - 1] : 0ull);
                const uint64_t qrow = d ? pre[d - 1] : 0ull;
                const uint64_t Q = qrow - wave_sum_u64(qx);
                if (Q == 0) {
                    fail = (int)i;
                    break;
                }
                const uint64_t r = bounded_draw(k0, k1, c0, c1, c2, i, Q);
                uint64_t shift = 0;  // weights of the matched vertices passed so far
                uint32_t seg = 0;    // start of the current segment
                uint64_t left = __ballot(found);
                uint64_t ans = ~0ull;
                while (left) {
                    uint64_t key = (left >> lane & 1ull) ? (((uint64_t)pos << 8) | (uint64_t)lane) : ~0ull;
#pragma unroll
                    for (int of = 32; of > 0; of >>= 1) {
                        const uint64_t k2 = __shfl_xor(key, of, kWave);
                        key = k2 < key ? k2 : key;
                    }
                    const int L = (int)(key & 0xFF);
                    const uint32_t e = (uint32_t)(key >> 8);
                    if (e > 0) mt.uni(pre + e - 1, 8);
                    const uint64_t before = e > 0 ? pre[e - 1] : 0ull;
                    if (before - shift > r) {
                        ans = seg + wave_first_greater(pre + seg, e - seg, r + shift, mt);
                        break;
                    }
                    shift += readlane_u64(qx, L);
                    seg = e + 1;
                    left &= ~(1ull << L);
                }
                if (ans == ~0ull) ans = seg + wave_first_greater(pre + seg, d - seg, r + shift, mt);
                if constexpr (MT::kOn) {
                    mt.uni(list + ans, 4);
                    mt.uni(pre + (ans > 0 ? ans - 1 : ans), ans > 0 ? 16u : 8u);
                }
                v = list[ans];
                drawn_row = w;
                drawn_pos = (uint32_t)ans;
                num = Q;
                den = pre[ans] - (ans > 0 ? pre[ans - 1] : 0ull);
            } else if (!weighted && __builtin_popcount(bm) == 1) {
                // Uniform draw from N(w) minus the matched vertices, without
                // materialising the set: probe each matched vertex in N(w)
                // and skip the positions found.
                const uint32_t w = readlane_u32(my_tau, __builtin_ctz(bm));
                mt.uni(g.off + w, 16);
                const uint64_t o = g.off[w];
                const uint32_t d = (uint32_t)(g.off[w + 1] - o);
                const uint32_t* list = g.nbr + o;
                uint32_t pos = 0xFFFFFFFFu;
                bool found = false;
                const bool mine = (uint32_t)lane < i && my_tau != w;  // w is never in its own list
                const bool need = mine && my_row != w;
                if (__ballot(need)) {
                    bool f;
                    const uint32_t pq = wave_lower_bound_keys(list, d, my_tau, need, i, f, mt);
                    if (need) {
                        pos = pq;
                        found = f;
                    }
                }
                if (mine && my_row == w) {
                    pos = my_rpos;
                    found = true;
                }
                const uint32_t ex = (uint32_t)__popcll(__ballot(found));
                const uint64_t m = (uint64_t)d - ex;
                if (m == 0) {
                    fail = (int)i;
                    break;
                }
                v = 0;
                if (!count_only) {
                    const uint64_t r = bounded_draw(k0, k1, c0, c1, c2, i, m);
                    uint64_t idx = r;
                    for (;;) {
                        const uint64_t c = (uint64_t)__popcll(__ballot(found && (uint64_t)pos <= idx));
                        if (r + c == idx) break;
                        idx = r + c;
                    }
                    mt.uni(list + idx, 4);
                    v = list[idx];
                    drawn_row = w;
                    drawn_pos = (uint32_t)idx;
                }
                num = m;
                den = 1;
            } else if (kPairs && count_only && t.pairs != 0 && __builtin_popcount(bm) == 2 &&
                       pair_hub_count(t, my_tau, bm, i, num, mt)) {
                // only the number of common neighbours of two pair hubs
                // enters X: one table read, less the matched vertices in
                // both lists
                if (num == 0) {
                    fail = (int)i;
                    break;
                }
                v = 0;
                den = 1;
            } else if (kPairs && !weighted && !count_only && P->reuse[i] == 0 && t.pairs != 0 &&
                       __builtin_popcount(bm) == 2 && (i + 1 == k || P->reuse[i + 1] == 0) &&
                       pair_hub_count(t, my_tau, bm, i, num, mt)) {
                // A uniform draw from the common neighbours of two pair hubs
                // (a set no later step reuses): |S| from the table, then the
                // drawn rank is found by walking from the nearer end.
                if (num == 0) {
                    fail = (int)i;
                    break;
                }
                const uint64_t r = bounded_draw(k0, k1, c0, c1, c2, i, num);
                v = pair_hub_select(g, t, my_tau, bm, i, r, num, mt);
                den = 1;
            } else if (weighted && __builtin_popcount(bm) == 2 && P->cbp[i] != nullptr && t.cores != 0 &&
                       core_pair_of(t, my_tau, bm, cpr, mt)) {
                // Two backward vertices, both in the core: I is their
                // common-neighbour list, drawn through the signature's pick
                // table over the core lists -- the block holding the rank
                // from the block prefixes, then the entry within the block,
                // whose 64 weights are recomputed from the step's weights.
                // S is I minus the matched vertices lying in it (from step 3
                // on, vertices matched earlier but not backward here): their
                // weights leave the total and the rank passes over them, as
                // over a row table.  The next step starts from the list
                // itself.
                mt.uni(t.core_start + cpr, 8);
                mt.uni(t.core_len + cpr, 4);
                mt.uni(P->clm[i] + cpr, 4);
                const uint64_t st = t.core_start[cpr];
                const uint32_t len = t.core_len[cpr];
                const int32_t lm = P->clm[i][cpr];
                const uint32_t* list = t.core_nbr + st;
                const AGIS_GMEM int32_t* swi = P->sw[i];
                const uint64_t nb = ((uint64_t)len + kCoreBlock - 1) / kCoreBlock;
                const AGIS_GMEM uint64_t* bp = P->cbp[i] + st / kCoreBlock;
                if (nb) mt.uni(bp + nb - 1, 8);
                const uint64_t qi = nb ? bp[nb - 1] : 0ull;
                if (qi == 0) {
                    fail = (int)i;
                    break;
                }
                // lane j, a matched vertex in the list: its position, its
                // weight and the list's weight before it
                CoreMatched cm{0, 0, 0, 0};
                if (i > 2) cm = core_matched(list, len, swi, lm, bp, my_tau, bm, i, mt);
                const uint32_t pos = cm.pos;
                const uint64_t qx = cm.qx, px = cm.px;
                const bool found = cm.found != 0;
                const uint64_t Q = qi - wave_sum_u64(qx);
                if (Q == 0) {
                    fail = (int)i;
                    break;
                }
                const uint64_t r = bounded_draw(k0, k1, c0, c1, c2, i, Q);
                // the rank within I: past every matched vertex at or below
                // it, in ascending order of position
                uint64_t rr = r;
                for (uint64_t left = __ballot(found); left;) {
                    uint64_t key = (left >> lane & 1ull) ? (((uint64_t)pos << 8) | (uint64_t)lane) : ~0ull;
#pragma unroll
                    for (int of = 32; of > 0; of >>= 1) {
                        const uint64_t k2 = __shfl_xor(key, of, kWave);
                        key = k2 < key ? k2 : key;
                    }
                    const int L = (int)(key & 0xFF);
                    if (rr < readlane_u64(px, L)) break;
                    rr += readlane_u64(qx, L);
                    left &= ~(1ull << L);
                }
                const uint64_t kb = wave_first_greater(bp, nb, rr, mt);
                if (kb > 0) mt.uni(bp + kb - 1, 8);
                const uint64_t before = kb > 0 ? bp[kb - 1] : 0ull;
                uint32_t xv;
                const uint32_t qv = core_block_q(list, len, swi, lm, kb, xv, mt);
                const uint64_t incl = wave_incl_scan_u64((uint64_t)qv);
                const int L = __ffsll((unsigned long long)__ballot(before + incl > rr)) - 1;
                v = readlane_u32(xv, L);
                num = Q;
                den = readlane_u32(qv, L);
                core_set = list;
                core_loose = i > 2;
                scnt = len;
            } else {
                // Candidate set I = intersection of the backward lists, S = I
                // minus the matched vertices, in ascending id order.  The
                // walk goes over a base list in chunks of 64; every other
                // list is co-iterated through a window that only moves
                // forward (see co_iterate_member).  When the previous step
                // built its candidate set in the scratch and its backward
                // set is contained in this one (every step of a clique),
                // that set (already free of the earlier matched vertices) is
                // the base and only the new backward lists are intersected.
                const bool reuse = P->reuse[i] != 0;
                const uint32_t lists = reuse ? (bm & ~P->bmask[i - 1]) : bm;
                // A long reused core list of (tau_0, tau_1) and one new
                // backward vertex: the set may be walked from a shorter core
                // list (below), which takes the lists of tau_0 and tau_1 too.
                const bool core_swap = reuse && prev_core != nullptr && t.cores != 0 && P->bmask[i - 1] == 3u &&
                                       __builtin_popcount(lists) == 1 && scnt > kCoreSwapMin;
                const uint32_t offl = lists | (core_swap ? 3u : 0u);
                uint64_t my_o = 0;
                uint32_t my_d = 0xFFFFFFFFu;
                mt.vec(g.off + my_tau, 16, (uint32_t)lane < i && (offl >> lane & 1u));
                if ((uint32_t)lane < i && (offl >> lane & 1u)) {
                    my_o = g.off[my_tau];
                    my_d = (uint32_t)(g.off[my_tau + 1] - my_o);
                }
                const uint32_t* base;
                uint32_t db;
                uint32_t others;
                // whether the base is the reused set (else it covers all of I:
                // a core list that may hold matched vertices is walked with
                // every matched vertex tested, like a fresh list)
                bool walk_reuse = reuse && !(prev_core != nullptr && prev_loose);
                if (reuse) {
                    base = prev_core ? prev_core : sv;
                    db = (uint32_t)scnt;
                    others = lists;
                    if (core_swap) {
                        // S = N(tau_0) n N(tau_1) n N(tau_n) minus the matched
                        // vertices is the same set, in the same ascending
                        // order, whichever two of the three lists are read as
                        // their common-neighbour list and walked against the
                        // third: with tau_n in the core, the shortest of the
                        // three core lists is walked.  The walk covers all of
                        // I (tau_1, say, lies in the list of tau_0 and tau_n
                        // but not in its own), so every matched vertex is
                        // tested as over a fresh list.
                        const int jn = __builtin_ctz(lists);
                        const bool cl = lane == 0 || lane == 1 || lane == jn;
                        mt.vec(t.core_slot + my_tau, 4, cl);
                        const int32_t cs = cl ? t.core_slot[my_tau] : -1;
                        const int32_t sn = (int32_t)readlane_u32((uint32_t)cs, jn);
                        if (sn >= 0) {
                            // lane 0: the list of (tau_0, tau_n); lane 1: (tau_1, tau_n)
                            const bool pl = lane < 2;
                            const uint64_t pr = (uint64_t)(pl ? cs : 0) * t.cores + (uint64_t)sn;
                            mt.vec(t.core_len + pr, 4, pl);
                            const uint32_t len = pl ? t.core_len[pr] : 0xFFFFFFFFu;
                            const uint32_t l0 = readlane_u32(len, 0), l1 = readlane_u32(len, 1);
                            const int jk = l0 <= l1 ? 0 : 1;  // the pair's matched vertex besides tau_n
                            const uint32_t lmin = jk == 0 ? l0 : l1;
                            if (lmin < db) {
                                const uint64_t prm = readlane_u64(pr, jk);
                                mt.uni(t.core_start + prm, 8);
                                base = t.core_nbr + t.core_start[prm];
                                db = lmin;
                                others = 1u << (1 - jk);
                                walk_reuse = false;
                            }
                        }
                    }
                } else {
                    // Two backward vertices of the core: start from their
                    // common-neighbour list (ascending: the set and order a
                    // walk of one list against the other would produce) and
                    // intersect only the remaining lists.
                    int32_t my_core = -1;
                    if (t.cores != 0) {
                        const bool cand = (uint32_t)lane < i && (lists >> lane & 1u);
                        mt.vec(t.core_slot + my_tau, 4, cand);
                        if (cand) my_core = t.core_slot[my_tau];
                    }
                    const uint64_t cm = __ballot(my_core >= 0);
                    if (__popcll(cm) >= 2) {
                        const int ja = __ffsll((unsigned long long)cm) - 1;
                        const int jc = __ffsll((unsigned long long)(cm & (cm - 1))) - 1;
                        const uint64_t pr = (uint64_t)readlane_u32((uint32_t)my_core, ja) * t.cores +
                                            (uint64_t)readlane_u32((uint32_t)my_core, jc);
                        mt.uni(t.core_start + pr, 8);
                        mt.uni(t.core_len + pr, 4);
                        base = t.core_nbr + t.core_start[pr];
                        db = t.core_len[pr];
                        others = uniform_u32(lists & ~(1u << ja) & ~(1u << jc));
                    } else {
                        // base = smallest degree, ties to the smallest position
                        uint64_t key = ((uint64_t)my_d << 8) | (uint64_t)lane;
#pragma unroll
                        for (int o = 32; o > 0; o >>= 1) {
                            uint64_t w2 = __shfl_xor(key, o, kWave);
                            key = w2 < key ? w2 : key;
                        }
                        const int jb = (int)(key & 0xFF);
                        base = g.nbr + readlane_u64(my_o, jb);
                        db = readlane_u32(my_d, jb);
                        others = uniform_u32(lists & ~(1u << jb));
                    }
                }
                const uint32_t b = P->b[i], f1 = P->f1[i], ie = P->ie[i], f2 = P->f2[i];
                const AGIS_GMEM int32_t* lt = P->lt[i];
                const AGIS_GMEM int32_t* sw = P->sw[i];
                const uint32_t vprev = readlane_u32(my_tau, (int)i - 1);
                int32_t lmax_l = kCertainZero;
                if constexpr (MT::kOn) {
                    const bool cand = weighted && walk_reuse && (uint32_t)lane + 1 < i && !(bm >> lane & 1u);
                    uint32_t offl = 0, loads = 0;
                    bool in_all = true;
                    if (cand) {
                        for (uint32_t bits = bm; bits && in_all; bits &= bits - 1) {
                            const uint32_t w = readlane_u32(my_tau, __builtin_ctz(bits));
                            const uint64_t o = g.off[w];
                            ++offl;
                            in_all = contains_u32_counted(g.nbr + o, (uint32_t)(g.off[w + 1] - o), my_tau, loads);
                        }
                    }
                    mt.lanes(offl, 16);
                    mt.lanes(loads, 4);
                    meter_step_log_weight(t, sw, lt, my_tau, b, f1, cand && in_all, mt);
                }
                if (weighted && walk_reuse && (uint32_t)lane + 1 < i && !(bm >> lane & 1u)) {
                    // matched vertices were dropped from the reused set; the
                    // normalising maximum still covers those lying in I (a
                    // backward vertex is not in its own list, so never in I)
                    bool in_all = true;
                    for (uint32_t bits = bm; bits && in_all; bits &= bits - 1) {
                        const uint32_t w = readlane_u32(my_tau, __builtin_ctz(bits));
                        const uint64_t o = g.off[w];
                        in_all = contains_u32(g.nbr + o, (uint32_t)(g.off[w + 1] - o), my_tau);
                    }
                    if (in_all) lmax_l = step_log_weight(t, sw, lt, my_tau, b, f1, ie, f2);
                }
                uint32_t my_pos = 0;  // lane j: window start in backward list j
                // lane j: bitmap row of backward vertex j when it is a hub
                int32_t my_slot = -1;
                mt.vec(t.hub_slot + my_tau, 4,
                       t.hub_slot && (uint32_t)lane < i && (others >> lane & 1u) &&
                           (uint64_t)my_d * kWave >= (uint64_t)hub_window * db);
                if (t.hub_slot && (uint32_t)lane < i && (others >> lane & 1u) &&
                    (uint64_t)my_d * kWave >= (uint64_t)hub_window * db)
                    my_slot = t.hub_slot[my_tau];
                uint64_t cnt = 0;
                // Software pipeline over the chunks: the next chunk's base
                // elements are loaded one chunk ahead, and a chunk's weights
                // (gathered from the step table) are stored and folded into
                // the maximum during the next chunk, so base, window and
                // weight loads of neighbouring chunks are in flight together.
                // Two register sets take turns (the loop runs chunks in
                // pairs), so no value still in flight is copied from one
                // chunk to the next: the copy would wait for its load.  A
                // chunk's largest element (xlast) is read from the prefetch
                // after the previous chunk's list loads, which the prefetch
                // preceded, have been waited for.
                // In-place compaction stays safe when base == sv: every store
                // lands below the chunk being read, and the prefetched chunk
                // lies above both.
                constexpr uint32_t kNone = 0xFFFFFFFFu;
                mt.vec(base + lane, 4, (uint32_t)lane < db);
                uint32_t xa = (uint32_t)lane < db ? base[lane] : kNone, xb = kNone;
                // (read unconditionally: every load issued so far is then
                // known to have arrived before the loop)
                uint32_t xlast_next = readlane_u32(xa, db == 0 ? 0 : (int)(db < (uint32_t)kWave ? db : (uint32_t)kWave) - 1);
                // per set: a chunk's gathered log weight (kCertainZero when
                // the candidate is not in I or the step is unweighted) and
                // the scratch slot it is stored at (kNone: not stored)
                int32_t la = kCertainZero, lb = kCertainZero;
                uint32_t pa = kNone, pb = kNone;
                auto chunk = [&](uint32_t c, uint32_t xv, uint32_t& x_next, int32_t& l_out, uint32_t& p_out,
                                 int32_t l_prev, uint32_t p_prev) {
                    const uint32_t nvalid = (db - c) < (uint32_t)kWave ? (db - c) : (uint32_t)kWave;
                    const bool valid = (uint32_t)lane < nvalid;
                    const uint32_t xlast = xlast_next;
                    const uint32_t nx = c + (uint32_t)kWave + (uint32_t)lane;
                    mt.vec(base + nx, 4, nx < db);
                    x_next = nx < db ? base[nx] : kNone;
                    bool member = valid;
                    for (uint32_t bits = others; bits; bits &= bits - 1) {
                        const int j = __builtin_ctz(bits);
                        const int32_t slot = (int32_t)readlane_u32((uint32_t)my_slot, j);
                        if (slot >= 0) {
                            // a hub's list: one bit probe per element
                            mt.vec(t.hub_bits + (uint64_t)slot * t.hub_words + (xv >> 5), 4, member);
                            if (member) {
                                // xv passes through an empty asm statement, so
                                // that the probe's address is not computed
                                // ahead of the list loop (where it would wait
                                // for the prefetch issued just before)
                                uint32_t x = xv;
                                asm volatile("" : "+v"(x));
                                const uint32_t wd = t.hub_bits[(uint64_t)slot * t.hub_words + (x >> 5)];
                                member = (wd >> (x & 31u)) & 1u;
                            }
                            continue;
                        }
                        const uint32_t* lj = g.nbr + readlane_u64(my_o, j);
                        const uint32_t dj = readlane_u32(my_d, j);
                        const uint32_t pos = readlane_u32(my_pos, j);
                        const uint32_t end = co_iterate_member(lj, pos, dj, xv, xlast, db - c, member, mt);
                        if (lane == j) my_pos = end;
                    }
                    {
                        // elements of the next chunk (none past the last)
                        const uint32_t nn = db - c > (uint32_t)kWave ? db - c - (uint32_t)kWave : 1u;
                        xlast_next = readlane_u32(x_next, (int)(nn < (uint32_t)kWave ? nn : (uint32_t)kWave) - 1);
                    }
                    // the previous chunk's weights (kCertainZero is the
                    // identity of the maximum)
                    lmax_l = l_prev > lmax_l ? l_prev : lmax_l;
                    mt.vec(sl + p_prev, 4, p_prev != kNone, true);
                    if (p_prev != kNone) sl[p_prev] = l_prev;
                    int32_t l = kCertainZero;
                    meter_step_log_weight(t, sw, lt, xv, b, f1, weighted && member, mt);
                    if (weighted && member) l = step_log_weight(t, sw, lt, xv, b, f1, ie, f2);
                    bool in_tau = false;
                    if (walk_reuse) {
                        in_tau = xv == vprev;
                    } else {
                        for (uint32_t j = 0; j < i; ++j) in_tau |= (xv == readlane_u32(my_tau, (int)j));
                    }
                    const bool keep = member && !in_tau;
                    const uint64_t km = __ballot(keep);
                    uint32_t p = kNone;
                    mt.vec(sv + (uint32_t)cnt + (uint32_t)__popcll(km & lanemask_lt()), 4, keep && !count_only, true);
                    if (keep && !count_only) {
                        p = (uint32_t)cnt + (uint32_t)__popcll(km & lanemask_lt());
                        sv[p] = xv;
                    }
                    l_out = l;
                    p_out = weighted && keep ? p : kNone;
                    cnt += (uint64_t)__popcll(km);
                };
                for (uint32_t c = 0; c < db; c += 2 * (uint32_t)kWave) {
                    chunk(c, xa, xb, la, pa, lb, pb);
                    if (c + (uint32_t)kWave >= db) break;
                    chunk(c + (uint32_t)kWave, xb, xa, lb, pb, la, pa);
                }
                // The last chunk's weights.  The other set was taken up by
                // that chunk already: storing it again writes the same value
                // and the maximum is unchanged.
                lmax_l = la > lmax_l ? la : lmax_l;
                lmax_l = lb > lmax_l ? lb : lmax_l;
                mt.vec(sl + pa, 4, pa != kNone, true);
                mt.vec(sl + pb, 4, pb != kNone, true);
                if (pa != kNone) sl[pa] = la;
                if (pb != kNone) sl[pb] = lb;
                scnt = cnt;
                __threadfence_block();
                if (!weighted) {
                    if (cnt == 0) {
                        fail = (int)i;
                        break;
                    }
                    v = 0;
                    if constexpr (MT::kOn) {
                        if (!count_only) mt.uni(sv + bounded_draw(k0, k1, c0, c1, c2, i, cnt), 4);
                    }
                    if (!count_only) v = sv[bounded_draw(k0, k1, c0, c1, c2, i, cnt)];
                    num = cnt;
                    den = 1;
                } else {
                    const int32_t lmax = (int32_t)uniform_u32((uint32_t)wave_max_i32(lmax_l));
                    // Lane l takes the consecutive candidates [l B, (l + 1) B);
                    // one scan of the 64 block sums then finds the block
                    // holding the draw, and the wave searches that block
                    // alone (candidate order is kept throughout).  Up to
                    // kPickBlock candidates per lane, a lane keeps its block's
                    // weights and vertices in registers (all its loads in
                    // flight together) and the search reads them from the
                    // chosen lane; for larger sets a lane's block is read in
                    // strides of 64 (coalesced), and the blocks are 64 wide.
                    if (cnt <= (uint64_t)kWave * kPickBlock) {
                        const uint32_t B = (uint32_t)((cnt + kWave - 1) / kWave);
                        const uint32_t b0 = (uint32_t)lane * B;
                        if constexpr (MT::kOn) {
                            const uint32_t nb = b0 < (uint32_t)cnt ? ((uint32_t)cnt - b0 < B ? (uint32_t)cnt - b0 : B) : 0u;
                            mt.vec(sl + b0, 4u * (nb ? nb : 1u), nb > 0);
                            mt.vec(sv + b0, 4u * (nb ? nb : 1u), nb > 0);
                        }
                        uint32_t wk[kPickBlock], vk[kPickBlock];
#pragma unroll
                        for (int e = 0; e < kPickBlock; ++e) {
                            const uint32_t c = b0 + (uint32_t)e;
                            wk[e] = (uint32_t)kCertainZero;
                            vk[e] = 0;
                            if ((uint32_t)e < B && c < (uint32_t)cnt) {
                                wk[e] = (uint32_t)sl[c];
                                vk[e] = sv[c];
                            }
                        }
                        uint64_t qs = 0;
#pragma unroll
                        for (int e = 0; e < kPickBlock; ++e) {
                            // decoded unconditionally (defined for any l), so
                            // that the table reads are issued together
                            const int32_t l = (int32_t)wk[e];
                            const uint32_t w = weight_from_log(lmax, l, s_exp2tab);
                            wk[e] = l == kCertainZero ? 0u : w;
                            qs += wk[e];
                        }
                        const uint64_t lincl = wave_incl_scan_u64(qs);
                        const uint64_t Q = uniform_u64(readlane_u64(lincl, kWave - 1));
                        if (Q == 0) {
                            fail = (int)i;
                            break;
                        }
                        const uint64_t r = bounded_draw(k0, k1, c0, c1, c2, i, Q);
                        const int LB = __ffsll((unsigned long long)__ballot(lincl > r)) - 1;
                        // weights before block LB: at most r, so the block's
                        // zero weights are never chosen
                        uint64_t run = readlane_u64(lincl - qs, LB);
                        v = 0;
                        den = 0;
                        bool found = false;
#pragma unroll
                        for (int e = 0; e < kPickBlock; ++e) {
                            const uint32_t w = readlane_u32(wk[e], LB);
                            const uint32_t xe = readlane_u32(vk[e], LB);
                            if (!found && run + w > r) {
                                found = true;
                                v = xe;
                                den = w;
                            }
                            run += w;
                        }
                        num = Q;
                    } else {
                        uint64_t qs = 0;
                        mt.span(sl, cnt * 4, 4 * kWave);
                        for (uint64_t c = (uint64_t)lane; c < cnt; c += kWave) {
                            const int32_t l = sl[c];
                            qs += l == kCertainZero ? 0u : weight_from_log(lmax, l, s_exp2tab);
                        }
                        const uint64_t Q = uniform_u64(wave_sum_u64(qs));
                        if (Q == 0) {
                            fail = (int)i;
                            break;
                        }
                        const uint64_t r = bounded_draw(k0, k1, c0, c1, c2, i, Q);
                        uint64_t run = 0;
                        v = 0;
                        den = 0;
                        for (uint64_t c0i = 0; c0i < cnt; c0i += kWave) {
                            const uint64_t c = c0i + (uint64_t)lane;
                            uint32_t q = 0;
                            mt.vec(sl + c, 4, c < cnt);
                            if (c < cnt) {
                                const int32_t l = sl[c];
                                q = l == kCertainZero ? 0u : weight_from_log(lmax, l, s_exp2tab);
                            }
                            const uint64_t incl = wave_incl_scan_u64((uint64_t)q);
                            const uint64_t tot = readlane_u64(incl, kWave - 1);
                            if (run + tot > r) {
                                const uint64_t hm = __ballot(run + incl > r);
                                const int L = __ffsll((unsigned long long)hm) - 1;
                                mt.uni(sv + c0i + (uint64_t)L, 4);
                                v = sv[c0i + (uint64_t)L];
                                den = readlane_u32(q, L);
                                break;
                            }
                            run += tot;
                        }
                        num = Q;
                    }
                }
            }
            num = uniform_u64(num);
            den = uniform_u64(den);
            x = x * ((double)num / (double)den);
        }
        v = uniform_u32(v);
        if ((uint32_t)lane == i) {
            my_tau = v;
            my_row = drawn_row;
            my_rpos = drawn_pos;
        }
        if (kDump && lane == 0) {
            rec->v[i] = v;
            rec->num[i] = num;
            rec->den[i] = den;
        }
    }
    if (fail >= 0) x = 0.0;
    if (kDump && lane == 0) {
        for (uint32_t j = i; j < (uint32_t)kMaxK; ++j) {
            rec->v[j] = 0;
            rec->num[j] = 0;
            rec->den[j] = 0;
        }
        rec->x = x;
        rec->steps = (int32_t)i;
        rec->fail_step = fail;
    }
    return x;
}

}  // namespace

// Chan et al.'s pairwise update, a then b, rounded as written (no fused
// multiply-adds: the host merges tiles with the same arithmetic).
__device__ __forceinline__ Partial chan_merge(Partial a, const Partial& b) {
#pragma clang fp contract(off)
    if (b.n == 0.0) return a;
    if (a.n == 0.0) return b;
    const double n = a.n + b.n;
    const double delta = b.mean - a.mean;
    a.mean = a.mean + delta * (b.n / n);
    a.m2 = a.m2 + b.m2 + delta * delta * (a.n * b.n / n);
    a.n = n;
    a.nonzero += b.nonzero;
    return a;
}

// Persistent sampler over one round: slots [0, total) are the concatenated
// segments of the round (pattern plan, first sample index, slot range).
// Each wave repeatedly takes the next `grab` slots from device-wide
// counters (so heavy and light samples balance across waves), runs them one
// at a time and stores each weight at its slot.  The next grab is requested
// before the current one is processed, so the atomic's round trip overlaps
// sampling work.  A sample's result does not depend on which wave runs it.
// kMode: kRun (production), kDumpRecords (the record-writing variant:
// index lists and records) or kMeterSamples (production paths, index lists,
// and per sample the memory requests it made: read bytes, written bytes,
// 64-byte segments, wave-level requests), compiled apart so the production
// kernel carries none of that state.  kWavesPerEU:
// register budget of the variant -- at least that many waves per SIMD must
// fit (4 leaves the compiler its own choice, 80 registers and 6 waves here;
// 7 and 8 trade spills for more resident waves); the autotuner picks the
// fastest.
template <int kMode, int kWavesPerEU, bool kPairs>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWavesPerEU)))
void k_sample(const LaunchDesc* __restrict__ D) {
    constexpr bool kDump = kMode == kDumpRecords;
    constexpr bool kIdx = kMode != kRun;
    const int lane = lane_id();
    for (uint32_t e = threadIdx.x; e < 4096u; e += blockDim.x) s_exp2tab[e] = c_exp2tab[e];
    __syncthreads();
    const uint64_t gw = (uint64_t)blockIdx.x * (blockDim.x / kWave) + uniform_u32(threadIdx.x / kWave);
    const uint64_t cap = D->cap;
    uint32_t* sv = D->scratch + gw * cap * 2;
    int32_t* sl = (int32_t*)(sv + cap);
    const RoundDesc* __restrict__ round = &D->round;
    const uint64_t total = round->total;
    const uint32_t grab = D->grab;
    const DevGraph g = D->g;
    const DevTables t = D->t;
    const uint32_t hub_window = D->hub_window;
    AGIS_GMEM double* xout = D->xout;
    // The slots are split into kQueues contiguous parts, each with its own
    // counter (atomics on one address are serialised: with cheap samples a
    // single counter bounds the launch).  A wave starts on part
    // blockIdx % kQueues and, when that part runs out, moves on to the next
    // part, until it has found every part empty.
    uint32_t q = blockIdx.x % kQueues;
    uint64_t lo = total * q / kQueues, hi = total * (q + 1) / kQueues;
    auto take = [&]() -> uint64_t {
        unsigned long long o = 0;
        if (lane == 0) o = atomicAdd(D->queue + (uint64_t)q * kQueueStride, (unsigned long long)grab);
        o = uniform_u64(o);
        return o < hi - lo ? lo + o : kNoSlot;
    };
    uint32_t sg = 0;  // segment of the current slot (within a part, slots only increase)
    uint32_t unvisited = kQueues - 1;
    uint64_t cur = take();
    for (;;) {
        while (cur == kNoSlot && unvisited > 0) {
            --unvisited;
            q = (q + 1) % kQueues;
            lo = total * q / kQueues;
            hi = total * (q + 1) / kQueues;
            sg = 0;
            cur = take();
        }
        if (cur == kNoSlot) break;
        const uint64_t next = take();  // requested before the current grab runs
        const uint64_t j1 = (cur + grab) < hi ? (cur + grab) : hi;
        for (uint64_t j = cur; j < j1; ++j) {
            while (sg + 1 < round->nseg && j >= round->seg[sg].base + round->seg[sg].count) ++sg;
            const Segment& S = round->seg[sg];
            const uint64_t off = j - S.base;
            const uint64_t sidx = kIdx ? D->idx[off] : S.start + off;
            Record* rec = kDump ? D->dump + j : nullptr;
            if constexpr (kMode == kMeterSamples) {
                Meter mt;
                const double xv = sample_one<false, kPairs>(g, t, D->plans + S.plan, round->k0, round->k1, sidx, sv,
                                                            sl, rec, hub_window, mt);
                mt.uni(xout + j, 8, true);
                if (lane == 0) {
                    xout[j] = xv;
                    D->meter[4 * j + 0] = mt.rbytes;
                    D->meter[4 * j + 1] = mt.wbytes;
                    D->meter[4 * j + 2] = mt.segs;
                    D->meter[4 * j + 3] = mt.reqs;
                }
            } else {
                NoMeter mt;
                const double xv = sample_one<kDump, kPairs>(g, t, D->plans + S.plan, round->k0, round->k1, sidx, sv,
                                                            sl, rec, hub_window, mt);
                if (lane == 0) xout[j] = xv;
            }
        }
        cur = uniform_u64(next);
    }
}

// ---------------------------------------------------------------------------
// One lane per sample
// ---------------------------------------------------------------------------
// Plans whose steps after the first are all uniform draws from the row of a
// single backward vertex (stars under switching, every tree under
// f_uniform) build no candidate set: a sample is the first-step search, one
// Philox draw and one neighbour load per step, and positions in one row.
// The wave sampler spends most of such a sample in wave-uniform (scalar)
// work; here each lane runs its own sample, so 64 samples share every
// instruction.  The draws, factors and records are those of sample_one.

// A per-lane request meter: every load of a lane counts as one request of
// its own (lanes do not share segments in this count).
struct LaneMeter {
    uint64_t rbytes = 0, wbytes = 0, segs = 0, reqs = 0;
    __device__ __forceinline__ void ld(const void* p, uint32_t width) {
        const uint64_t a = (uint64_t)(uintptr_t)p;
        rbytes += width;
        segs += ((a + width - 1) >> 6) - (a >> 6) + 1;
        reqs += 1;
    }
};
struct NoLaneMeter {
    __device__ __forceinline__ void ld(const void*, uint32_t) {}
};

// First p in [lo, hi] with a[p] > r, given a[hi] > r (one lane's binary search).
template <class T, class LM>
__device__ __forceinline__ uint64_t lane_first_greater(const T* __restrict__ a, uint64_t lo, uint64_t hi, uint64_t r,
                                                       LM& mt) {
    while (lo < hi) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        mt.ld(a + mid, sizeof(T));
        if ((uint64_t)a[mid] > r)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Whether x is in list[0, d) (ascending), and where.
template <class LM>
__device__ __forceinline__ bool lane_find(const uint32_t* __restrict__ list, uint32_t d, uint32_t x, uint32_t& pos,
                                          LM& mt) {
    uint32_t lo = 0, hi = d;
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        mt.ld(list + mid, 4);
        if (list[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo < d) {
        mt.ld(list + lo, 4);
        if (list[lo] == x) {
            pos = lo;
            return true;
        }
    }
    return false;
}

// v[j] for a lane-dependent j < kMaxK, by selects (no private-memory array).
__device__ __forceinline__ uint32_t pick_k(const uint32_t (&v)[kMaxK], uint32_t j) {
    uint32_t r = v[0];
#pragma unroll
    for (uint32_t q = 1; q < (uint32_t)kMaxK; ++q) r = j == q ? v[q] : r;
    return r;
}

template <bool kDump, class LM>
__device__ __forceinline__ double lane_sample(const DevGraph& g, const DevPlan* __restrict__ P, uint32_t k0,
                                              uint32_t k1, uint64_t s, Record* __restrict__ rec, LM& mt) {
    const uint32_t c0 = (uint32_t)s, c1 = (uint32_t)(s >> 32), c2 = P->pattern_id;
    const uint32_t k = P->k;
    // per matched vertex: the vertex, the row it was drawn from (or none)
    // and its position there
    uint32_t tau[kMaxK], row[kMaxK], rpos[kMaxK];
#pragma unroll
    for (int j = 0; j < kMaxK; ++j) {
        tau[j] = 0u;
        row[j] = 0xFFFFFFFFu;
        rpos[j] = 0u;
    }
    double x = 1.0;
    int fail = -1;
    uint32_t steps = 0;
    // step 0: the weighted first-step table (through its guide) or an
    // edge-uniform slot
    {
        uint64_t num = 0, den = 1;
        uint32_t v = 0;
        bool ok = true;
        if (P->weighted[0]) {
            if (P->s1_total == 0) {
                ok = false;
            } else {
                const uint64_t r = bounded_draw(k0, k1, c0, c1, c2, 0, P->s1_total);
                uint64_t lo = 0, hi = g.n - 1;
                if (P->s1_guide) {
                    const uint64_t bkt = r >> P->s1_shift;
                    mt.ld(P->s1_guide + bkt, 8);
                    lo = P->s1_guide[bkt];
                    hi = P->s1_guide[bkt + 1];
                }
                v = (uint32_t)lane_first_greater(P->s1_pre, lo, hi, r, mt);
                num = P->s1_total;
                mt.ld(P->s1_q + v, 4);
                den = P->s1_q[v];
            }
        } else {
            if (g.nnz == 0) {
                ok = false;
            } else {
                const uint64_t r = bounded_draw(k0, k1, c0, c1, c2, 0, g.nnz);
                v = (uint32_t)lane_first_greater(g.off + 1, 0, g.n - 1, r, mt);
                num = g.nnz;
                mt.ld(g.off + v, 16);
                den = g.off[v + 1] - g.off[v];
            }
        }
        if (!ok) {
            fail = 0;
        } else {
            x = (double)num / (double)den;
            tau[0] = v;
            steps = 1;
            if (kDump) {
                rec->v[0] = v;
                rec->num[0] = num;
                rec->den[0] = den;
            }
        }
    }
#pragma unroll
    for (uint32_t i = 1; i < (uint32_t)kMaxK; ++i) {
        if (fail >= 0 || i >= k) break;
        // uniform draw from N(w) minus the matched vertices
        const uint32_t bslot = (uint32_t)__builtin_ctz((uint32_t)P->bmask[i]);
        const uint32_t w = pick_k(tau, bslot);
        mt.ld(g.off + w, 16);
        const uint64_t o = g.off[w];
        const uint32_t d = (uint32_t)(g.off[w + 1] - o);
        const uint32_t* list = g.nbr + o;
        bool found[kMaxK];
        uint32_t pos[kMaxK];
        uint32_t ex = 0;
#pragma unroll
        for (uint32_t j = 0; j < (uint32_t)kMaxK; ++j) {
            found[j] = false;
            pos[j] = 0u;
            // w itself is matched but never in its own list (no loops)
            if (j < i && tau[j] != w) {
                if (row[j] == w) {
                    pos[j] = rpos[j];
                    found[j] = true;
                } else {
                    found[j] = lane_find(list, d, tau[j], pos[j], mt);
                }
                ex += found[j] ? 1u : 0u;
            }
        }
        const uint64_t m = (uint64_t)d - ex;
        if (m == 0) {
            fail = (int)i;
            break;
        }
        // at the last step only |S| enters X (see sample_one)
        const bool count_only = !kDump && i + 1 == k;
        uint32_t v = 0;
        if (!count_only) {
            const uint64_t r = bounded_draw(k0, k1, c0, c1, c2, i, m);
            // the r-th position of the row that holds no matched vertex
            uint64_t idx = r;
            for (;;) {
                uint64_t c = 0;
#pragma unroll
                for (uint32_t j = 0; j < (uint32_t)kMaxK; ++j) c += (found[j] && (uint64_t)pos[j] <= idx) ? 1u : 0u;
                if (r + c == idx) break;
                idx = r + c;
            }
            mt.ld(list + idx, 4);
            v = list[idx];
#pragma unroll
            for (uint32_t j = 0; j < (uint32_t)kMaxK; ++j)
                if (j == i) {
                    tau[j] = v;
                    row[j] = w;
                    rpos[j] = (uint32_t)idx;
                }
        }
        x = x * ((double)m / (double)1ull);
        steps = i + 1;
        if (kDump) {
            rec->v[i] = v;
            rec->num[i] = m;
            rec->den[i] = 1;
        }
    }
    if (fail >= 0) x = 0.0;
    if (kDump) {
        const uint32_t first = fail >= 0 ? (uint32_t)fail : steps;
        for (uint32_t j = first; j < (uint32_t)kMaxK; ++j) {
            rec->v[j] = 0;
            rec->num[j] = 0;
            rec->den[j] = 0;
        }
        rec->x = x;
        rec->steps = (int32_t)(fail >= 0 ? (uint32_t)fail : steps);
        rec->fail_step = fail;
    }
    return x;
}

// Persistent lane sampler over one round (slots and segments as k_sample's):
// a wave takes 64 x grab consecutive slots per queue access, lane l runs
// slots cur + l, cur + 64 + l, ...
template <int kMode>
__global__ __launch_bounds__(256) void k_sample_lanes(const LaunchDesc* __restrict__ D) {
    constexpr bool kDump = kMode == kDumpRecords;
    constexpr bool kIdx = kMode != kRun;
    const int lane = lane_id();
    const RoundDesc* __restrict__ round = &D->round;
    const uint64_t total = round->total;
    const uint64_t span = (uint64_t)D->grab * kWave;
    const DevGraph g = D->g;
    AGIS_GMEM double* xout = D->xout;
    uint32_t q = blockIdx.x % kQueues;
    uint64_t lo = total * q / kQueues, hi = total * (q + 1) / kQueues;
    auto take = [&]() -> uint64_t {
        unsigned long long o = 0;
        if (lane == 0) o = atomicAdd(D->queue + (uint64_t)q * kQueueStride, (unsigned long long)span);
        o = uniform_u64(o);
        return o < hi - lo ? lo + o : kNoSlot;
    };
    uint32_t sg = 0;  // this lane's segment (within a part, a lane's slots only increase)
    uint32_t unvisited = kQueues - 1;
    uint64_t cur = take();
    for (;;) {
        while (cur == kNoSlot && unvisited > 0) {
            --unvisited;
            q = (q + 1) % kQueues;
            lo = total * q / kQueues;
            hi = total * (q + 1) / kQueues;
            sg = 0;
            cur = take();
        }
        if (cur == kNoSlot) break;
        const uint64_t next = take();
        const uint64_t j1 = (cur + span) < hi ? (cur + span) : hi;
        for (uint64_t j = cur + (uint64_t)lane; j < j1; j += kWave) {
            while (sg + 1 < round->nseg && j >= round->seg[sg].base + round->seg[sg].count) ++sg;
            const Segment& S = round->seg[sg];
            const uint64_t off = j - S.base;
            const uint64_t sidx = kIdx ? D->idx[off] : S.start + off;
            Record* rec = kDump ? D->dump + j : nullptr;
            if constexpr (kMode == kMeterSamples) {
                LaneMeter mt;
                const double xv = lane_sample<false>(g, D->plans + S.plan, round->k0, round->k1, sidx, rec, mt);
                xout[j] = xv;
                D->meter[4 * j + 0] = mt.rbytes;
                D->meter[4 * j + 1] = mt.wbytes + 8;
                D->meter[4 * j + 2] = mt.segs + 1;
                D->meter[4 * j + 3] = mt.reqs + 1;
            } else {
                NoLaneMeter mt;
                xout[j] = lane_sample<kDump>(g, D->plans + S.plan, round->k0, round->k1, sidx, rec, mt);
            }
        }
        cur = uniform_u64(next);
    }
}

// Welford over the (up to) kReducePer weights xs[first ..] below lim, as one
// thread of the fixed reduction tree.
constexpr int kReducePer = 8;
__device__ __forceinline__ Partial welford8(const double* __restrict__ xs, uint64_t first, uint64_t lim) {
#pragma clang fp contract(off)
    Partial a{0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j < kReducePer; ++j) {
        const uint64_t p = first + j;
        if (p >= lim) break;
        const double x = xs[p];
        a.n += 1.0;
        const double d = x - a.mean;
        a.mean += d / a.n;
        a.m2 += d * (x - a.mean);
        a.nonzero += x != 0.0 ? 1.0 : 0.0;
    }
    return a;
}

// Estimator statistics of a round's weights in a fixed order: each segment
// is cut into tiles of kReduceTile consecutive slots; threads run Welford
// over 8 consecutive weights, then merge pairwise in a fixed tree.  The
// result depends only on the weights and the segment lengths, not on the
// launch that produced the weights.
constexpr int kReduceThreads = 256;
constexpr int kReduceTile = kReducePer * kReduceThreads;
static_assert(kReduceTile == kReduceTileSamples, "tile size");

__global__ __launch_bounds__(kReduceThreads) void k_reduce_x(const LaunchDesc* __restrict__ D,
                                                              Partial* __restrict__ tiles) {
    const RoundDesc* __restrict__ round = &D->round;
    const double* __restrict__ xs = D->xout;
    const uint32_t nseg = round->nseg;
    if (nseg == 0 || blockIdx.x >= round->seg[nseg - 1].tile_base + round->seg[nseg - 1].ntiles) return;
    uint32_t sg = 0;
    while (sg + 1 < nseg && blockIdx.x >= round->seg[sg + 1].tile_base) ++sg;
    const Segment& S = round->seg[sg];
    const uint64_t t0 = (uint64_t)(blockIdx.x - S.tile_base) * kReduceTile;
    const uint64_t lim = S.count;
    const uint64_t first = t0 + (uint64_t)threadIdx.x * kReducePer;
    Partial a = welford8(xs + S.base, first, lim);
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        Partial b;
        b.n = __shfl_xor(a.n, o, kWave);
        b.mean = __shfl_xor(a.mean, o, kWave);
        b.m2 = __shfl_xor(a.m2, o, kWave);
        b.nonzero = __shfl_xor(a.nonzero, o, kWave);
        if ((lane & o) == 0) a = chan_merge(a, b);  // lower lane keeps (lower, upper)
    }
    __shared__ Partial wp[kReduceThreads / kWave];
    if (lane == 0) wp[threadIdx.x / kWave] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial r = wp[0];
        for (int w = 1; w < kReduceThreads / kWave; ++w) r = chan_merge(r, wp[w]);
        tiles[blockIdx.x] = r;
    }
}

__global__ void k_zero_queues(unsigned long long* p) {
    if (threadIdx.x < kQueues) p[threadIdx.x * kQueueStride] = 0ull;
}

// ---------------------------------------------------------------------------
// Run to epsilon in one persistent launch
// ---------------------------------------------------------------------------
// Reads and writes of run state shared by all waves go to memory at device
// scope (bypassing the caches of the other XCDs).
__device__ __forceinline__ unsigned long long ld_dev(const AGIS_GMEM unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_dev(const AGIS_GMEM uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(AGIS_GMEM unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(AGIS_GMEM uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Statistics of one tile (len <= kEpsTile weights from xs) by one wave, in
// the fixed tree of k_reduce_x: 256 "threads" of 8 consecutive weights
// (lane l plays thread 64 w + l in pass w), a butterfly per 64 threads, the
// four results merged in order.  Every lane returns the result.
__device__ __forceinline__ Partial reduce_tile_wave(const AGIS_GMEM double* xs, uint64_t len) {
    const int lane = lane_id();
    Partial r{0.0, 0.0, 0.0, 0.0};
    for (int w = 0; w < kReduceThreads / kWave; ++w) {
        const uint64_t first = ((uint64_t)w * kWave + (uint64_t)lane) * kReducePer;
        Partial a = welford8((const double*)xs, first, len);
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            Partial b;
            b.n = __shfl_xor(a.n, o, kWave);
            b.mean = __shfl_xor(a.mean, o, kWave);
            b.m2 = __shfl_xor(a.m2, o, kWave);
            b.nonzero = __shfl_xor(a.nonzero, o, kWave);
            if ((lane & o) == 0) a = chan_merge(a, b);
        }
        Partial wp;
        wp.n = __shfl(a.n, 0, kWave);
        wp.mean = __shfl(a.mean, 0, kWave);
        wp.m2 = __shfl(a.m2, 0, kWave);
        wp.nonzero = __shfl(a.nonzero, 0, kWave);
        r = w == 0 ? wp : chan_merge(r, wp);
    }
    return r;
}

// Algorithm 1's estimated relative error of the merged statistics.
__device__ __forceinline__ double eps_hat_dev(const Partial& a, double z) {
#pragma clang fp contract(off)
    if (a.n == 0.0 || a.mean == 0.0) return __builtin_huge_val();
    const double sigma = sqrt(a.m2 > 0 ? a.m2 / a.n : 0.0);
    return z * sigma / (sqrt(a.n) * fabs(a.mean));
}

// Merges the ready tiles of pattern p in order (lane 0 does the work; the
// call is made by the whole wave).  One wave at a time holds the merge
// token; a wave that finds it taken leaves, and the holder looks for newly
// ready tiles again after giving it up, so no ready tile is left behind and
// no wave ever waits for another.  At every check point (a multiple of
// check samples, or the budget) Algorithm 1 decides whether to stop; once a
// pattern has stopped (converged, budget, cancel or a fault) nothing more is
// merged into it.
__device__ void merge_ready(const EpsDesc& E, uint32_t p) {
    if (lane_id() != 0) return;
    AGIS_GMEM EpsPattern* P = E.pat + p;
    const uint64_t rtiles = E.ring_samples / kEpsTile;
    for (;;) {
        // A full fence before looking: the wave that just published a tile
        // (and fails to take the token) and the holder that just gave the
        // token up (and looks again) cannot both miss each other.
        __threadfence();
        uint64_t m = ld_dev(&P->merged);
        uint64_t tm = m / kEpsTile;
        if (ld_dev(&P->stop)) return;
        if (ld_dev(E.tile_ready + (uint64_t)p * rtiles + (tm & (rtiles - 1))) != tm + 1) return;
        if (atomicCAS(&P->owner, 0u, 1u) != 0u) return;
        __threadfence();
        Partial acc = P->acc;
        const uint64_t budget = P->budget, check = P->check;
        bool stopped = false;
        for (;;) {
            // the stop is looked at again under the token: the previous
            // holder may have stopped the pattern after this wave's first
            // look, and tiles past the stopping point (samples already
            // handed out) must not be merged
            if (ld_dev(&P->stop)) {
                stopped = true;
                break;
            }
            m = ld_dev(&P->merged);
            tm = m / kEpsTile;
            const uint64_t slot = (uint64_t)p * rtiles + (tm & (rtiles - 1));
            if (m >= budget || ld_dev(E.tile_ready + slot) != tm + 1) break;
            __threadfence();
            const Partial b = E.tile_part[slot];
            acc = chan_merge(acc, b);
            const uint64_t len = (budget - m) < kEpsTile ? (budget - m) : kEpsTile;
            m += len;
            P->acc = acc;
            __threadfence();
            st_dev(&P->merged, m);
            if (m % check == 0 || m == budget) {
                const bool conv = m >= P->min_samples && eps_hat_dev(acc, E.z) <= E.eps;
                if (conv || m == budget) {
                    if (conv) st_dev(&P->converged, 1u);
                    P->stop_clock = wall_clock64();
                    __threadfence();
                    st_dev(&P->stop, 1u);
                    stopped = true;
                    break;
                }
            }
        }
        __threadfence();
        atomicExch(&P->owner, 0u);
        if (stopped) return;
    }
}

// Persistent sampler for runs to epsilon.  Each pattern hands out its slots
// in grabs from its own counter, never beyond merged + window (a wave whose
// grab lies beyond waits for the merge: the wave holding the lowest
// unfinished slot never waits, so the merge always advances).  A wave stays
// on its pattern while that pattern hands out samples.  A sample's weight
// goes to the pattern's ring; a wave counts its finished samples into their
// tile once per tile it touched in the grab (one release, one atomic), and
// the wave that completes a tile reduces it and merges what is ready.
// Samples past a pattern's stopping point are dropped: a wave looks at the
// stop flag before each sample.  The waves leave once every pattern has
// stopped or handed out its budget; the host's cancel flag stops every
// pattern at its merged prefix.
constexpr uint32_t kWindowSpins = 1u << 22;

template <int kWavesPerEU, bool kPairs>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWavesPerEU)))
void k_sample_eps(const LaunchDesc* __restrict__ D) {
    const int lane = lane_id();
    for (uint32_t e = threadIdx.x; e < 4096u; e += blockDim.x) s_exp2tab[e] = c_exp2tab[e];
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) *D->eps.clock0 = wall_clock64();
    const uint64_t gw = (uint64_t)blockIdx.x * (blockDim.x / kWave) + uniform_u32(threadIdx.x / kWave);
    const uint64_t cap = D->cap;
    uint32_t* sv = D->scratch + gw * cap * 2;
    int32_t* sl = (int32_t*)(sv + cap);
    const DevGraph g = D->g;
    const DevTables t = D->t;
    const uint32_t hub_window = D->hub_window;
    const EpsDesc& E = D->eps;
    const uint32_t npat = E.npat;
    const uint64_t rmask = E.ring_samples - 1, rtiles = E.ring_samples / kEpsTile;
    const uint32_t grab = E.grab;
    // The waves of one XCD (workgroups are dealt to the XCDs round robin)
    // start on their own share of the patterns, so each XCD's L2 holds the
    // step tables and lists of a few patterns rather than of all of them.
    uint32_t cur = (uint32_t)(((uint64_t)(blockIdx.x % kXcds) * npat) / kXcds);
    uint32_t rounds = 0;
    // patterns this wave has seen stopped or out of samples (both final)
    uint64_t dead = npat < 64 ? ~((1ull << npat) - 1ull) : 0ull;
    bool fresh = true;  // look at every pattern before the next grab
    // Grab sizes.  Atomics on one counter are served one at a time (a few
    // million per second), so a grab is just large enough that the waves'
    // takes stay under one per 200 ns: waves x 200 ns / (the wave's last
    // sample time), and at most min(grab, max(merged / (4 x waves), first
    // check point / waves)), so the samples in flight stay about a quarter
    // of those merged (few drawn past an early stop) and a slow sample
    // holds few slots behind it (the merge is in index order).
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / kWave);
    uint64_t seen = 0;  // the current pattern's merged count, as last read
    uint64_t cost = 0;  // wall-clock ticks (10 ns) of this wave's last sample
    for (;;) {
        if (fresh || (dead >> cur & 1ull)) {
            // lane q looks at pattern q, all at once
            const uint32_t q = (uint32_t)lane;
            bool out = (dead >> q & 1ull) != 0;
            if (!out) out = ld_dev(&E.pat[q].stop) != 0u || ld_dev(&E.pat[q].next) >= E.pat[q].budget;
            dead |= __ballot(out);
            if (dead == ~0ull) break;
            const uint64_t live = ~dead;
            const uint64_t from = live & ~((1ull << cur) - 1ull);
            const uint32_t pick = (uint32_t)__builtin_ctzll(from ? from : live);
            if (pick != cur) seen = 0;
            cur = pick;
            fresh = false;
        }
        const uint32_t p = cur;
        if ((++rounds & 15u) == 0 &&
            uniform_u32(__hip_atomic_load(E.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))) {
            for (uint32_t q = (uint32_t)lane; q < npat; q += kWave) st_dev(&E.pat[q].stop, 1u);
            break;
        }
        AGIS_GMEM EpsPattern* P = E.pat + p;
        const uint64_t budget = P->budget;
        // (no stop comes before the first check point, so the samples up to
        // it are spread over all waves at once)
        const uint64_t chk = P->check;
        const uint64_t first = ((P->min_samples + chk - 1) / chk) * chk;
        const uint64_t early = (first > chk ? first : chk) / nwaves;
        uint64_t take = seen / (4 * nwaves);
        take = take > early ? take : early;
        const uint64_t need = cost ? (nwaves * 20 + cost - 1) / cost : 1;
        take = take < need ? take : need;
        take = take < 1 ? 1 : (take > grab ? grab : take);
        unsigned long long s0 = 0;
        if (lane == 0) s0 = atomicAdd(&P->next, (unsigned long long)take);
        s0 = uniform_u64(s0);
        if (s0 >= budget) {
            dead |= 1ull << p;
            continue;
        }
        const uint64_t s1 = (s0 + take) < budget ? (s0 + take) : budget;
        // wait until the whole grab is inside the window (or the pattern
        // stops); the wait is bounded all the same: past kWindowSpins the
        // wave reports a fault, stops every pattern and leaves
        bool live = true;
        {
            uint32_t spins = 0;
            for (;;) {
                if (ld_dev(&P->stop)) {
                    live = false;
                    break;
                }
                seen = ld_dev(&P->merged);
                if (s1 - 1 < seen + E.window) break;
                if (++spins > kWindowSpins) {
                    live = false;
                    if (lane == 0) {
                        st_dev(E.fault, 1u);
                        for (uint32_t q = 0; q < npat; ++q) st_dev(&E.pat[q].stop, 1u);
                    }
                    break;
                }
                // back off after a short wait: thousands of waves polling
                // one address would queue behind each other
                if (spins < 64)
                    __builtin_amdgcn_s_sleep(4);
                else
                    __builtin_amdgcn_s_sleep(32);
            }
        }
        if (!uniform_u32(live ? 1u : 0u)) {
            dead |= 1ull << p;
            continue;
        }
        // the samples of the grab, tile segment by tile segment, each
        // segment counted into its tile at once
        bool stopped = false;
        for (uint64_t j = s0; j < s1 && !stopped;) {
            const uint64_t tcur = j / kEpsTile;
            const uint64_t tend = (tcur + 1) * kEpsTile < s1 ? (tcur + 1) * kEpsTile : s1;
            uint32_t cnt = 0;
            for (; j < tend; ++j) {
                // a sample past the stopping point would be dropped: skip
                // the rest of the grab (its tiles are never merged)
                if (uniform_u32(ld_dev(&P->stop))) {
                    stopped = true;
                    break;
                }
                NoMeter mt;
                const uint64_t t0 = wall_clock64();
                const double xv = sample_one<false, kPairs>(g, t, D->plans + P->plan, D->round.k0, D->round.k1,
                                                             P->start + j, sv, sl, nullptr, hub_window, mt);
                if (lane == 0) E.ring[(uint64_t)p * E.ring_samples + (j & rmask)] = xv;
                cost = uniform_u64(wall_clock64() - t0);
                ++cnt;
            }
            if (cnt == 0) break;
            const uint64_t slot = (uint64_t)p * rtiles + (tcur & (rtiles - 1));
            uint32_t last = 0;
            if (lane == 0) {
                // one release for the weights of this segment: an acquire
                // here (a cache invalidation) in every wave would cost the
                // others their cached lists and bitmaps; the wave that
                // completes the tile acquires once for the whole tile
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                const uint64_t rem = budget - tcur * kEpsTile;
                const uint32_t len = (uint32_t)(rem < kEpsTile ? rem : kEpsTile);
                last = atomicAdd(E.tile_done + slot, cnt) + cnt == len ? 1u : 0u;
            }
            if (uniform_u32(last)) {
                __threadfence();
                const uint64_t rem = budget - tcur * kEpsTile;
                const uint64_t len = rem < kEpsTile ? rem : kEpsTile;
                const Partial part =
                    reduce_tile_wave(E.ring + (uint64_t)p * E.ring_samples + ((tcur * kEpsTile) & rmask), len);
                if (lane == 0) {
                    E.tile_done[slot] = 0u;
                    E.tile_part[slot] = part;
                    __threadfence();
                    __hip_atomic_store(E.tile_ready + slot, (unsigned long long)(tcur + 1), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
                merge_ready(E, p);
            }
        }
    }
}

template <int kW, bool kPairs>
const void* sample_eps_kernel_of() {
    return reinterpret_cast<const void*>(k_sample_eps<kW, kPairs>);
}

const void* sample_eps_kernel(int variant, bool pairs) {
    switch (variant) {
        case 1:
            return pairs ? sample_eps_kernel_of<7, true>() : sample_eps_kernel_of<7, false>();
        case 2:
            return pairs ? sample_eps_kernel_of<8, true>() : sample_eps_kernel_of<8, false>();
        default:
            return pairs ? sample_eps_kernel_of<6, true>() : sample_eps_kernel_of<6, false>();
    }
}

template <int kW, bool kPairs>
const void* sample_kernel_of(bool dump) {
    return dump ? reinterpret_cast<const void*>(k_sample<kDumpRecords, kW, kPairs>)
                : reinterpret_cast<const void*>(k_sample<kRun, kW, kPairs>);
}

bool lane_plan(const DevPlan& hp) {
    if (hp.k < 2 || hp.k > (uint32_t)kMaxK) return false;
    if (hp.weighted[0] && hp.s1_blk) return false;
    for (uint32_t i = 1; i < hp.k; ++i)
        if (hp.weighted[i] || __builtin_popcount((uint32_t)hp.bmask[i]) != 1) return false;
    return true;
}

const void* sample_lanes_kernel(bool dump, bool meter) {
    if (meter) return reinterpret_cast<const void*>(k_sample_lanes<kMeterSamples>);
    return dump ? reinterpret_cast<const void*>(k_sample_lanes<kDumpRecords>)
                : reinterpret_cast<const void*>(k_sample_lanes<kRun>);
}

const void* sample_kernel(bool dump, int variant, bool pairs, bool meter) {
    // the metering variant follows the production paths (one register
    // budget: the paths do not depend on it)
    if (meter)
        return pairs ? reinterpret_cast<const void*>(k_sample<kMeterSamples, 6, true>)
                     : reinterpret_cast<const void*>(k_sample<kMeterSamples, 6, false>);
    switch (variant) {
        case 1:
            return pairs ? sample_kernel_of<7, true>(dump) : sample_kernel_of<7, false>(dump);
        case 2:
            return pairs ? sample_kernel_of<8, true>(dump) : sample_kernel_of<8, false>(dump);
        default:
            return pairs ? sample_kernel_of<6, true>(dump) : sample_kernel_of<6, false>(dump);
    }
}

int plan_sample_launch(agis_ctx* ctx, const agis_graph& g, uint64_t max_slots, uint32_t max_segs, SampleLaunch* L,
                       std::string* err, Arena* arena) {
    L->threads = 256;
    // capacity >= the largest degree, rounded up to 16 entries so that every
    // wave's two scratch arrays start on a 64-byte boundary
    L->cap = ((uint64_t)g.max_deg + 1 + 15) / 16 * 16;
    const uint64_t per_wave = L->cap * 2 * sizeof(uint32_t);
    // scratch budget: half of the free device memory, within [8, 64] GiB (a
    // wave may need a whole maximum-degree list: 3.2 MB per wave at R-MAT
    // scale 24, 48 MB at scale 30, where the budget sets the number of waves)
    uint64_t budget = 8ull << 30;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) {
        const uint64_t q = (uint64_t)free_b / 2 + ctx->scratch_bytes / 2;
        budget = q < (8ull << 30) ? (8ull << 30) : (q > (64ull << 30) ? (64ull << 30) : q);
    }
    L->variant = ctx->tune_variant;
    L->hub_window = ctx->tune_hub_window;
    int& cached = L->lanes ? ctx->lanes_blocks_per_cu : ctx->sample_blocks_per_cu[L->variant * 2 + (L->pairs ? 1 : 0)];
    if (cached == 0) {
        int nb = 0;
        const void* kern = L->lanes ? sample_lanes_kernel(false, false) : sample_kernel(false, L->variant, L->pairs, false);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, L->threads, 0) != hipSuccess || nb < 1) nb = 4;
        cached = nb;
    }
    // as many waves as can be resident at once (a persistent grid), scaled
    // by the tuning fraction
    uint64_t blocks_per_cu = (uint64_t)cached;
    if (ctx->tune_blocks_per_cu > 0 && (uint64_t)ctx->tune_blocks_per_cu < blocks_per_cu)
        blocks_per_cu = (uint64_t)ctx->tune_blocks_per_cu;
    uint64_t waves = (uint64_t)ctx->num_cus * blocks_per_cu * 4;
    L->max_tiles = (max_slots + kReduceTile - 1) / kReduceTile + max_segs;
    if (arena) {
        // the round buffers first, then as many waves as the rest holds
        L->xout = (double*)arena->take(max_slots * sizeof(double));
        L->partials = (Partial*)arena->take((uint64_t)L->max_tiles * sizeof(Partial));
        if (!L->xout || !L->partials) {
            *err = "the fixed workspace cannot hold the round buffers";
            return AGIS_E_UNSUPPORTED;
        }
        budget = arena->left() > 256 ? arena->left() - 256 : 0;
    }
    if (!L->lanes && waves * per_wave > budget) waves = budget / per_wave / 4 * 4;
    if (waves < 4) {
        *err = arena ? "maximum degree too large for the fixed workspace (one workgroup's scratch does not fit)"
                     : "maximum degree too large for the sampler scratch budget";
        return AGIS_E_UNSUPPORTED;
    }
    // (a lane-sampler wave runs 64 slots at a time)
    const uint64_t need = L->lanes ? ((max_slots + kWave - 1) / kWave + 3) / 4 * 4 : (max_slots + 3) / 4 * 4;
    if (waves > need) waves = need < 4 ? 4 : need;
    L->blocks = (int)(waves / 4);
    if (ctx->tune_grab > 0) {
        L->grab = ctx->tune_grab;
    } else {
        const uint64_t per = max_slots / (waves * 32);
        L->grab = (uint32_t)(per < 1 ? 1 : (per > 8 ? 8 : per));
    }
    // the lane sampler keeps no candidate set: no scratch
    const uint64_t bytes = L->lanes ? 0 : (uint64_t)L->blocks * 4 * per_wave;
    if (arena) {
        L->scratch = bytes ? arena->take(bytes) : nullptr;
        if (bytes && !L->scratch) {
            *err = "the fixed workspace cannot hold the sampler scratch";
            return AGIS_E_UNSUPPORTED;
        }
        L->max_slots = max_slots;
        return AGIS_OK;
    }
    if (ctx->scratch_bytes < bytes) {
        if (ctx->d_scratch) (void)hipFree(ctx->d_scratch);
        ctx->d_scratch = nullptr;
        ctx->scratch_bytes = 0;
        if (hipMalloc(&ctx->d_scratch, bytes) != hipSuccess) {
            *err = "could not allocate sampler scratch";
            return AGIS_E_OOM;
        }
        ctx->scratch_bytes = bytes;
    }
    if (ctx->partials_cap < (size_t)L->max_tiles) {
        if (ctx->d_partials) (void)hipFree(ctx->d_partials);
        ctx->d_partials = nullptr;
        ctx->partials_cap = 0;
        if (hipMalloc(&ctx->d_partials, (size_t)L->max_tiles * sizeof(Partial)) != hipSuccess) {
            *err = "could not allocate partials";
            return AGIS_E_OOM;
        }
        ctx->partials_cap = (size_t)L->max_tiles;
    }
    if (ctx->xout_cap < max_slots) {
        if (ctx->d_xout) (void)hipFree(ctx->d_xout);
        ctx->d_xout = nullptr;
        ctx->xout_cap = 0;
        if (hipMalloc(&ctx->d_xout, (size_t)max_slots * sizeof(double)) != hipSuccess) {
            *err = "could not allocate the sample-weight buffer";
            return AGIS_E_OOM;
        }
        ctx->xout_cap = max_slots;
    }
    L->scratch = ctx->d_scratch;
    L->partials = ctx->d_partials;
    L->xout = ctx->d_xout;
    L->max_slots = max_slots;
    return AGIS_OK;
}

void fill_launch(agis_ctx* ctx, const SampleLaunch& L, const DevGraph& g, const DevTables& t, const uint64_t* idx,
                 Record* dump, LaunchDesc* D, uint64_t* meter) {
    D->g = g;
    D->meter = gmem(meter);
    D->t = t;
    D->plans = cmem((const DevPlan*)ctx->d_plans);
    D->idx = gmem(idx);
    D->dump = gmem(dump);
    D->scratch = gmem((uint32_t*)L.scratch);
    D->cap = L.cap;
    D->queue = gmem((unsigned long long*)((char*)ctx->d_small + kQueueOffset));
    D->xout = gmem(L.xout);
    D->grab = L.grab;
    D->hub_window = L.hub_window;
}

hipError_t launch_round(agis_ctx* ctx, hipStream_t stream, const SampleLaunch& L, hipEvent_t before,
                        hipEvent_t after) {
    unsigned long long* queue = (unsigned long long*)((char*)ctx->d_small + kQueueOffset);
    hipError_t e;
    // the counters are cleared by a kernel (the sequence may be captured in a graph)
    hipLaunchKernelGGL(k_zero_queues, dim3(1), dim3(64), 0, stream, queue);
    if (before && (e = hipEventRecord(before, stream)) != hipSuccess) return e;
    const LaunchDesc* desc = ctx->d_launch;
    void* args[] = {(void*)&desc};
    const void* kern = L.lanes ? sample_lanes_kernel(L.dump, L.meter) : sample_kernel(L.dump, L.variant, L.pairs, L.meter);
    e = hipLaunchKernel(kern, dim3((unsigned)L.blocks), dim3((unsigned)L.threads), args, 0, stream);
    if (e != hipSuccess) return e;
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (after && (e = hipEventRecord(after, stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_x, dim3((unsigned)L.max_tiles), dim3(kReduceThreads), 0, stream, ctx->d_launch,
                       L.partials);
    return hipGetLastError();
}

}  // namespace agis
