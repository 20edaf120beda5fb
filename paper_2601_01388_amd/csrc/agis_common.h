// Shared host/device definitions of the AGIS library: the random stream,
// the Q16 log2 encoding of proposal weights, and the plain structs that the
// kernels take by value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define AGIS_HD __host__ __device__ __forceinline__

namespace agis {

constexpr int kMaxK = 8;
constexpr int32_t kCertainZero = INT32_MIN;

// ---------------------------------------------------------------------------
// Philox4x32-10 block function (Salmon, Moraes, Dror, Shaw, SC'11): ten
// rounds of two 32x32->64 multiplies with a Weyl-sequence key schedule.
// ---------------------------------------------------------------------------
struct U32x4 {
    uint32_t x, y, z, w;
};

AGIS_HD void mulhilo32(uint32_t a, uint32_t b, uint32_t& hi, uint32_t& lo) {
#ifdef __HIP_DEVICE_COMPILE__
    lo = a * b;
    hi = __umulhi(a, b);
#else
    uint64_t p = (uint64_t)a * (uint64_t)b;
    hi = (uint32_t)(p >> 32);
    lo = (uint32_t)p;
#endif
}

AGIS_HD U32x4 philox4x32_10(U32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(0xD2511F53u, c.x, hi0, lo0);
        mulhilo32(0xCD9E8D57u, c.z, hi1, lo1);
        U32x4 n;
        n.x = hi1 ^ c.y ^ k0;
        n.y = lo1;
        n.z = hi0 ^ c.w ^ k1;
        n.w = lo0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// 64-bit word number `attempt` of stream (key; c0, c1, c2, tag): the Philox
// counter is (c0, c1, c2, attempt << 4 | tag) and the word is out.y:out.x.
AGIS_HD uint64_t stream_word(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag,
                             uint32_t attempt) {
    U32x4 c{c0, c1, c2, (attempt << 4) | (tag & 0xFu)};
    U32x4 o = philox4x32_10(c, k0, k1);
    return ((uint64_t)o.y << 32) | (uint64_t)o.x;
}

AGIS_HD uint64_t mul64hi(uint64_t a, uint64_t b) {
#ifdef __HIP_DEVICE_COMPILE__
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
#endif
}

// Uniform integer in [0, range) (range >= 1) by Lemire's multiply-shift with
// rejection (ACM TOMACS 2019): accept word x when the low half of x*range is
// at least 2^64 mod range, else take the next attempt of the same stream.
AGIS_HD uint64_t bounded_draw(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag,
                              uint64_t range) {
    for (uint32_t attempt = 0;; ++attempt) {
        uint64_t x = stream_word(k0, k1, c0, c1, c2, tag, attempt);
        uint64_t lo = x * range;
        // the threshold (2^64 mod range) is below range, so only a low half
        // under range needs the (slow) modulo
        if (lo >= range || lo >= (0ull - range) % range) return mul64hi(x, range);
    }
}

// ---------------------------------------------------------------------------
// Q16 log2 encoding.  log2fx(x) = (msb(x) << 16) + LOG[next 12 bits of x],
// LOG[j] = round(2^16 log2(1 + j/4096)).  A candidate with log weight l,
// when the largest log weight is lmax, gets the integer weight
// max(1, EXP[(d & 0xffff) >> 4] >> (d >> 16)) with d = lmax - l and
// EXP[j] = round(2^31 2^(-j/4096)); shifts of 32 or more give the floor 1.
// ---------------------------------------------------------------------------
AGIS_HD int32_t log2fx(uint64_t x, const int32_t* logtab) {
    int p = 63 - __builtin_clzll(x);
    uint32_t m = p >= 12 ? (uint32_t)((x >> (p - 12)) & 0xFFFu) : (uint32_t)((x << (12 - p)) & 0xFFFu);
    return (int32_t)(p << 16) + logtab[m];
}

AGIS_HD uint32_t weight_from_log(int32_t lmax, int32_t l, const uint32_t* exp2tab) {
    const uint32_t delta = (uint32_t)lmax - (uint32_t)l;
    const uint32_t sh = delta >> 16;
    const uint32_t e = exp2tab[(delta & 0xFFFFu) >> 4];  // in the table for any delta
    const uint32_t q = sh >= 32u ? 0u : (e >> sh);
    return q < 1u ? 1u : q;
}

// ---------------------------------------------------------------------------
// Structs passed to kernels by value.
// ---------------------------------------------------------------------------

// Buffers behind the pointers below are always global memory.  In device
// code the pointers carry that address space, so loads through them are
// global loads (scalar base + 32-bit vector offset) rather than FLAT loads,
// which take 64-bit vector addresses and share the wait counter of scalar
// and LDS accesses.  Host code sees ordinary pointers of the same size.
#if defined(__HIP_DEVICE_COMPILE__)
#define AGIS_GMEM __attribute__((address_space(1)))
#define AGIS_CMEM __attribute__((address_space(4)))
#else
#define AGIS_GMEM
#define AGIS_CMEM
#endif

// Host code stores ordinary pointers into these fields through gmem().
template <typename T>
AGIS_HD AGIS_GMEM T* gmem(T* p) {
    return (AGIS_GMEM T*)p;
}
template <typename T>
AGIS_HD AGIS_CMEM T* cmem(T* p) {
    return (AGIS_CMEM T*)p;
}

struct DevGraph {
    AGIS_GMEM const uint64_t* off;
    AGIS_GMEM const uint32_t* nbr;
    uint64_t n;
    uint64_t nnz;
};

// Per-vertex record: x = degree, y = LA (Q16 log2 of S2/d), z = LC (Q16
// log2 of C_v, clamped), w = unused.
struct DevTables {
    AGIS_GMEM const uint4* rec;
    // neighbourhood bitmaps of the highest-degree vertices: bit x of row
    // hub_slot[v] is set iff x is a neighbour of v (hub_slot[v] < 0: none);
    // a membership test against such a list is one probe
    AGIS_GMEM const uint32_t* hub_bits;
    AGIS_GMEM const int32_t* hub_slot;
    uint64_t hub_words;  // 32-bit words per bitmap row
    // common-neighbour counts of the "pair hubs" (the highest-degree hubs):
    // pair_count[pair_slot[a] * pairs + pair_slot[b]] = |N(a) cap N(b)|
    // (pair_slot < 0: not a pair hub; pairs = 0: no table)
    AGIS_GMEM const int32_t* pair_slot;
    AGIS_GMEM const uint32_t* pair_count;
    uint64_t pairs;
    // per pair, kPairParts - 1 entries: the common neighbours lying before
    // positions j d / kPairParts (j = 1 .. kPairParts - 1) of the walked list
    // (the shorter of the two by (degree, id))
    AGIS_GMEM const uint32_t* pair_quart;
    // the common neighbours of every pair among the "core" hubs (the
    // highest-degree pair hubs, within a memory budget): core_slot[v] >= 0
    // for a core vertex, and the list of the pair with slots (a, b), either
    // order, is core_nbr[core_start[a * cores + b] ...] of core_len[a * cores
    // + b] vertices, ascending (cores = 0: none)
    AGIS_GMEM const int32_t* core_slot;
    AGIS_GMEM const uint64_t* core_start;
    AGIS_GMEM const uint32_t* core_len;
    AGIS_GMEM const uint32_t* core_nbr;
    uint64_t cores;
};

// Every core-pair list starts on a block of this many entries.
constexpr uint64_t kCoreBlock = 64;
// A reused core list longer than this may give way to a shorter one of
// the same candidate set (three core vertices: three lists to choose from).
constexpr uint64_t kCoreSwapMin = 256;

constexpr int kPairParts = 8;

struct DevPlan {
    uint32_t k;
    uint32_t pattern_id;
    uint8_t bmask[kMaxK];
    uint8_t b[kMaxK];
    uint8_t f1[kMaxK];
    uint8_t ie[kMaxK];
    uint8_t f2[kMaxK];
    uint8_t weighted[kMaxK];  // 1: draw from integer weights; 0: uniform draw
    uint8_t reuse[kMaxK];     // 1: intersect the previous step's candidate set (see sample_one)
    AGIS_GMEM const int32_t* lt[kMaxK];  // learned log weights per step, or nullptr
    // per-vertex Q16 log weight of a weighted step that builds its candidate
    // set (certain zeros folded in), or nullptr: then the weight is computed
    // from the vertex record (and lt)
    AGIS_GMEM const int32_t* sw[kMaxK];
    // per-row inclusive prefixes of a weighted single-backward step's integer
    // weights (one entry per CSR slot), or nullptr
    AGIS_GMEM const uint64_t* rowpre[kMaxK];
    // first-step table of a weighted first step: integer weight of every
    // vertex, its inclusive prefix and the total
    AGIS_GMEM const uint32_t* s1_q;
    AGIS_GMEM const uint64_t* s1_pre;
    uint64_t s1_total;
    // guide of the prefix (or nullptr): s1_guide[b] = first v with
    // s1_pre[v] > b << s1_shift, and s1_guide[last bucket + 1] = n - 1, so a
    // draw r is searched for only between the guides of buckets r >> shift
    // and the next
    AGIS_GMEM const uint32_t* s1_guide;
    uint32_t s1_shift;
    // blocked first-step table (instead of s1_q and s1_pre): s1_blk[b] is
    // the inclusive prefix of the weights over blocks of kStep1Block
    // vertices (s1_blk[-1] is 0 and readable), the block's weights are
    // recomputed from the vertex records against the largest log weight
    // s1_lmax, and the guide indexes blocks
    int32_t s1_lmax;
    AGIS_GMEM const uint64_t* s1_blk;
    // a weighted step whose two backward vertices are in the core: the pick
    // table of its signature over the core-pair lists -- per list its
    // largest log weight (clm, indexed like core_len; kCertainZero when the
    // list has no weight), and per block of kCoreBlock entries the inclusive
    // prefix within the list of the integer weights against it (cbp, indexed
    // by entry / kCoreBlock); a block's weights are recomputed from sw at the
    // draw -- or nullptr
    AGIS_GMEM const int32_t* clm[kMaxK];
    AGIS_GMEM const uint64_t* cbp[kMaxK];
};

constexpr uint32_t kStep1Block = 256;

// One launch ("round") of the sampler covers up to kMaxSegs segments: the
// slots [base, base + count) run samples start .. start + count - 1 of
// plan `plan`; the segment's weights are reduced in tiles numbered from
// tile_base.
constexpr uint32_t kMaxSegs = 64;

// Slot-queue counters of a round: kQueues of them, kQueueStride 64-bit
// entries (256 bytes) apart, from byte kQueueOffset of the context's small
// device buffer; kNoSlot marks an empty part.
constexpr uint32_t kQueues = 8;
// XCDs of the device (MI355X: 8, each with its own L2); workgroups are dealt
// to them round robin by workgroup index
constexpr uint32_t kXcds = 8;
constexpr uint32_t kQueueStride = 32;
constexpr uint32_t kQueueOffset = 2048;
constexpr uint64_t kNoSlot = ~0ull;

struct Segment {
    uint32_t plan;
    uint32_t ntiles;
    uint64_t start;
    uint64_t base;
    uint64_t count;
    uint64_t tile_base;
};

struct RoundDesc {
    uint64_t total;  // slots in the round
    uint32_t nseg;
    uint32_t k0, k1;  // Philox key (the sampling seed)
    uint32_t pad;
    Segment seg[kMaxSegs];
};

struct Record;

// Welford/Chan accumulator of the sample weights of one workgroup.
struct Partial {
    double n;
    double mean;
    double m2;
    double nonzero;
};

// Samples per reduction tile of a run to epsilon in one launch (the tiles
// of the round-by-round path have the same size, so the statistics are
// merged from the same tiles in the same order).
constexpr uint64_t kEpsTile = 2048;

// Device state of one pattern of a run to epsilon in one persistent
// launch (the host fills the first block and zeroes the rest).
struct EpsPattern {
    // its own 128-byte line: the slot counter every wave takes grabs from
    // (kept apart from the state the waves poll, so the atomics and the
    // polls do not queue behind each other at one address)
    unsigned long long next;  // next sample slot to hand out (relative to start)
    uint64_t pad_next[15];
    uint64_t budget;       // samples at most
    uint64_t start;        // index of the first sample
    uint64_t check;        // samples between checks (a multiple of kEpsTile)
    uint64_t min_samples;  // no convergence before this many samples
    uint32_t plan;
    uint32_t pad0;
    // run state
    unsigned long long merged;  // samples whose tiles are merged, in order
    uint32_t stop;              // 1: no more samples (converged, budget reached or cancelled)
    uint32_t owner;             // merge token: 1 while a wave merges
    uint32_t converged;
    uint32_t pad1;
    Partial acc;                       // statistics of the merged samples
    unsigned long long stop_clock;     // wall clock when the pattern stopped
    uint64_t pad_state[3];
};
static_assert(sizeof(EpsPattern) == 256, "two 128-byte lines per pattern");

// The buffers of a run to epsilon in one launch: per pattern a ring of
// ring_samples weights and ring_samples / kEpsTile tiles (completed-sample
// counter, partial statistics, and the index + 1 of the tile whose partial
// is ready); slots are handed out only below merged + window.
struct EpsDesc {
    AGIS_GMEM EpsPattern* pat;
    AGIS_GMEM double* ring;
    AGIS_GMEM uint32_t* tile_done;
    AGIS_GMEM Partial* tile_part;
    AGIS_GMEM unsigned long long* tile_ready;
    const volatile uint32_t* cancel;     // pinned host flag, set by the host while the launch runs
    AGIS_GMEM uint32_t* fault;           // set by a wave whose window wait ran out
    AGIS_GMEM unsigned long long* clock0;  // wall clock at the launch's start
    uint64_t ring_samples;  // a power of two, a multiple of kEpsTile
    uint64_t window;
    uint32_t npat;
    uint32_t grab;          // slots per take from a pattern's counter
    double z;
    double eps;
};

// Sampler kernel modes: production, record-writing, request-metering.
constexpr int kRun = 0;
constexpr int kDumpRecords = 1;
constexpr int kMeterSamples = 2;

// Everything the sampling and reduction kernels of one round read, held in
// device memory (one pointer argument: the fields are fetched through the
// scalar cache where used instead of occupying registers for the whole
// kernel, and a captured graph stays valid while only the contents change).
struct LaunchDesc {
    DevGraph g;
    DevTables t;
    AGIS_CMEM const DevPlan* plans;  // read-only while a round runs: scalar loads
    AGIS_GMEM const uint64_t* idx;        // non-null: the single segment's sample indices
    AGIS_GMEM Record* dump;               // non-null: one record per slot
    AGIS_GMEM uint64_t* meter;            // metering variant: 4 counters per slot
    AGIS_GMEM uint32_t* scratch;          // per wave: cap vertices + cap log weights
    uint64_t cap;
    AGIS_GMEM unsigned long long* queue;  // kQueues counters, kQueueStride apart
    AGIS_GMEM double* xout;               // weight per slot
    EpsDesc eps;                          // run to epsilon in one launch
    uint32_t grab;
    // a hub's bitmap replaces the merge with its list when the list is at
    // least hub_window / 64 times as long as the base it is intersected with
    uint32_t hub_window;
    RoundDesc round;
};

struct Record {
    uint32_t v[kMaxK];
    uint64_t num[kMaxK];
    uint64_t den[kMaxK];
    double x;
    int32_t steps;
    int32_t fail_step;
};

}  // namespace agis
