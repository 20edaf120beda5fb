// Random-gather ceiling of the device: the rate at which waves can read
// randomly placed segments of S bytes from a buffer much larger than the
// caches.  The sampler's memory traffic is of this kind (a search probe, a
// neighbour-list window, a weight-table entry, a bitmap word per access), so
// its achieved useful bytes per second are judged against this ceiling
// rather than against the streaming peak alone.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "agis.h"
#include "agis_internal.h"

namespace agis {
namespace {

constexpr int kGatherThreads = 256;
constexpr int kGatherWave = 64;
constexpr uint64_t kSinkWords = 1024;  // 8 KiB of folded values (never read)

// 64-bit mixing function (the finaliser of SplitMix64, Steele, Lea and
// Flood, OOPSLA 2014): a counter in, a well-spread word out.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Each wave runs `rounds` rounds; in each, lane groups of L = S / 16 lanes
// (S >= 16) read one S-byte segment at a random S-aligned offset, one
// 16-byte word per lane, or (S = 4 or 8) every lane reads one item of S
// bytes at a random aligned offset.  kDep = 0: the rounds' addresses come
// from a counter (up to kIndep reads in flight per lane); kDep = 1: each
// round's address depends on the value the previous round read (a chain of
// dependent loads per group, as in the sampler's searches).  The folded
// values go to sink so no load is dead.
template <int kDep>
__global__ __launch_bounds__(kGatherThreads) void k_gather(const unsigned char* __restrict__ buf, uint64_t segments,
                                                            uint32_t seg_bytes, uint32_t rounds, uint64_t seed,
                                                            unsigned long long* __restrict__ sink) {
    const int lane = (int)__lane_id();
    const uint64_t wave = (uint64_t)blockIdx.x * (kGatherThreads / kGatherWave) + threadIdx.x / kGatherWave;
    const uint32_t per = seg_bytes >= 16 ? seg_bytes / 16 : 1;  // lanes per segment
    const uint32_t group = (uint32_t)lane / per, sub = (uint32_t)lane % per;
    uint64_t state = mix64(seed ^ (wave << 8) ^ group);
    uint64_t acc = 0;
    auto read = [&](uint64_t segment) -> uint64_t {
        const unsigned char* p = buf + segment * seg_bytes;
        if (seg_bytes >= 16) {
            const uint4 q = *reinterpret_cast<const uint4*>(p + (uint64_t)sub * 16);
            return (uint64_t)q.x ^ ((uint64_t)q.y << 7) ^ ((uint64_t)q.z << 13) ^ ((uint64_t)q.w << 21);
        }
        if (seg_bytes == 8) return *reinterpret_cast<const uint64_t*>(p);
        return *reinterpret_cast<const uint32_t*>(p);
    };
    if (kDep) {
        for (uint32_t r = 0; r < rounds; ++r) {
            const uint64_t v = read(__umul64hi(mix64(state + r), segments));
            acc += v;
            // the next address depends on the value just read
            state ^= v & 1ull;
        }
    } else {
        constexpr uint32_t kIndep = 8;
        uint32_t r = 0;
        for (; r + kIndep <= rounds; r += kIndep) {
            uint64_t v[kIndep];
#pragma unroll
            for (uint32_t u = 0; u < kIndep; ++u) v[u] = read(__umul64hi(mix64(state + r + u), segments));
#pragma unroll
            for (uint32_t u = 0; u < kIndep; ++u) acc += v[u];
        }
        for (; r < rounds; ++r) acc += read(__umul64hi(mix64(state + r), segments));
    }
    // one store per wave
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kGatherWave);
    if (lane == 0) sink[wave % kSinkWords] = acc;
}

}  // namespace
}  // namespace agis

extern "C" int agis_gather_bench(agis_ctx* ctx, const void* buffer, uint64_t bytes, uint32_t seg_bytes,
                                 int32_t dependent, uint32_t waves_per_cu, uint32_t rounds, uint64_t seed,
                                 void* sink, double* seconds, double* useful_bytes) {
    if (!ctx) return AGIS_E_INVALID_ARG;
    if (!buffer || !sink || !seconds || !useful_bytes || rounds == 0 || waves_per_cu == 0 || waves_per_cu % 4 != 0 ||
        waves_per_cu > 32) {
        ctx->err = "gather bench: null pointer, zero rounds, or waves per CU not a multiple of 4 in [4, 32]";
        return AGIS_E_INVALID_ARG;
    }
    if (!(seg_bytes == 4 || seg_bytes == 8 || seg_bytes == 16 || seg_bytes == 32 || seg_bytes == 64 ||
          seg_bytes == 128 || seg_bytes == 256 || seg_bytes == 512 || seg_bytes == 1024)) {
        ctx->err = "gather bench: segment size must be a power of two in [4, 1024]";
        return AGIS_E_INVALID_ARG;
    }
    if (((uintptr_t)buffer & 15u) != 0 || bytes < 1024) {
        ctx->err = "gather bench: the buffer must be 16-byte aligned and at least 1 KiB";
        return AGIS_E_INVALID_ARG;
    }
    hipError_t e = hipSetDevice(ctx->device);
    const uint64_t segments = bytes / seg_bytes;
    const uint32_t blocks = (uint32_t)ctx->num_cus * (waves_per_cu / 4);
    const uint64_t waves = (uint64_t)blocks * 4;
    const uint64_t bytes_per_lane_round = seg_bytes >= 16 ? 16 : seg_bytes;
    hipEvent_t a = nullptr, b = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, ctx->stream);
    if (e == hipSuccess) {
        const unsigned char* p = (const unsigned char*)buffer;
        unsigned long long* s = (unsigned long long*)sink;
        if (dependent)
            hipLaunchKernelGGL(agis::k_gather<1>, dim3(blocks), dim3(agis::kGatherThreads), 0, ctx->stream, p,
                               segments, seg_bytes, rounds, seed, s);
        else
            hipLaunchKernelGGL(agis::k_gather<0>, dim3(blocks), dim3(agis::kGatherThreads), 0, ctx->stream, p,
                               segments, seg_bytes, rounds, seed, s);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) {
        ctx->err = std::string("gather bench: ") + hipGetErrorString(e);
        return AGIS_E_HIP;
    }
    *seconds = 1e-3 * (double)ms;
    *useful_bytes = (double)waves * 64.0 * (double)rounds * (double)bytes_per_lane_round;
    return AGIS_OK;
}
