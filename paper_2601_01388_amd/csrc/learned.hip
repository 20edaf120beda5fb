// Learned proposal: per-vertex features, training targets produced by the
// sampler itself, an 8 -> 64 -> 64 -> 1 GELU MLP trained with this file's
// forward/backward kernels (FP32, deterministic reductions, Adam), and
// BF16 MFMA inference quantised into Q16 log2 pick tables that the sampler
// reads in its learned mode.
//
// Parameter layout (float[kMlpParams]): W1[64][8], b1[64], W2[64][64]
// (W2[j][i]: output j, input i), b2[64], w3[64], b3.
// Input row: the 4 vertex features (log2(1 + d), log2(1 + S2),
// log2(1 + estimated triangles), log2(1 + h-index of neighbour degrees))
// followed by a one-hot of the step's position class {1, 2, 3, >=4}.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "agis.h"
#include "agis_internal.h"

namespace agis {

constexpr int kH = 64;
constexpr int kIn = 8;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH * kIn;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kH;
constexpr int kMlpParams = kOffB3 + 1;
static_assert(kMlpParams == 4801, "parameter count");

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ float gelu(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float a) {
    return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) + a * 0.39894228040143268f * expf(-0.5f * a * a);
}

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

}  // namespace

// ---------------------------------------------------------------------------
// Features.  The h-index of the neighbour degrees -- the largest h with at
// least h neighbours of degree >= h, an upper bound of the core number --
// is found per vertex from a histogram of the neighbour degrees capped at
// the vertex's own degree d (h <= d).
//
// k_features: each wave takes 64 consecutive vertices.  The neighbour lists
// of those with d <= kLaneDeg are gathered by the whole wave as one
// concatenated list (element e belongs to the lane whose exclusive prefix
// of degrees is the last one <= e), so the loads are independent; each such
// lane then scans its histogram column from h = d down.  Vertices of larger
// degree go to a list for k_features_big.
//
// k_features_big: one workgroup per listed vertex narrows [lo, hi] (lo
// always feasible) by 256-bucket histograms of the degrees >= lo: bucket b
// holds degrees in [lo + b w, lo + (b + 1) w) with w a power of two, the
// last bucket also everything above; suffix sums give the count of degrees
// >= lo + b w, and the feasible thresholds form a prefix of the buckets.
// Three passes cover any degree below 2^24.
// ---------------------------------------------------------------------------
constexpr uint32_t kLaneDeg = 32;
constexpr int kFeatThreads = 256;
constexpr int kFeatWaves = kFeatThreads / kWave;

__device__ __forceinline__ void write_features(float* __restrict__ feats, uint64_t v, uint32_t d, uint64_t s2,
                                               uint64_t hits, uint64_t trials, uint32_t hidx) {
    const double tri = trials ? (double)hits / (double)trials * 0.5 * (double)d * (double)(d - 1) : 0.0;
    float* f = feats + v * 4;
    f[0] = (float)log2(1.0 + (double)d);
    f[1] = (float)log2(1.0 + (double)s2);
    f[2] = (float)log2(1.0 + tri);
    f[3] = (float)log2(1.0 + (double)hidx);
}

__global__ __launch_bounds__(kFeatThreads) void k_features(DevGraph g, const uint4* __restrict__ rec,
                                                           const uint64_t* __restrict__ s2,
                                                           const uint64_t* __restrict__ hits,
                                                           const uint64_t* __restrict__ trials,
                                                           float* __restrict__ feats, uint32_t* __restrict__ big,
                                                           uint32_t* __restrict__ nbig) {
    // histogram bin b of lane l of wave w: hist[w][b][l], bins 0..kLaneDeg
    __shared__ uint32_t hist[kFeatWaves][kLaneDeg + 1][kWave];
    __shared__ uint32_t s_excl[kFeatWaves][kWave];
    __shared__ uint32_t s_deg[kFeatWaves][kWave];
    __shared__ uint64_t s_off[kFeatWaves][kWave];
    const int lane = lane_id();
    const int wib = (int)threadIdx.x / kWave;
    const uint64_t groups = (g.n + kWave - 1) / kWave;
    // all waves of a workgroup run the same iterations (workgroup barriers)
    for (uint64_t gb = (uint64_t)blockIdx.x * kFeatWaves; gb < groups; gb += (uint64_t)gridDim.x * kFeatWaves) {
        const uint64_t v = (gb + (uint64_t)wib) * kWave + (uint64_t)lane;
        const bool have = v < g.n;
        uint64_t o = 0;
        uint32_t d = 0;
        if (have) {
            o = g.off[v];
            d = (uint32_t)(g.off[v + 1] - o);
        }
        const bool small = have && d <= kLaneDeg;
        const uint32_t ds = small ? d : 0u;
        uint32_t incl = ds;
#pragma unroll
        for (int sh = 1; sh < kWave; sh <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)incl, sh, kWave);
            if (lane >= sh) incl += t;
        }
        const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
        s_excl[wib][lane] = incl - ds;
        s_deg[wib][lane] = d;
        s_off[wib][lane] = o;
        for (uint32_t b = 0; b <= kLaneDeg; ++b) hist[wib][b][lane] = 0;
        __syncthreads();
        for (uint32_t e = (uint32_t)lane; e < total; e += kWave) {
            // owner: the last lane whose exclusive prefix is <= e
            int lo = 0;
#pragma unroll
            for (int step = kWave / 2; step > 0; step >>= 1)
                if (s_excl[wib][lo + step] <= e) lo += step;
            const uint32_t od = s_deg[wib][lo];
            const uint32_t nd = rec[g.nbr[s_off[wib][lo] + (e - s_excl[wib][lo])]].x;
            atomicAdd(&hist[wib][nd < od ? nd : od][lo], 1u);
        }
        __syncthreads();
        if (small) {
            uint32_t h = d, at_least = 0;
            for (; h > 0; --h) {
                at_least += hist[wib][h][lane];
                if (at_least >= h) break;
            }
            write_features(feats, v, d, s2[v], hits[v], trials[v], h);
        }
        const uint64_t bm = __ballot(have && !small);
        if (bm) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(nbig, (uint32_t)__popcll(bm));
            base = (uint32_t)__shfl((int)base, 0, kWave);
            if (have && !small) big[base + (uint32_t)__popcll(bm & ((1ull << lane) - 1ull))] = (uint32_t)v;
        }
        __syncthreads();  // the LDS of this iteration is rewritten by the next
    }
}

__global__ __launch_bounds__(kFeatThreads) void k_features_big(DevGraph g, const uint4* __restrict__ rec,
                                                               const uint64_t* __restrict__ s2,
                                                               const uint64_t* __restrict__ hits,
                                                               const uint64_t* __restrict__ trials,
                                                               float* __restrict__ feats,
                                                               const uint32_t* __restrict__ big,
                                                               const uint32_t* __restrict__ nbig) {
    __shared__ uint32_t cnt[kFeatThreads];
    const uint32_t m = *nbig;
    const int t = (int)threadIdx.x;
    for (uint32_t i = blockIdx.x; i < m; i += gridDim.x) {
        const uint64_t v = big[i];
        const uint64_t o = g.off[v];
        const uint32_t d = (uint32_t)(g.off[v + 1] - o);
        uint32_t lo = 0, hi = d;  // the h-index is in [lo, hi]; lo is feasible
        while (lo < hi) {
            const uint64_t span = (uint64_t)hi - lo + 1;
            uint32_t sh = 0;
            while (((uint64_t)kFeatThreads << sh) < (uint64_t)span) ++sh;
            cnt[t] = 0;
            __syncthreads();
            for (uint32_t e = (uint32_t)t; e < d; e += kFeatThreads) {
                const uint32_t x = rec[g.nbr[o + e]].x;
                if (x >= lo) {
                    const uint32_t b = (x - lo) >> sh;
                    atomicAdd(&cnt[b < (uint32_t)kFeatThreads ? b : (uint32_t)kFeatThreads - 1u], 1u);
                }
            }
            __syncthreads();
            // suffix sums: cnt[b] becomes the number of degrees >= lo + b w
            for (int step = 1; step < kFeatThreads; step <<= 1) {
                const uint32_t add = t + step < kFeatThreads ? cnt[t + step] : 0u;
                __syncthreads();
                cnt[t] += add;
                __syncthreads();
            }
            const uint64_t thr = (uint64_t)lo + ((uint64_t)t << sh);
            const int ok = thr <= hi && (uint64_t)cnt[t] >= thr;
            const int nok = __syncthreads_count(ok);
            const uint32_t nlo = lo + ((uint32_t)(nok - 1) << sh);
            hi = (uint32_t)min<uint64_t>((uint64_t)hi, (uint64_t)nlo + (1ull << sh) - 1ull);
            lo = nlo;
        }
        if (t == 0) write_features(feats, v, d, s2[v], hits[v], trials[v], lo);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Training targets from sample records: for a successful sample and step i,
// R_i = product of the factors num_t / den_t of the steps t > i (in FP64,
// from the last step backwards) estimates the number of successful
// extensions of the prefix v_1..v_i without bias; a sample that failed
// after step i contributes R_i = 0.  Sums and counts per (step, vertex).
// ---------------------------------------------------------------------------
__global__ void k_targets(const Record* __restrict__ recs, uint64_t m, uint32_t k, uint64_t n,
                          double* __restrict__ sums, uint32_t* __restrict__ counts) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const Record& r = recs[j];
    const int steps = r.steps;
    const bool ok = r.fail_step < 0;
    double prod = 1.0;
    for (int i = (int)k - 1; i >= 0; --i) {
        if (i < steps) {
            const double R = ok ? prod : 0.0;
            atomicAdd(&sums[(uint64_t)i * n + r.v[i]], R);
            atomicAdd(&counts[(uint64_t)i * n + r.v[i]], 1u);
        }
        if (ok && i > 0) prod = prod * ((double)r.num[i] / (double)r.den[i]);
    }
}

// ---------------------------------------------------------------------------
// Training: per tile of 64 rows, forward and backward in FP32 by a workgroup
// of four waves: lane r of every wave holds row r, and wave q computes the
// hidden units 16 q .. 16 q + 15 of both layers.  The tile's parameter
// gradient is summed over its rows in row order and written to its own
// slot; k_mlp_reduce adds the slots in tile order, so the gradient does not
// depend on scheduling.
// ---------------------------------------------------------------------------
constexpr int kTile = 64;
constexpr int kGradWaves = 4;
constexpr int kGradThreads = kTile * kGradWaves;
constexpr int kUnitsPerWave = kH / kGradWaves;
static_assert(kH == kTile, "the bias and w3 sums give unit r to lane r");

__global__ __launch_bounds__(kGradThreads) void k_mlp_grad(const float* __restrict__ params,
                                                           const float* __restrict__ feats,
                                                           const uint32_t* __restrict__ vtx,
                                                           const uint8_t* __restrict__ cls,
                                                           const float* __restrict__ target,
                                                           const float* __restrict__ weight,
                                                           const uint32_t* __restrict__ order, uint64_t rows,
                                                           float inv_wsum, float* __restrict__ partial,
                                                           float* __restrict__ loss_part) {
    // activations are stored [unit][row] with one padding column so that both
    // per-row (forward) and per-unit (gradient) walks avoid bank conflicts
    constexpr int kLd = kTile + 1;
    __shared__ float P[kMlpParams];
    __shared__ float X[kIn][kLd];
    __shared__ float H1[kH][kLd];
    __shared__ float G1[kH][kLd];  // GELU'(layer-1 pre-activation), later dL/d(pre1)
    __shared__ float H2[kH][kLd];
    __shared__ float D2[kH][kLd];  // dL/d(pre2)
    __shared__ float YP[kGradWaves][kTile];
    __shared__ float DY[kTile];
    __shared__ float LS[kTile];
    const int t = threadIdx.x;
    const int r = t % kTile;
    const int q = t / kTile;  // wave-uniform
    const int j0 = q * kUnitsPerWave;
    for (int p = t; p < kMlpParams; p += kGradThreads) P[p] = params[p];
    const uint64_t rix = (uint64_t)blockIdx.x * kTile + (uint64_t)r;
    float w = 0.0f, tgt = 0.0f;
    float x[kIn];
    for (int c = 0; c < kIn; ++c) x[c] = 0.0f;
    if (rix < rows) {
        const uint32_t ri = order ? order[rix] : (uint32_t)rix;
        const uint32_t v = vtx[ri];
        for (int c = 0; c < 4; ++c) x[c] = feats[(uint64_t)v * 4 + c];
        x[4 + (cls[ri] < 3 ? cls[ri] : 3)] = 1.0f;
        w = weight[ri];
        tgt = target[ri];
    }
    if (q == 0)
        for (int c = 0; c < kIn; ++c) X[c][r] = x[c];
    __syncthreads();
    // forward, layer 1 (this wave's units)
    for (int j = j0; j < j0 + kUnitsPerWave; ++j) {
        float a = P[kOffB1 + j];
        for (int c = 0; c < kIn; ++c) a += P[kOffW1 + j * kIn + c] * x[c];
        H1[j][r] = gelu(a);
        G1[j][r] = gelu_grad(a);
    }
    __syncthreads();
    // layer 2 and this wave's share of the output
    float yp = 0.0f;
    for (int j = j0; j < j0 + kUnitsPerWave; ++j) {
        float a = P[kOffB2 + j];
        for (int i = 0; i < kH; ++i) a += P[kOffW2 + j * kH + i] * H1[i][r];
        const float h2 = gelu(a);
        H2[j][r] = h2;
        D2[j][r] = gelu_grad(a);  // completed below once dy is known
        yp += P[kOffW3 + j] * h2;
    }
    YP[q][r] = yp;
    __syncthreads();
    float y = P[kOffB3];
    for (int qq = 0; qq < kGradWaves; ++qq) y += YP[qq][r];
    const float err = y - tgt;
    const float dy = 2.0f * w * err * inv_wsum;
    if (q == 0) {
        DY[r] = dy;
        LS[r] = w * err * err * inv_wsum;  // loss of the row (weighted squared error / total weight)
    }
    for (int j = j0; j < j0 + kUnitsPerWave; ++j) D2[j][r] *= dy * P[kOffW3 + j];
    __syncthreads();
    // back to layer 1 (this wave's units)
    for (int i = j0; i < j0 + kUnitsPerWave; ++i) {
        float sacc = 0.0f;
        for (int j = 0; j < kH; ++j) sacc += P[kOffW2 + j * kH + i] * D2[j][r];
        G1[i][r] *= sacc;  // dL/d(pre1)
    }
    __syncthreads();
    // parameter gradients of the tile, each a sum over its 64 rows in order
    float* out = partial + (uint64_t)blockIdx.x * kMlpParams;
    for (int p = t; p < kH * kH; p += kGradThreads) {
        const int j = p / kH, i = p % kH;
        float sacc = 0.0f;
        for (int rr = 0; rr < kTile; ++rr) sacc += D2[j][rr] * H1[i][rr];
        out[kOffW2 + p] = sacc;
    }
    for (int p = t; p < kH * kIn; p += kGradThreads) {
        const int j = p / kIn, c = p % kIn;
        float sacc = 0.0f;
        for (int rr = 0; rr < kTile; ++rr) sacc += G1[j][rr] * X[c][rr];
        out[kOffW1 + p] = sacc;
    }
    if (q < 3) {
        // wave 0: b1, wave 1: b2, wave 2: w3 (unit r)
        float sacc = 0.0f;
        for (int rr = 0; rr < kTile; ++rr)
            sacc += q == 0 ? G1[r][rr] : q == 1 ? D2[r][rr] : DY[rr] * H2[r][rr];
        out[(q == 0 ? kOffB1 : q == 1 ? kOffB2 : kOffW3) + r] = sacc;
    } else if (r < 2) {
        // wave 3: b3 and the tile's loss
        float sacc = 0.0f;
        for (int rr = 0; rr < kTile; ++rr) sacc += r == 0 ? DY[rr] : LS[rr];
        if (r == 0)
            out[kOffB3] = sacc;
        else
            loss_part[blockIdx.x] = sacc;
    }
}

// Sum of the tiles' gradient slots in tile order; with m1 set, also the
// Adam update of the parameters (bias corrections c1 = 1 - b1^t, c2 =
// 1 - b2^t).
__global__ void k_mlp_reduce(const float* __restrict__ partial, uint64_t tiles, const float* __restrict__ loss_part,
                             float* __restrict__ grad, float* __restrict__ loss, float* __restrict__ params,
                             float* __restrict__ m1, float* __restrict__ m2, float lr, float b1, float b2, float eps,
                             float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpParams) {
        float s = 0.0f;
#pragma unroll 8
        for (uint64_t b = 0; b < tiles; ++b) s += partial[b * kMlpParams + p];
        if (grad) grad[p] = s;
        if (m1) {
            const float a = b1 * m1[p] + (1.0f - b1) * s;
            const float bb = b2 * m2[p] + (1.0f - b2) * s * s;
            m1[p] = a;
            m2[p] = bb;
            params[p] -= lr * (a / c1) / (sqrtf(bb / c2) + eps);
        }
    }
    if (p == kMlpParams && loss) {
        float s = 0.0f;
        for (uint64_t b = 0; b < tiles; ++b) s += loss_part[b];
        *loss = s;
    }
}

// ---------------------------------------------------------------------------
// BF16 MFMA inference.  One wave handles 32 rows at a time: layer 1 in FP32
// on the vector units (K = 8 is too small for the matrix cores), layer 2 as
// a 32 x 64 x 64 product on v_mfma_f32_32x32x16_bf16 (two 32-column output
// tiles, four K steps of 16, FP32 accumulation), layer 3 in FP32 with a
// cross-lane sum.  Operand layout of the instruction: lane l supplies
// A[m = l % 32][k = 8 (l / 32) + j] and B[k = 8 (l / 32) + j][n = l % 32],
// j = 0..7, and receives D[m = 8 (j / 4) + 4 (l / 32) + j % 4][n = l % 32],
// j = 0..15.  Output: y (optional) and the Q16 table round(2^16 y).
// ---------------------------------------------------------------------------
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__global__ __launch_bounds__(256) void k_mlp_infer(const float* __restrict__ params, const float* __restrict__ feats,
                                                   uint64_t n, uint32_t cls, const int32_t* __restrict__ base,
                                                   float y_min, float y_max, int32_t* __restrict__ lt,
                                                   float* __restrict__ yout) {
    const int lane = lane_id();
    const int col = lane & 31;   // m for A, n for B and D
    const int half = lane >> 5;  // which 8-wide slice of each K step
    // B operand (W2 transposed) in LDS, in the order lanes read it: slice
    // (nt, kc) of lane l is s_w2[(nt * 4 + kc) * 64 + l]
    __shared__ bf16x8 s_w2[2 * 4 * kWave];
    for (int i = (int)threadIdx.x; i < 2 * 4 * kWave; i += (int)blockDim.x) {
        const int l = i % kWave, nt = i / (4 * kWave), kc = (i / kWave) % 4;
        bf16x8 v;
        for (int j = 0; j < 8; ++j)
            v[j] = (__bf16)params[kOffW2 + (nt * 32 + (l & 31)) * kH + kc * 16 + (l >> 5) * 8 + j];
        s_w2[i] = v;
    }
    const float b2n[2] = {params[kOffB2 + col], params[kOffB2 + 32 + col]};
    const float w3n[2] = {params[kOffW3 + col], params[kOffW3 + 32 + col]};
    const float b3 = params[kOffB3];
    // layer 1 weights in LDS, per hidden unit: the bias plus the weight of
    // this position class's one-hot input, then the four feature weights
    __shared__ float s_l1[kH * 5];
    const uint32_t cc = cls < 3 ? cls : 3;
    for (int h = (int)threadIdx.x; h < kH; h += (int)blockDim.x) {
        s_l1[h * 5] = params[kOffB1 + h] + params[kOffW1 + h * kIn + 4 + (int)cc];
        for (int c = 0; c < 4; ++c) s_l1[h * 5 + 1 + c] = params[kOffW1 + h * kIn + c];
    }
    __syncthreads();
    const uint64_t gw = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x / kWave);
    const uint64_t tiles = (n + 31) / 32;
    for (uint64_t tile = gw; tile < tiles; tile += nw) {
        const uint64_t row = tile * 32 + (uint64_t)col;
        float x[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (row < n)
            for (int c = 0; c < 4; ++c) x[c] = feats[row * 4 + c];
        // layer 1: this lane's 32 of the row's 64 hidden units, as bf16 A
        // slices.  The weights are read from LDS in every tile: an opaque
        // zero offset keeps the compiler from hoisting all 160 of them into
        // registers, which would cut occupancy.
        int w0 = half * 8 * 5;
        asm volatile("" : "+v"(w0));
        bf16x8 a[4];
        for (int kc = 0; kc < 4; ++kc)
            for (int j = 0; j < 8; ++j) {
                const float* wl = s_l1 + w0 + (kc * 16 + j) * 5;
                float s = wl[0];
                for (int c = 0; c < 4; ++c) s += wl[1 + c] * x[c];
                a[kc][j] = (__bf16)gelu(s);
            }
        f32x16 acc0 = {}, acc1 = {};
        for (int kc = 0; kc < 4; ++kc) {
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[kc], s_w2[kc * kWave + lane], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[kc], s_w2[(4 + kc) * kWave + lane], acc1, 0, 0, 0);
        }
        // layer 3: contribution of this lane's two output columns to each of
        // its 16 rows, summed over the 32 lanes of the half
        float part[16];
        for (int j = 0; j < 16; ++j)
            part[j] = w3n[0] * gelu(acc0[j] + b2n[0]) + w3n[1] * gelu(acc1[j] + b2n[1]);
        for (int j = 0; j < 16; ++j) {
#pragma unroll
            for (int s = 16; s > 0; s >>= 1) part[j] += __shfl_xor(part[j], s, kWave);
        }
        // lane with col j < 16 of each half writes row m = 8 (j / 4) + 4 half + j % 4
        if (col < 16) {
            float y = b3;
            for (int j = 0; j < 16; ++j)
                if (j == col) y += part[j];
            const int m = 8 * (col / 4) + 4 * half + (col % 4);
            const uint64_t r = tile * 32 + (uint64_t)m;
            if (r < n) {
                // clamped to [y_min, y_max] and to +-2^13 (also maps NaN to a
                // finite value) so the Q16 code and the residual sum stay
                // inside int32
                const float yc = fminf(fmaxf(fminf(fmaxf(y, y_min), y_max), -8192.0f), 8192.0f);
                const int32_t q = (int32_t)rintf(yc * 65536.0f);
                // residual tables: the network's output corrects the f_approx
                // log weight; certain zeros stay marked
                lt[r] = base ? (base[r] == kCertainZero ? kCertainZero : base[r] + q) : q;
                if (yout) yout[r] = y;
            }
        }
    }
}

}  // namespace agis

using agis::kMlpParams;

namespace {

int lfail(agis_ctx* ctx, int code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return code;
}

#define LHIP(ctx, expr, what)                                                                     \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return lfail(ctx, e_ == hipErrorOutOfMemory ? AGIS_E_OOM : AGIS_E_HIP,                \
                         std::string(what) + ": " + hipGetErrorString(e_));                      \
    } while (0)

unsigned grid1(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

extern "C" {

int agis_mlp_param_count(void) { return kMlpParams; }

int agis_features(agis_ctx* ctx, const agis_tables* t, float* feats) {
    if (!ctx || !t || t->ctx != ctx || !feats) return AGIS_E_INVALID_ARG;
    LHIP(ctx, hipSetDevice(ctx->device), "set device");
    const agis::DevGraph& g = t->graph->g;
    if (g.n == 0) return AGIS_OK;
    if (g.n > UINT32_MAX) return lfail(ctx, AGIS_E_INVALID_ARG, "features: more than 2^32 - 1 vertices");
    // list of the vertices of degree above the per-lane limit, and its length
    uint32_t* big = nullptr;
    LHIP(ctx, hipMalloc(&big, (size_t)(g.n + 1) * sizeof(uint32_t)), "allocate feature list");
    uint32_t* nbig = big + g.n;
    hipError_t e = hipMemsetAsync(nbig, 0, sizeof(uint32_t), ctx->stream);
    const uint64_t groups = (g.n + 63) / 64;
    const uint64_t blocks = std::min<uint64_t>((groups + agis::kFeatWaves - 1) / agis::kFeatWaves,
                                               (uint64_t)ctx->num_cus * 8);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(agis::k_features, dim3((unsigned)blocks), dim3(agis::kFeatThreads), 0, ctx->stream, g,
                           t->rec, t->s2, t->hits, t->trials, feats, big, nbig);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(agis::k_features_big, dim3((unsigned)ctx->num_cus * 4), dim3(agis::kFeatThreads), 0,
                           ctx->stream, g, t->rec, t->s2, t->hits, t->trials, feats, big, nbig);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(big);
    LHIP(ctx, e, "features");
    return AGIS_OK;
}

int agis_learn_targets(agis_ctx* ctx, const agis_graph* g, const agis_tables* t, const agis_pattern* p,
                       const uint8_t* order, uint64_t n_samples, uint64_t seed, const agis_run_params* params,
                       double* sums, uint32_t* counts) {
    if (!ctx || !g || !t || !p || !sums || !counts) return AGIS_E_INVALID_ARG;
    if (p->k < 2 || p->k > 8) return lfail(ctx, AGIS_E_PATTERN, "pattern size must be in [2, 8]");
    LHIP(ctx, hipSetDevice(ctx->device), "set device");
    const uint64_t n = g->g.n;
    LHIP(ctx, hipMemsetAsync(sums, 0, (size_t)p->k * n * sizeof(double), ctx->stream), "clear sums");
    LHIP(ctx, hipMemsetAsync(counts, 0, (size_t)p->k * n * sizeof(uint32_t), ctx->stream), "clear counts");
    const uint64_t chunk = 1ull << 20;
    uint64_t* d_idx = nullptr;
    agis::Record* d_rec = nullptr;
    LHIP(ctx, hipMalloc(&d_idx, chunk * sizeof(uint64_t)), "allocate indices");
    hipError_t e = hipMalloc(&d_rec, chunk * sizeof(agis::Record));
    if (e != hipSuccess) {
        (void)hipFree(d_idx);
        return lfail(ctx, AGIS_E_OOM, "allocate records");
    }
    std::vector<uint64_t> idx(chunk);
    int rc = AGIS_OK;
    for (uint64_t done = 0; done < n_samples && rc == AGIS_OK; done += chunk) {
        const uint64_t m = std::min(chunk, n_samples - done);
        for (uint64_t j = 0; j < m; ++j) idx[j] = done + j;
        e = hipMemcpyAsync(d_idx, idx.data(), m * sizeof(uint64_t), hipMemcpyHostToDevice, ctx->stream);
        if (e != hipSuccess) {
            rc = lfail(ctx, AGIS_E_HIP, "upload indices");
            break;
        }
        rc = agis_dump_samples(ctx, g, t, p, order, seed, params, d_idx, m, (agis_record*)d_rec);
        if (rc != AGIS_OK) break;
        hipLaunchKernelGGL(agis::k_targets, dim3(grid1(m, 256)), dim3(256), 0, ctx->stream, d_rec, m, p->k, n, sums,
                           counts);
        e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) rc = lfail(ctx, AGIS_E_HIP, std::string("targets: ") + hipGetErrorString(e));
    }
    (void)hipFree(d_idx);
    (void)hipFree(d_rec);
    return rc;
}

int agis_learn_rows(agis_ctx* ctx, const double* sums, const uint32_t* counts, uint32_t k, uint64_t n,
                    uint32_t step_mask, uint32_t min_count, const int32_t* base, uint32_t* vtx, uint8_t* cls,
                    float* target, float* weight, uint64_t* rows) {
    if (!ctx || !sums || !counts || !vtx || !cls || !target || !weight || !rows || k == 0 || k > 8)
        return AGIS_E_INVALID_ARG;
    LHIP(ctx, hipSetDevice(ctx->device), "set device");
    std::vector<double> s(n);
    std::vector<uint32_t> c(n);
    std::vector<int32_t> bl(base ? n : 0);
    std::vector<uint32_t> hv;
    std::vector<uint8_t> hc;
    std::vector<float> ht, hw;
    for (uint32_t i = 0; i < k; ++i) {
        if (!(step_mask >> i & 1u)) continue;
        LHIP(ctx, hipMemcpy(s.data(), sums + (uint64_t)i * n, n * sizeof(double), hipMemcpyDeviceToHost), "read sums");
        LHIP(ctx, hipMemcpy(c.data(), counts + (uint64_t)i * n, n * sizeof(uint32_t), hipMemcpyDeviceToHost),
             "read counts");
        if (base)
            LHIP(ctx, hipMemcpy(bl.data(), base + (uint64_t)i * n, n * sizeof(int32_t), hipMemcpyDeviceToHost),
                 "read base");
        auto kept = [&](uint64_t v) {
            return c[v] >= min_count && c[v] != 0 && !(base && bl[v] == agis::kCertainZero);
        };
        // f_approx log weights are relative (constant factors cancel in the
        // pick), so their scale is calibrated first: kappa = sum s / sum c B
        double kappa = 1.0;
        if (base) {
            double num = 0.0, den = 0.0;
            for (uint64_t v = 0; v < n; ++v)
                if (kept(v)) {
                    num += s[v];
                    den += (double)c[v] * std::exp2((double)bl[v] / 65536.0);
                }
            if (num > 0.0 && den > 0.0) kappa = num / den;
        }
        for (uint64_t v = 0; v < n; ++v) {
            if (!kept(v)) continue;
            double tv;
            if (base) {
                // posterior mean of the completions with the calibrated
                // f_approx value kappa B as one pseudo-observation, relative
                // to kappa B
                const double kb = kappa * std::exp2((double)bl[v] / 65536.0);
                tv = std::log2((s[v] / kb + 1.0) / ((double)c[v] + 1.0));
            } else {
                tv = std::log2(1.0 + s[v] / (double)c[v]);
            }
            hv.push_back((uint32_t)v);
            hc.push_back((uint8_t)(i < 3 ? i : 3));
            ht.push_back((float)tv);
            hw.push_back((float)c[v]);
        }
    }
    const uint64_t r = hv.size();
    if (r) {
        LHIP(ctx, hipMemcpy(vtx, hv.data(), r * sizeof(uint32_t), hipMemcpyHostToDevice), "write rows");
        LHIP(ctx, hipMemcpy(cls, hc.data(), r * sizeof(uint8_t), hipMemcpyHostToDevice), "write rows");
        LHIP(ctx, hipMemcpy(target, ht.data(), r * sizeof(float), hipMemcpyHostToDevice), "write rows");
        LHIP(ctx, hipMemcpy(weight, hw.data(), r * sizeof(float), hipMemcpyHostToDevice), "write rows");
    }
    *rows = r;
    return AGIS_OK;
}

int agis_mlp_grad(agis_ctx* ctx, const float* params, const float* feats, const uint32_t* vtx, const uint8_t* cls,
                  const float* target, const float* weight, uint64_t rows, float weight_sum, float* grad, float* loss) {
    if (!ctx || !params || !feats || !vtx || !cls || !target || !weight || !grad || rows == 0 || !(weight_sum > 0))
        return AGIS_E_INVALID_ARG;
    LHIP(ctx, hipSetDevice(ctx->device), "set device");
    const uint64_t tiles = (rows + agis::kTile - 1) / agis::kTile;
    float* partial = nullptr;
    float* lpart = nullptr;
    LHIP(ctx, hipMalloc(&partial, tiles * kMlpParams * sizeof(float)), "allocate gradient partials");
    hipError_t e = hipMalloc(&lpart, tiles * sizeof(float));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(agis::k_mlp_grad, dim3((unsigned)tiles), dim3(agis::kGradThreads), 0, ctx->stream, params,
                           feats, vtx, cls, target, weight, nullptr, rows, 1.0f / weight_sum, partial, lpart);
        hipLaunchKernelGGL(agis::k_mlp_reduce, dim3(grid1(kMlpParams + 1, 256)), dim3(256), 0, ctx->stream, partial,
                           tiles, lpart, grad, loss, nullptr, nullptr, nullptr, 0.0f, 0.0f, 0.0f, 0.0f, 1.0f, 1.0f);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    }
    (void)hipFree(partial);
    if (lpart) (void)hipFree(lpart);
    LHIP(ctx, e, "mlp gradient");
    return AGIS_OK;
}

int agis_mlp_train(agis_ctx* ctx, float* params, const float* feats, const uint32_t* vtx, const uint8_t* cls,
                   const float* target, const float* weight, uint64_t rows, uint32_t epochs, uint32_t batch,
                   float lr, uint64_t shuffle_seed, float* loss_per_epoch) {
    if (!ctx || !params || !feats || !vtx || !cls || !target || !weight || rows == 0 || batch == 0)
        return AGIS_E_INVALID_ARG;
    if (rows >= (1ull << 32)) return lfail(ctx, AGIS_E_INVALID_ARG, "at most 2^32 - 1 rows");
    LHIP(ctx, hipSetDevice(ctx->device), "set device");
    const uint64_t bt = std::min<uint64_t>(batch, rows);
    const uint64_t tiles = (bt + agis::kTile - 1) / agis::kTile;
    std::vector<float> w(rows);
    LHIP(ctx, hipMemcpy(w.data(), weight, rows * sizeof(float), hipMemcpyDeviceToHost), "read weights");
    float *partial = nullptr, *lpart = nullptr, *m1 = nullptr, *m2 = nullptr, *loss = nullptr;
    uint32_t* order = nullptr;
    hipError_t e = hipMalloc(&partial, tiles * kMlpParams * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&lpart, tiles * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&m1, kMlpParams * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&m2, kMlpParams * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&loss, sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&order, rows * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemsetAsync(m1, 0, kMlpParams * sizeof(float), ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m2, 0, kMlpParams * sizeof(float), ctx->stream);
    std::vector<uint32_t> perm(rows);
    for (uint64_t i = 0; i < rows; ++i) perm[i] = (uint32_t)i;
    std::mt19937_64 rng(shuffle_seed);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    uint64_t step = 0;
    for (uint32_t ep = 0; ep < epochs && e == hipSuccess; ++ep) {
        std::shuffle(perm.begin(), perm.end(), rng);
        e = hipMemcpyAsync(order, perm.data(), rows * sizeof(uint32_t), hipMemcpyHostToDevice, ctx->stream);
        double ep_loss = 0.0;
        for (uint64_t s0 = 0; s0 < rows && e == hipSuccess; s0 += bt) {
            const uint64_t cnt = std::min(bt, rows - s0);
            double ws = 0.0;
            for (uint64_t i = 0; i < cnt; ++i) ws += w[perm[s0 + i]];
            if (!(ws > 0)) continue;
            const uint64_t tl = (cnt + agis::kTile - 1) / agis::kTile;
            hipLaunchKernelGGL(agis::k_mlp_grad, dim3((unsigned)tl), dim3(agis::kGradThreads), 0, ctx->stream, params,
                               feats, vtx, cls, target, weight, order + s0, cnt, (float)(1.0 / ws), partial, lpart);
            ++step;
            const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
            hipLaunchKernelGGL(agis::k_mlp_reduce, dim3(grid1(kMlpParams + 1, 256)), dim3(256), 0, ctx->stream,
                               partial, tl, lpart, nullptr, loss_per_epoch ? loss : nullptr, params, m1, m2, lr, b1,
                               b2, eps, c1, c2);
            e = hipGetLastError();
            if (loss_per_epoch) {
                float l = 0.0f;
                if (e == hipSuccess) e = hipMemcpyAsync(&l, loss, sizeof(float), hipMemcpyDeviceToHost, ctx->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
                ep_loss += (double)l * ws;
            }
        }
        if (loss_per_epoch) {
            double wt = 0.0;
            for (float x : w) wt += x;
            loss_per_epoch[ep] = (float)(ep_loss / wt);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    for (void* q : {(void*)partial, (void*)lpart, (void*)m1, (void*)m2, (void*)loss, (void*)order})
        if (q) (void)hipFree(q);
    LHIP(ctx, e, "mlp training");
    return AGIS_OK;
}

int agis_step_log_weights(agis_ctx* ctx, const agis_tables* t, uint32_t b, uint32_t f1, uint32_t ie, uint32_t f2,
                          int32_t* out) {
    if (!ctx || !t || t->ctx != ctx || !out || b > 7 || f1 > 7 || ie > 7 || f2 > 64) return AGIS_E_INVALID_ARG;
    LHIP(ctx, hipSetDevice(ctx->device), "set device");
    LHIP(ctx, agis::launch_step_log_weights(*t, t->graph->g.n, b, f1, ie, f2, nullptr, out, ctx->stream), "step log weights");
    LHIP(ctx, hipStreamSynchronize(ctx->stream), "step log weights");
    return AGIS_OK;
}

int agis_mlp_infer(agis_ctx* ctx, const float* params, const float* feats, uint64_t n, uint32_t position_class,
                   const int32_t* base, float y_min, float y_max, int32_t* lt, float* y) {
    if (!ctx || !params || !feats || !lt || position_class > 3 || !(y_min <= y_max)) return AGIS_E_INVALID_ARG;
    LHIP(ctx, hipSetDevice(ctx->device), "set device");
    if (n == 0) return AGIS_OK;
    const uint64_t tiles = (n + 31) / 32;
    const uint64_t blocks = std::min<uint64_t>((tiles + 3) / 4, (uint64_t)ctx->num_cus * 8);
    hipLaunchKernelGGL(agis::k_mlp_infer, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, params, feats, n,
                       position_class, base, y_min, y_max, lt, y);
    LHIP(ctx, hipGetLastError(), "mlp inference");
    LHIP(ctx, hipStreamSynchronize(ctx->stream), "mlp inference");
    return AGIS_OK;
}

}  // extern "C"
