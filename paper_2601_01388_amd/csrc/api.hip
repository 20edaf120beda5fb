// C-ABI entry points of the AGIS library (declared in include/agis.h).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "agis.h"
#include "agis_internal.h"

using agis::DevPlan;
using agis::Partial;

namespace {

int fail(agis_ctx* ctx, int code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int hip_fail(agis_ctx* ctx, hipError_t e, const char* what) {
    const int code = (e == hipErrorOutOfMemory) ? AGIS_E_OOM : AGIS_E_HIP;
    return fail(ctx, code, std::string(what) + ": " + hipGetErrorString(e));
}

#define AGIS_HIP(ctx, expr, what)                     \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)

// Standard normal quantile: Abramowitz-Stegun 26.2.23 start, refined by
// Newton steps on Phi(z) = erfc(-z / sqrt 2) / 2.
double normal_quantile(double p) {
    if (p <= 0.0) return -INFINITY;
    if (p >= 1.0) return INFINITY;
    const double q = p < 0.5 ? p : 1.0 - p;
    const double t = std::sqrt(-2.0 * std::log(q));
    double z = t - (2.515517 + 0.802853 * t + 0.010328 * t * t) / (1.0 + 1.432788 * t + 0.189269 * t * t +
                                                                     0.001308 * t * t * t);
    if (p < 0.5) z = -z;
    for (int it = 0; it < 6; ++it) {
        const double cdf = 0.5 * std::erfc(-z / std::sqrt(2.0));
        const double pdf = std::exp(-0.5 * z * z) / std::sqrt(2.0 * M_PI);
        z -= (cdf - p) / pdf;
    }
    return z;
}

struct Acc {
    double n = 0, mean = 0, m2 = 0, nonzero = 0;
    void merge(const Partial& b) {
        if (b.n == 0.0) return;
        if (n == 0.0) {
            n = b.n;
            mean = b.mean;
            m2 = b.m2;
            nonzero = b.nonzero;
            return;
        }
        const double tot = n + b.n;
        const double delta = b.mean - mean;
        mean = mean + delta * (b.n / tot);
        m2 = m2 + b.m2 + delta * delta * (n * b.n / tot);
        n = tot;
        nonzero += b.nonzero;
    }
};

double eps_hat_of(const Acc& a, double z) {
    if (a.n == 0.0 || a.mean == 0.0) return INFINITY;
    const double sigma = std::sqrt(a.m2 > 0 ? a.m2 / a.n : 0.0);
    return z * sigma / (std::sqrt(a.n) * std::fabs(a.mean));
}

agis_run_params default_params() {
    agis_run_params p;
    std::memset(&p, 0, sizeof(p));
    p.mode = AGIS_MODE_SWITCH;
    p.beta_num = 4;
    p.beta_den = 5;
    p.delta = 0.05;
    return p;
}

// Everything an estimate or dump needs, prepared on the device.
struct Prepared {
    agis_plan plan;
    DevPlan hp;
    agis::Step1 s1{nullptr, nullptr, 0};
    uint32_t* q1 = nullptr;
    uint64_t* pre = nullptr;
    std::vector<uint64_t*> rowtabs;
    int32_t* rowmax = nullptr;
    double tables_seconds = 0;
    ~Prepared() {
        if (q1) (void)hipFree(q1);
        if (pre) (void)hipFree(pre);
        if (rowmax) (void)hipFree(rowmax);
        for (uint64_t* r : rowtabs) (void)hipFree(r);
    }
};

// Per-row pick tables are built for runs of at least this many samples
// (AUTO): their build streams every CSR slot once, which a short run does
// not amortise.
constexpr uint64_t kRowtabMinSamples = 65536;
constexpr uint64_t kRowtabBudgetBytes = 32ull << 30;

int prepare(agis_ctx* ctx, const agis_graph* g, const agis_tables* t, const agis_pattern* p, const uint8_t* order,
            const agis_run_params* params, uint64_t n_samples, Prepared* out) {
    int rc = agis::compile_plan(p, order, params->mode, params->beta_num, params->beta_den, &out->plan, &ctx->err);
    if (rc != AGIS_OK) return rc;
    if (params->flags > AGIS_RUN_ROWTAB_OFF) return fail(ctx, AGIS_E_INVALID_ARG, "unknown run flag");
    DevPlan& hp = out->hp;
    std::memset(&hp, 0, sizeof(hp));
    hp.k = out->plan.k;
    hp.pattern_id = params->pattern_id;
    for (uint32_t i = 0; i < hp.k; ++i) {
        hp.bmask[i] = out->plan.bmask[i];
        hp.b[i] = out->plan.b[i];
        hp.f1[i] = out->plan.f1[i];
        hp.ie[i] = out->plan.ie[i];
        hp.f2[i] = out->plan.f2[i];
        // |F1| = 0 makes every weight C(d - b, 0) = 1: a uniform draw.
        hp.weighted[i] = (out->plan.decision[i] && out->plan.f1[i] > 0) ? 1 : 0;
        if (params->mode == AGIS_MODE_LEARNED && hp.weighted[i]) {
            if (!params->learned[i]) return fail(ctx, AGIS_E_INVALID_ARG, "learned mode needs a table for every weighted step");
            hp.lt[i] = params->learned[i];
        }
    }
    const auto t0 = std::chrono::steady_clock::now();
    // per-row pick tables for weighted steps with one backward vertex
    bool want_rows = params->flags == AGIS_RUN_ROWTAB_ON ||
                     (params->flags == AGIS_RUN_ROWTAB_AUTO && n_samples >= kRowtabMinSamples);
    int32_t* rowmax = nullptr;
    if (want_rows && g->g.nnz > 0) {
        struct Key {
            uint32_t f1, ie, f2;
            const int32_t* lt;
            uint64_t* buf;
        };
        std::vector<Key> built;
        for (uint32_t i = 1; i < hp.k; ++i) {
            if (!hp.weighted[i] || __builtin_popcount(hp.bmask[i]) != 1) continue;
            uint64_t* buf = nullptr;
            for (const Key& k : built)
                if (k.f1 == hp.f1[i] && k.ie == hp.ie[i] && k.f2 == hp.f2[i] && k.lt == hp.lt[i]) buf = k.buf;
            if (!buf) {
                if ((built.size() + 1) * g->g.nnz * sizeof(uint64_t) > kRowtabBudgetBytes) continue;
                AGIS_HIP(ctx, hipMalloc(&buf, g->g.nnz * sizeof(uint64_t)), "allocate row pick table");
                out->rowtabs.push_back(buf);
                if (!rowmax) {
                    AGIS_HIP(ctx, hipMalloc(&rowmax, g->g.n * sizeof(int32_t)), "allocate row maxima");
                    out->rowmax = rowmax;
                }
                AGIS_HIP(ctx,
                         agis::launch_rowtab(ctx, g->g, t->rec, 1, hp.f1[i], hp.ie[i], hp.f2[i], hp.lt[i], buf, rowmax),
                         "row pick table");
                built.push_back(Key{hp.f1[i], hp.ie[i], hp.f2[i], hp.lt[i], buf});
            }
            hp.rowpre[i] = buf;
        }
    }
    // A step builds its candidate set in the wave's scratch unless it draws
    // uniformly from one backward list or through a row table.  When step
    // i-1 did and its backward set is contained in step i's, step i starts
    // from that set.
    auto general = [&](uint32_t i) {
        return (hp.weighted[i] && hp.rowpre[i] == nullptr) || __builtin_popcount(hp.bmask[i]) > 1;
    };
    for (uint32_t i = 2; i < hp.k; ++i)
        hp.reuse[i] = (general(i) && general(i - 1) && (hp.bmask[i - 1] & ~hp.bmask[i]) == 0) ? 1 : 0;
    if (hp.weighted[0] && g->g.n > 0) {
        AGIS_HIP(ctx, hipMalloc(&out->q1, g->g.n * sizeof(uint32_t)), "allocate first-step weights");
        AGIS_HIP(ctx, hipMalloc(&out->pre, g->g.n * sizeof(uint64_t)), "allocate first-step prefix");
        uint64_t total = 0;
        AGIS_HIP(ctx, agis::build_step1(ctx, *g, *t, hp, out->q1, out->pre, &total), "first-step table");
        out->s1 = agis::Step1{out->q1, out->pre, total};
    }
    AGIS_HIP(ctx, hipMemcpyAsync(ctx->d_plan, &hp, sizeof(hp), hipMemcpyHostToDevice, ctx->stream), "upload plan");
    AGIS_HIP(ctx, hipStreamSynchronize(ctx->stream), "upload plan");
    out->tables_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return AGIS_OK;
}

int check_handles(const agis_ctx* ctx, const agis_graph* g, const agis_tables* t) {
    if (!ctx || !g || !t) return AGIS_E_INVALID_ARG;
    if (g->ctx != ctx || t->ctx != ctx || t->graph != g) return AGIS_E_INVALID_ARG;
    return AGIS_OK;
}

}  // namespace

extern "C" {

int agis_create(agis_ctx** out, int device, void* hip_stream) {
    if (!out) return AGIS_E_INVALID_ARG;
    *out = nullptr;
    agis_ctx* ctx = new (std::nothrow) agis_ctx();
    if (!ctx) return AGIS_E_OOM;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, device);
        if (e == hipSuccess) ctx->num_cus = prop.multiProcessorCount;
    }
    if (e == hipSuccess) e = hipMalloc(&ctx->d_plan, sizeof(DevPlan));
    if (e == hipSuccess) e = hipMalloc(&ctx->d_small, 4096);
    if (e == hipSuccess) e = hipEventCreate(&ctx->ev_start);
    if (e == hipSuccess) e = hipEventCreate(&ctx->ev_stop);
    if (e == hipSuccess) e = agis::upload_fixed_point_tables(ctx->stream);
    if (e != hipSuccess) {
        agis_destroy(ctx);
        return e == hipErrorOutOfMemory ? AGIS_E_OOM : AGIS_E_HIP;
    }
    *out = ctx;
    return AGIS_OK;
}

void agis_destroy(agis_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->d_plan) (void)hipFree(ctx->d_plan);
    if (ctx->d_small) (void)hipFree(ctx->d_small);
    if (ctx->d_partials) (void)hipFree(ctx->d_partials);
    if (ctx->d_scratch) (void)hipFree(ctx->d_scratch);
    if (ctx->d_xout) (void)hipFree(ctx->d_xout);
    if (ctx->d_blocksums) (void)hipFree(ctx->d_blocksums);
    if (ctx->ev_start) (void)hipEventDestroy(ctx->ev_start);
    if (ctx->ev_stop) (void)hipEventDestroy(ctx->ev_stop);
    delete ctx;
}

const char* agis_last_error(const agis_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int agis_load_csr(agis_ctx* ctx, const uint64_t* off, const uint32_t* nbr, uint64_t n, uint64_t nnz, uint32_t flags,
                  agis_graph** out) {
    if (!ctx || !out) return AGIS_E_INVALID_ARG;
    *out = nullptr;
    if (n == 0 || n >= (1ull << 32)) return fail(ctx, AGIS_E_INVALID_ARG, "n must be in [1, 2^32)");
    if (!off || (nnz > 0 && !nbr)) return fail(ctx, AGIS_E_INVALID_ARG, "null CSR pointer");
    if (flags & ~AGIS_CSR_VALIDATE) return fail(ctx, AGIS_E_INVALID_ARG, "unknown flag");
    AGIS_HIP(ctx, hipSetDevice(ctx->device), "set device");
    uint64_t ends[2] = {1, 1};
    AGIS_HIP(ctx, hipMemcpyAsync(&ends[0], off, sizeof(uint64_t), hipMemcpyDeviceToHost, ctx->stream), "read off[0]");
    AGIS_HIP(ctx, hipMemcpyAsync(&ends[1], off + n, sizeof(uint64_t), hipMemcpyDeviceToHost, ctx->stream),
             "read off[n]");
    AGIS_HIP(ctx, hipStreamSynchronize(ctx->stream), "read offsets");
    if (ends[0] != 0 || ends[1] != nnz) return fail(ctx, AGIS_E_INVALID_CSR, "off[0] must be 0 and off[n] must be nnz");
    if (nnz & 1ull) return fail(ctx, AGIS_E_INVALID_CSR, "nnz of a symmetric graph must be even");
    agis::DevGraph dg{off, nbr, n, nnz};
    uint32_t* d_cells = (uint32_t*)ctx->d_small;
    uint32_t cells[2] = {0, 0};
    AGIS_HIP(ctx, hipMemsetAsync(d_cells, 0, 2 * sizeof(uint32_t), ctx->stream), "clear flags");
    if (flags & AGIS_CSR_VALIDATE) {
        AGIS_HIP(ctx, agis::launch_validate_rows(dg, d_cells, ctx->stream), "validate CSR rows");
        AGIS_HIP(ctx, hipMemcpyAsync(cells, d_cells, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream),
                 "read flags");
        AGIS_HIP(ctx, hipStreamSynchronize(ctx->stream), "validate CSR rows");
        if (cells[0] == 0) AGIS_HIP(ctx, agis::launch_validate_edges(dg, d_cells, ctx->stream), "validate CSR edges");
    }
    if (cells[0] == 0) AGIS_HIP(ctx, agis::launch_max_degree(dg, d_cells + 1, ctx->stream), "max degree");
    AGIS_HIP(ctx, hipMemcpyAsync(cells, d_cells, sizeof(cells), hipMemcpyDeviceToHost, ctx->stream), "read flags");
    AGIS_HIP(ctx, hipStreamSynchronize(ctx->stream), "validate CSR");
    if (cells[0]) {
        std::string m = "invalid CSR:";
        if (cells[0] & 1u) m += " offsets not non-decreasing or beyond nnz;";
        if (cells[0] & 2u) m += " neighbour id >= n;";
        if (cells[0] & 4u) m += " self-loop;";
        if (cells[0] & 8u) m += " row not strictly ascending (unsorted or duplicate);";
        if (cells[0] & 16u) m += " not symmetric;";
        return fail(ctx, AGIS_E_INVALID_CSR, m);
    }
    agis_graph* g = new (std::nothrow) agis_graph();
    if (!g) return fail(ctx, AGIS_E_OOM, "host allocation");
    g->ctx = ctx;
    g->g = dg;
    g->max_deg = cells[1];
    *out = g;
    return AGIS_OK;
}

void agis_graph_destroy(agis_graph* g) { delete g; }

int agis_build_proposal_tables(agis_ctx* ctx, const agis_graph* g, uint64_t cv_seed, int32_t lc_min_q16,
                               int32_t exact_cv, agis_tables** out) {
    if (!ctx || !g || !out || g->ctx != ctx) return AGIS_E_INVALID_ARG;
    *out = nullptr;
    if (lc_min_q16 > 0) return fail(ctx, AGIS_E_INVALID_ARG, "log2 of the clustering floor must be <= 0");
    AGIS_HIP(ctx, hipSetDevice(ctx->device), "set device");
    agis_tables* t = new (std::nothrow) agis_tables();
    if (!t) return fail(ctx, AGIS_E_OOM, "host allocation");
    t->ctx = ctx;
    t->graph = g;
    const uint64_t n = g->g.n;
    hipError_t e = hipMalloc(&t->rec, n * sizeof(uint4));
    if (e == hipSuccess) e = hipMalloc(&t->s2, n * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc(&t->hits, n * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc(&t->trials, n * sizeof(uint64_t));
    if (e == hipSuccess)
        e = agis::launch_build_tables(g->g, t->rec, t->s2, t->hits, t->trials, (uint32_t)cv_seed,
                                      (uint32_t)(cv_seed >> 32), lc_min_q16, exact_cv ? 1 : 0, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        agis_tables_destroy(t);
        return hip_fail(ctx, e, "build proposal tables");
    }
    *out = t;
    return AGIS_OK;
}

void agis_tables_destroy(agis_tables* t) {
    if (!t) return;
    if (t->rec) (void)hipFree(t->rec);
    if (t->s2) (void)hipFree(t->s2);
    if (t->hits) (void)hipFree(t->hits);
    if (t->trials) (void)hipFree(t->trials);
    delete t;
}

int agis_tables_export(agis_ctx* ctx, const agis_tables* t, uint32_t* deg, uint64_t* s2, uint64_t* hits,
                       uint64_t* trials, int32_t* la, int32_t* lc) {
    if (!ctx || !t || t->ctx != ctx) return AGIS_E_INVALID_ARG;
    AGIS_HIP(ctx, hipSetDevice(ctx->device), "set device");
    const uint64_t n = t->graph->g.n;
    hipStream_t st = ctx->stream;
    if (s2) AGIS_HIP(ctx, hipMemcpyAsync(s2, t->s2, n * 8, hipMemcpyDeviceToDevice, st), "export s2");
    if (hits) AGIS_HIP(ctx, hipMemcpyAsync(hits, t->hits, n * 8, hipMemcpyDeviceToDevice, st), "export hits");
    if (trials) AGIS_HIP(ctx, hipMemcpyAsync(trials, t->trials, n * 8, hipMemcpyDeviceToDevice, st), "export trials");
    AGIS_HIP(ctx, agis::launch_export_tables(*t, n, deg, la, lc, st), "export tables");
    AGIS_HIP(ctx, hipStreamSynchronize(st), "export tables");
    return AGIS_OK;
}

int agis_compile_pattern(const agis_pattern* p, const uint8_t* order, const agis_run_params* params, agis_plan* out) {
    const agis_run_params dp = default_params();
    const agis_run_params* pp = params ? params : &dp;
    std::string err;
    return agis::compile_plan(p, order, pp->mode, pp->beta_num, pp->beta_den, out, &err);
}

int agis_estimate(agis_ctx* ctx, const agis_graph* g, const agis_tables* t, const agis_pattern* p,
                  const uint8_t* order, uint64_t n_samples, uint64_t seed, const agis_run_params* params,
                  agis_result* out) {
    int rc = check_handles(ctx, g, t);
    if (rc != AGIS_OK) return ctx ? fail(ctx, rc, "bad handle") : rc;
    if (!p || !out) return fail(ctx, AGIS_E_INVALID_ARG, "null pattern or result");
    const agis_run_params dp = default_params();
    const agis_run_params* pp = params ? params : &dp;
    if (pp->eps > 0 && !(pp->delta > 0 && pp->delta < 1)) return fail(ctx, AGIS_E_INVALID_ARG, "delta must be in (0, 1)");
    AGIS_HIP(ctx, hipSetDevice(ctx->device), "set device");
    const auto t0 = std::chrono::steady_clock::now();
    Prepared prep;
    rc = prepare(ctx, g, t, p, order, pp, n_samples, &prep);
    if (rc != AGIS_OK) return rc;
    const bool to_eps = pp->eps > 0;
    const uint64_t batch = to_eps ? (pp->check_every ? pp->check_every : 65536) : n_samples;
    const double z = normal_quantile(1.0 - (to_eps ? pp->delta : 0.05) / 2.0);
    Acc acc;
    bool converged = false;
    uint64_t done = 0;
    double kernel_seconds = 0.0;
    uint64_t launches = 0;
    if (n_samples > 0) {
        agis::SampleLaunch L = agis::plan_sample_launch(ctx, *g, batch < n_samples ? batch : n_samples, &ctx->err, &rc);
        if (rc != AGIS_OK) return rc;
        std::vector<Partial> parts;
        const agis::DevTables dt{t->rec};
        while (done < n_samples) {
            const uint64_t cnt = (n_samples - done) < batch ? (n_samples - done) : batch;
            AGIS_HIP(ctx,
                     agis::launch_sample(ctx, L, g->g, dt, prep.s1, (uint32_t)seed, (uint32_t)(seed >> 32), done, cnt,
                                         nullptr, nullptr, ctx->ev_start, ctx->ev_stop),
                     "launch sampler");
            AGIS_HIP(ctx, agis::launch_reduce(ctx, L, cnt), "launch reduction");
            parts.resize((size_t)((cnt + agis::kReduceTileSamples - 1) / agis::kReduceTileSamples));
            AGIS_HIP(ctx,
                     hipMemcpyAsync(parts.data(), ctx->d_partials, parts.size() * sizeof(Partial),
                                    hipMemcpyDeviceToHost, ctx->stream),
                     "read partials");
            AGIS_HIP(ctx, hipStreamSynchronize(ctx->stream), "sampler");
            float ms = 0.0f;
            AGIS_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop), "event time");
            kernel_seconds += 1e-3 * (double)ms;
            ++launches;
            for (const Partial& q : parts) acc.merge(q);
            done += cnt;
            if (to_eps && done >= pp->min_samples && eps_hat_of(acc, z) <= pp->eps) {
                converged = true;
                break;
            }
        }
    }
    std::memset(out, 0, sizeof(*out));
    out->estimate = acc.mean;
    out->copies = prep.plan.aut ? acc.mean / (double)prep.plan.aut : 0.0;
    out->variance = acc.n > 0 ? acc.m2 / acc.n : 0.0;
    out->eps_hat = eps_hat_of(acc, z);
    out->n = (uint64_t)acc.n;
    out->n_nonzero = (uint64_t)acc.nonzero;
    out->aut = prep.plan.aut;
    out->converged = converged ? 1 : 0;
    out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    out->tables_seconds = prep.tables_seconds;
    out->sample_kernel_seconds = kernel_seconds;
    out->sample_launches = launches;
    out->plan = prep.plan;
    if (to_eps && !converged) return fail(ctx, AGIS_E_NOT_CONVERGED, "sample budget reached before eps");
    return AGIS_OK;
}

int agis_dump_samples(agis_ctx* ctx, const agis_graph* g, const agis_tables* t, const agis_pattern* p,
                      const uint8_t* order, uint64_t seed, const agis_run_params* params, const uint64_t* idx,
                      uint64_t m, agis_record* out) {
    int rc = check_handles(ctx, g, t);
    if (rc != AGIS_OK) return ctx ? fail(ctx, rc, "bad handle") : rc;
    if (!p || (m > 0 && (!idx || !out))) return fail(ctx, AGIS_E_INVALID_ARG, "null pattern, index list or output");
    static_assert(sizeof(agis_record) == sizeof(agis::Record), "record layout");
    const agis_run_params dp = default_params();
    const agis_run_params* pp = params ? params : &dp;
    AGIS_HIP(ctx, hipSetDevice(ctx->device), "set device");
    Prepared prep;
    rc = prepare(ctx, g, t, p, order, pp, m, &prep);
    if (rc != AGIS_OK) return rc;
    if (m == 0) return AGIS_OK;
    agis::SampleLaunch L = agis::plan_sample_launch(ctx, *g, m, &ctx->err, &rc);
    if (rc != AGIS_OK) return rc;
    const agis::DevTables dt{t->rec};
    AGIS_HIP(ctx,
             agis::launch_sample(ctx, L, g->g, dt, prep.s1, (uint32_t)seed, (uint32_t)(seed >> 32), 0, m, idx,
                                 (agis::Record*)out, nullptr, nullptr),
             "launch sampler");
    AGIS_HIP(ctx, hipStreamSynchronize(ctx->stream), "sampler");
    return AGIS_OK;
}

int agis_fixed_point_tables(int32_t* logtab, uint32_t* exp2tab) {
    if (!logtab || !exp2tab) return AGIS_E_INVALID_ARG;
    std::memcpy(logtab, agis::host_logtab(), 4096 * sizeof(int32_t));
    std::memcpy(exp2tab, agis::host_exp2tab(), 4096 * sizeof(uint32_t));
    return AGIS_OK;
}

int agis_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    if (!ctr || !key || !out) return AGIS_E_INVALID_ARG;
    agis::U32x4 o = agis::philox4x32_10(agis::U32x4{ctr[0], ctr[1], ctr[2], ctr[3]}, key[0], key[1]);
    out[0] = o.x;
    out[1] = o.y;
    out[2] = o.z;
    out[3] = o.w;
    return AGIS_OK;
}

}  // extern "C"
