/*
 * agis.h -- C-ABI of the MI355X (gfx950) implementation of the AGIS
 * structure-informed sampling estimator for approximate graph pattern
 * counting ("AGIS: Fast Approximate Graph Pattern Mining with
 * Structure-Informed Sampling", PVLDB 19(2)).
 *
 * The library estimates C(G, P), the number of embeddings (injective,
 * edge-preserving maps V_P -> V_G; Sec. 2.1) of a small pattern P in a large
 * undirected data graph G.  Each sample extends a partial embedding along a
 * matching order (Algorithm 3), drawing each next vertex either uniformly
 * (f_uniform, Sec. 5.3) or from the approximate ideal distribution
 * (f_approx, Eq. probability_function, Sec. 4.2.3) as the decision function
 * chooses (Definition "Decision Function", Sec. 5.1), and returns the
 * importance weight 1/p.  The mean of many samples is the estimate;
 * Algorithm 1 decides when it is within the requested error.
 *
 * Conventions for every entry point:
 *  - Return value: AGIS_OK (0) or a negative AGIS_E_* code.  No C++
 *    exception crosses this boundary.  After an error, agis_last_error()
 *    on the same context returns a message (valid until the next call).
 *  - Pointers documented as "device" point into memory of the context's
 *    GPU; "host" pointers point into ordinary process memory.
 *  - Ownership: the caller owns every buffer it passes; the library owns
 *    the handles it returns (free them with the matching *_destroy).
 *  - Streams: all GPU work of a context is enqueued on the stream given to
 *    agis_create (0 = the null stream); entry points return after the work
 *    they need has finished on that stream.
 *  - Determinism: sample s of pattern id p under seed S is a pure function
 *    of (graph, tables, pattern, order, mode, beta, S, p, s) -- independent
 *    of launch shape, batch size and of the GPU -- so its vertex choices
 *    and integer factors equal those of a CPU implementation of the same
 *    definitions bit for bit, and its weight X is the same IEEE double.
 */
#ifndef AGIS_H
#define AGIS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AGIS_MAX_K 8

/* Status codes. */
enum {
    AGIS_OK = 0,
    AGIS_E_INVALID_ARG = -1,   /* NULL handle/pointer, bad size or flag */
    AGIS_E_INVALID_CSR = -2,   /* CSR fails validation (see agis_load_csr) */
    AGIS_E_PATTERN = -3,       /* pattern not connected, or k outside [2, 8] */
    AGIS_E_ORDER = -4,         /* order not a permutation, or a prefix is disconnected */
    AGIS_E_OOM = -5,           /* device allocation failed */
    AGIS_E_HIP = -6,           /* HIP runtime error (message has the HIP string) */
    AGIS_E_NOT_CONVERGED = -7, /* run-to-epsilon hit its budget; result is filled */
    AGIS_E_UNSUPPORTED = -8,   /* request outside what this build supports */
    AGIS_E_CANCELLED = -9      /* the caller's cancel flag was seen; results hold the samples finished so far */
};

/* Proposal modes. */
enum {
    AGIS_MODE_UNIFORM = 0, /* f_uniform at every step: edge-uniform first vertex, then uniform over S */
    AGIS_MODE_SWITCH = 1,  /* the paper's hybrid: f_approx where the decision function says so */
    AGIS_MODE_ALWAYS = 2,  /* f_approx at every step (beta = -infinity) */
    AGIS_MODE_LEARNED = 3  /* decisions as SWITCH; weighted steps read learned log-weight tables */
};

/* agis_load_csr flags. */
#define AGIS_CSR_VALIDATE 1u

typedef struct agis_ctx agis_ctx;
typedef struct agis_graph agis_graph;
typedef struct agis_tables agis_tables;

/* A pattern graph on vertices 0..k-1: bit w of adj[u] is set iff {u, w} is
 * an edge (symmetric, no self-loops).  2 <= k <= 8, connected. */
typedef struct {
    uint32_t k;
    uint8_t adj[AGIS_MAX_K];
} agis_pattern;

/* Result of the pattern compiler (Sec. 4.2.2-4.2.3, 5.1, 5.2) for one
 * matching order: per step i (0-based, vertex order[i]):
 * bmask: bit j set iff order[j] (j < i) is adjacent to order[i];
 * b = |B|, f1 = |F1|, i1 = |I1|, ie = |I_effective|, f2 = |F2|;
 * certainty = cert_num / cert_den (Definition "Decision Function");
 * decision: 1 = f_approx (or learned), 0 = f_uniform, after the mode and
 * beta are applied; aut = |Aut(P)|. */
typedef struct {
    uint32_t k;
    uint32_t aut;
    uint8_t order[AGIS_MAX_K];
    uint8_t bmask[AGIS_MAX_K];
    uint8_t b[AGIS_MAX_K];
    uint8_t f1[AGIS_MAX_K];
    uint8_t i1[AGIS_MAX_K];
    uint8_t ie[AGIS_MAX_K];
    uint8_t f2[AGIS_MAX_K];
    uint8_t decision[AGIS_MAX_K];
    int32_t cert_num[AGIS_MAX_K];
    int32_t cert_den[AGIS_MAX_K];
} agis_plan;

/* Run parameters.
 * beta: decision threshold beta_num / beta_den compared exactly; with
 *   beta_den == 0 the threshold is +infinity if beta_num > 0 (always
 *   uniform) and -infinity otherwise (always f_approx).  The paper's
 *   default is 4/5 (Sec. 5.1).
 * eps, delta: Algorithm 1 target; eps <= 0 means "run exactly n_samples".
 * check_every: samples between convergence checks (0 = 65536).
 * min_samples: no convergence is declared before this many samples.
 * pattern_id: enters the random stream of every sample (Philox counter).
 * flags: AGIS_RUN_ROWTAB_* -- whether a weighted step with a single matched
 *   neighbour draws through per-row pick tables built for this estimate,
 *   and a weighted step over two matched neighbours of the core through
 *   pick tables over their common-neighbour lists (same samples either
 *   way; AUTO builds them for runs of >= 65536 samples when they fit in
 *   memory).  Also in flags: how a weighted first
 *   step's distribution over all vertices is held -- AGIS_RUN_STEP1_FULL
 *   (the integer weight and inclusive prefix of every vertex, 12 bytes per
 *   vertex) or AGIS_RUN_STEP1_BLOCKS (the prefix over blocks of 256
 *   vertices, 8 bytes per block; a draw recomputes its block's weights from
 *   the vertex records); neither = full up to 2 GiB, blocked beyond.  The
 *   samples are the same either way.  A run to epsilon (eps > 0) whose
 *   check_every is a multiple of 2048 runs in one persistent launch that
 *   merges, checks and stops every pattern on the device;
 *   AGIS_RUN_HOST_ROUNDS asks for one launch per round of check_every
 *   samples with the checks on the host instead.  Both stop at the same
 *   sample counts and give the same results (to relative 1e-9).
 *   Plans whose steps after the first are all uniform draws from the row of
 *   one matched vertex (stars under switching, trees under f_uniform) run
 *   one sample per lane in fixed-budget runs, records and round-by-round
 *   runs; AGIS_RUN_WAVE_SAMPLES keeps them on the one-wave-per-sample
 *   sampler.  The samples are the same either way.
 * terms: which factors of f_approx (Eq. probability_function) enter the
 *   weights -- AGIS_TERMS_ALL (T[F1] T[I1] T[F2], the method), or the
 *   incremental versions of the paper's analysis of the approximation
 *   (Sec. 6.2, analysis of the approximate distribution): AGIS_TERMS_F1
 *   (T[F1] only) and AGIS_TERMS_F1_I1 (T[F1] T[I1]).  The decision function
 *   and the reported plan are unchanged.
 * learned: for AGIS_MODE_LEARNED, per step a device int32[n] table of Q16
 *   log2 weights (NULL for steps that are not weighted); ignored otherwise.
 * first_sample: the run draws samples first_sample, first_sample + 1, ...
 *   (0 for a fresh run); a run resumed where an earlier one stopped
 *   continues the same sample sequence, so results over the concatenated
 *   ranges equal one run over the whole range (checks of a resumed run
 *   count its own samples).
 * cancel: host int32 polled while the call runs (NULL: none); once it reads
 *   nonzero the call returns AGIS_E_CANCELLED with every result filled from
 *   the samples merged so far: whole reduction tiles of 2048 samples in
 *   index order (whole rounds of the round-by-round run), a prefix of each
 *   pattern's sample sequence, so a consistent partial estimate.
 * batch_learned: for AGIS_MODE_LEARNED in agis_estimate_batch, a host array
 *   of n_patterns x AGIS_MAX_K device table pointers (pattern i's tables at
 *   [i * AGIS_MAX_K .. + AGIS_MAX_K), as `learned` of a single estimate);
 *   ignored elsewhere. */
#define AGIS_RUN_ROWTAB_AUTO 0u
#define AGIS_RUN_ROWTAB_ON 1u
#define AGIS_RUN_ROWTAB_OFF 2u
#define AGIS_RUN_STEP1_BLOCKS 4u
#define AGIS_RUN_STEP1_FULL 8u
#define AGIS_RUN_HOST_ROUNDS 16u
#define AGIS_RUN_WAVE_SAMPLES 32u
#define AGIS_TERMS_ALL 0u
#define AGIS_TERMS_F1 1u
#define AGIS_TERMS_F1_I1 2u
typedef struct {
    int32_t mode;
    int32_t beta_num;
    int32_t beta_den;
    uint32_t pattern_id;
    uint32_t flags;
    uint32_t terms;
    double eps;
    double delta;
    uint64_t check_every;
    uint64_t min_samples;
    const int32_t* learned[AGIS_MAX_K];
    uint64_t first_sample;
    const volatile int32_t* cancel;
    const int32_t* const* batch_learned;
} agis_run_params;

/* Estimator output.  estimate = mean of the sample weights X (an unbiased
 * estimate of C(G, P), embeddings); copies = estimate / |Aut(P)|;
 * variance = population variance of X (Algorithm 1's sigma^2);
 * eps_hat = Algorithm 1's estimated relative error at delta;
 * seconds = wall time from the first GPU launch of the estimate (including
 * the per-estimate tables) to the result; tables_seconds = building the
 * per-estimate proposal tables (the first-step distribution over all
 * vertices and any per-row pick tables); sample_kernel_seconds = GPU time of the sampling
 * kernel launches (HIP events on the context's stream) over
 * sample_launches launches. */
typedef struct {
    double estimate;
    double copies;
    double variance;
    double eps_hat;
    uint64_t n;
    uint64_t n_nonzero;
    uint32_t aut;
    int32_t converged;
    double seconds;
    double tables_seconds;
    double sample_kernel_seconds;
    uint64_t sample_launches;
    agis_plan plan;
} agis_result;

/* Per-sample record written by agis_dump_samples (176 bytes, host layout):
 * v[i] = data vertex picked at step i, num[i]/den[i] = the integer factor
 * of step i (|S| / 1 for uniform steps, Q / q(v) for weighted ones),
 * x = the sample weight (0 when the sample failed), steps = steps that
 * picked a vertex, fail_step = -1 on success, else the step whose
 * candidate set (or total weight) was empty.  Unused entries are 0. */
typedef struct {
    uint32_t v[AGIS_MAX_K];
    uint64_t num[AGIS_MAX_K];
    uint64_t den[AGIS_MAX_K];
    double x;
    int32_t steps;
    int32_t fail_step;
} agis_record;

/* Creates a context on GPU `device` that enqueues work on `hip_stream`
 * (a hipStream_t, borrowed; 0 = null stream).  *out receives the handle. */
int agis_create(agis_ctx** out, int device, void* hip_stream);
void agis_destroy(agis_ctx* ctx);
const char* agis_last_error(const agis_ctx* ctx);

/* Gives back the device memory a context keeps between estimates for its
 * sampler: the waves' candidate scratch (sized at an estimate to half of
 * the device memory then free, with what the context already holds, within
 * [8, 64] GiB), the round weights and partials, and the run-to-eps
 * buffers.  For callers that allocate memory of their own between
 * estimates; the next estimate allocates what it needs again, with the
 * same results.  Waits for the context's stream and drops its captured
 * launch graph.  Graphs, tables and their proposal-table caches are kept
 * (agis_tables_destroy frees those). */
int agis_release_scratch(agis_ctx* ctx);

/* Registers a symmetric CSR graph (Sec. 5.4: the graph is held in CSR).
 * off: device uint64[n + 1], off[0] = 0, off[n] = nnz, non-decreasing;
 * nbr: device uint32[nnz], each row strictly ascending, ids < n, no
 * self-loops, and x in row v iff v in row x.  Both are BORROWED: they must
 * stay valid and unchanged until agis_graph_destroy.  With
 * AGIS_CSR_VALIDATE every property is checked on the GPU and a violation
 * returns AGIS_E_INVALID_CSR.  n must be < 2^32. */
int agis_load_csr(agis_ctx* ctx, const uint64_t* off, const uint32_t* nbr, uint64_t n, uint64_t nnz,
                  uint32_t flags, agis_graph** out);
void agis_graph_destroy(agis_graph* g);

/* Degree orientation for clique patterns (Sec. 5.4, orientation
 * optimisation): a new graph, owned by the library, whose rows hold only
 * the neighbours w of v with (d(w), w) > (d(v), v) -- edges from the
 * higher-degree end are dropped, ties broken by id -- in ascending id order.
 * It must be destroyed before g.  On an oriented graph:
 *  - agis_build_proposal_tables counts out-degrees, and C_v over pairs of
 *    out-neighbours, deciding adjacency in g;
 *  - agis_estimate / _batch / dump / learn accept clique patterns only
 *    (AGIS_E_UNSUPPORTED otherwise).  Each k-clique is reached by exactly
 *    one trajectory (its vertices in increasing order); the f_approx weight
 *    of a candidate counts the remaining clique vertices among its
 *    out-neighbours (|B| enters as 0), and agis_result.estimate = k! x the
 *    sample mean (embeddings), copies = the mean (cliques), variance scaled
 *    alike. */
int agis_orient(agis_ctx* ctx, const agis_graph* g, agis_graph** out);

/* The CSR of a graph: n, nnz and device pointers to its offsets and
 * neighbours (the caller's for agis_load_csr, the library's for
 * agis_orient; valid until the graph is destroyed).  Any output may be
 * NULL. */
int agis_graph_export(agis_ctx* ctx, const agis_graph* g, uint64_t* n, uint64_t* nnz, const uint64_t** off,
                      const uint32_t** nbr);

/* Builds the per-vertex proposal tables (Sec. 4.4): degree d(v), the
 * neighbour-degree sum S2(v) = sum_{x in N(v)} d(x), and the clustering
 * coefficient C_v estimated from d(v) trials (exact_cv = 0; each trial
 * draws an ordered pair of distinct neighbours from Philox key cv_seed) or
 * counted exactly (exact_cv = 1).  Stored in Q16 log2 form with log2 C_v
 * clamped below at lc_min_q16 (log2 of the paper's small nonzero constant;
 * -655360 = log2 2^-10).  The tables are owned by the library.
 * With them the library builds three search aids of the sampler (they
 * change no sample): neighbourhood bitmaps of the highest-degree vertices
 * (up to 1 GiB); the common-neighbour counts of every pair among the hubs
 * of highest degree (up to H = 8,192 of them, within a bounded build work),
 * which make a uniform step over the common neighbours of two such hubs a
 * table read plus a partial walk (8 counts per ordered pair, the total and
 * 7 running counts at eighths of the shorter list, H^2 x 8 x 4 B: at most
 * 2 GiB); and the common-neighbour lists themselves of every pair among
 * the C highest-degree of those hubs (the core; C <= 4,096, the lists
 * within 4 GiB and an eighth of the free memory), from which a step over
 * two core vertices starts.
 * The tables also keep, for later calls, the f_approx proposal tables that
 * estimates with them build (per step signature: per-vertex step weights,
 * per-row pick tables, pick tables over the core-pair lists, the
 * first-step table): at most 16 GiB, least
 * recently used first, released at a call that finds less than 128 GiB of
 * device memory free, and freed by agis_tables_destroy.  Tables built from
 * learned weights are rebuilt at every call (the caller may change them).
 * Calls that use one tables handle from several threads are serialised
 * while they prepare their tables. */
int agis_build_proposal_tables(agis_ctx* ctx, const agis_graph* g, uint64_t cv_seed, int32_t lc_min_q16,
                               int32_t exact_cv, agis_tables** out);
void agis_tables_destroy(agis_tables* t);

/* Copies the tables into caller device buffers (each of n entries; any may
 * be NULL): deg uint32, s2 uint64, hits uint64, trials uint64, la int32
 * (Q16 log2 of S2/d), lc int32 (Q16 log2 of C_v, clamped). */
int agis_tables_export(agis_ctx* ctx, const agis_tables* t, uint32_t* deg, uint64_t* s2, uint64_t* hits,
                       uint64_t* trials, int32_t* la, int32_t* lc);

/* Pattern compiler alone (host only, no GPU needed): matching order by
 * Algorithm 2 when order == NULL (host uint8[k] otherwise), auxiliary
 * arrays and decisions for params->mode / beta (params may be NULL:
 * SWITCH, beta = 4/5). */
int agis_compile_pattern(const agis_pattern* p, const uint8_t* order, const agis_run_params* params,
                         agis_plan* out);

/* Estimates C(G, P) (Algorithm 3 samples, Algorithm 1 statistics).
 * order: host uint8[k] or NULL for Algorithm 2.  With params->eps > 0 the
 * run stops at the first check where eps_hat <= eps (and n >= min_samples),
 * or returns AGIS_E_NOT_CONVERGED after n_samples samples (result filled);
 * with eps <= 0 exactly n_samples samples are drawn.  Samples use indices
 * 0, 1, 2, ... under `seed`. */
int agis_estimate(agis_ctx* ctx, const agis_graph* g, const agis_tables* t, const agis_pattern* p,
                  const uint8_t* order, uint64_t n_samples, uint64_t seed, const agis_run_params* params,
                  agis_result* out);

/* agis_estimate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the same
 * arguments, samples and result -- estimates equal agis_estimate's to
 * relative 1e-9 -- but no hipMalloc, hipFree or allocating library routine is
 * called.  Every buffer (first-step table, per-step weight tables, round
 * weights and partials, the waves' scratch) is carved from a fixed device
 * workspace of 256 MiB that the library holds on each GPU it runs on until
 * the process ends.  Per-row pick tables are not built (flags are treated as
 * AGIS_RUN_ROWTAB_OFF: the same samples), step weight tables that do not fit
 * fall back to the vertex records, and the grid shrinks to the waves whose
 * scratch (2 x (max degree + 1) x 4 bytes each) fits.  A graph whose
 * first-step table (12 bytes per vertex) or one workgroup's scratch does not
 * fit returns AGIS_E_UNSUPPORTED with the reason.  Calls that overlap on one
 * GPU share the workspace and race: serialise them.  Rounds are launched
 * directly (no graph replay). */
int agis_estimate_noalloc(agis_ctx* ctx, const agis_graph* g, const agis_tables* t, const agis_pattern* p,
                          const uint8_t* order, uint64_t n_samples, uint64_t seed, const agis_run_params* params,
                          agis_result* out);

/* Estimates C(G, P) for n_patterns (1..64) patterns at once, the way the
 * paper runs independent samplers in parallel (Sec. 5.4), with uneven
 * sample budgets: budgets[i] host uint64 per pattern.  Each round is one
 * persistent launch over all still-active patterns (replayed from a
 * captured HIP graph unless disabled by agis_set_launch): waves take
 * sample slots from a shared queue, so heavy and light patterns balance.
 * Pattern i uses Algorithm 2's order and pattern id params->pattern_id + i;
 * with params->eps > 0 each pattern stops at its own convergence (checks
 * every check_every of its samples) or at its budget, otherwise it runs
 * exactly its budget.  Every per-pattern result equals what agis_estimate
 * gives for that pattern alone (same samples, same stopping point;
 * estimates to relative 1e-9).  out: host agis_result[n_patterns].
 * Learned mode takes each pattern's tables from params->batch_learned.
 * Returns AGIS_E_NOT_CONVERGED (results filled) if any pattern did not
 * converge within its budget. */
int agis_estimate_batch(agis_ctx* ctx, const agis_graph* g, const agis_tables* t, uint32_t n_patterns,
                        const agis_pattern* patterns, const uint64_t* budgets, uint64_t seed,
                        const agis_run_params* params, agis_result* out);

/* Launch shape of the sampler for later calls on this context (results do
 * not depend on it): use_graphs = replay rounds from a captured HIP graph;
 * blocks_per_cu = resident 256-thread workgroups per compute unit (0 = as
 * many as fit; each holds 16 KB of LDS, the weight decoder's table); grab = sample slots a wave takes from the queue at a time
 * (0 = chosen from the round size, at most 1024); variant = register
 * budget of the sampling kernel (0, 1 and 2 = small enough for 6, 7 and 8
 * resident waves per SIMD; the smaller budgets spill a few registers);
 * hub_window: a high-degree vertex's neighbourhood bitmap (built with the
 * tables) replaces the merge with its list when the list is at least
 * hub_window / 64 times as long as the set it is intersected with (0 =
 * whenever there is a bitmap). */
int agis_set_launch(agis_ctx* ctx, int32_t use_graphs, int32_t blocks_per_cu, uint32_t grab, int32_t variant,
                    uint32_t hub_window);

/* Launch configuration chosen by agis_autotune. */
typedef struct {
    int32_t use_graphs;
    int32_t blocks_per_cu;
    uint32_t grab;
    int32_t variant;
    double seconds;          /* sampling-kernel time of the chosen configuration's pilot */
    double default_seconds;  /* the same pilot under the default configuration */
    uint32_t hub_window;
    uint32_t reserved;
} agis_tuning;

/* Times pilot batches (pilot_samples samples of each of the n_patterns
 * patterns, fixed budgets, params' mode and beta) under each candidate
 * launch configuration -- kernel register-budget variant (0, 1, 2) x queue
 * grab (1, 2, 4 slots), then the hub-bitmap window (256, 1024, 4096) --
 * and applies the fastest to the context (as agis_set_launch would); a
 * candidate must beat the best so far by 2% to be taken.  Results of later
 * calls do not depend on the choice. */
int agis_autotune(agis_ctx* ctx, const agis_graph* g, const agis_tables* t, uint32_t n_patterns,
                  const agis_pattern* patterns, uint64_t pilot_samples, const agis_run_params* params,
                  agis_tuning* out);

/* The first-step proposal of an estimate (Algorithm 3, first step; Sec.
 * 5.3 for the uniform case) as integer weights: vertex v is drawn with
 * probability q1[v] / *total.  A weighted first step gives the Q16-encoded
 * f_approx (or learned, or term-ablated) weights the sampler draws from;
 * a uniform one (edge-uniform) gives q1[v] = d(v), *total = nnz.  With the
 * exact rooted counts n_(v) of small graphs this yields the divergence of
 * each proposal from the ideal f_ideal(v | ()) = n_(v) / C(G, P), the
 * paper's analysis of the approximate distribution.  q1: device
 * uint32[n]; total: host. */
int agis_step1_weights(agis_ctx* ctx, const agis_graph* g, const agis_tables* t, const agis_pattern* p,
                       const uint8_t* order, const agis_run_params* params, uint32_t* q1, uint64_t* total);

/* Every connected graph on k vertices (2 <= k <= 6) up to isomorphism --
 * 1, 2, 6, 21 and 112 of them -- ordered by edge count, then by canonical
 * adjacency code; the set agis_concentrations takes.  *count receives the
 * number; out (host, cap entries) receives the patterns unless NULL. */
int agis_connected_patterns(uint32_t k, agis_pattern* out, uint32_t cap, uint32_t* count);

/* Concentrations of the connected k-vertex patterns (2 <= k <= 6), the
 * quantity the paper compares with MCMC estimators (Sec. 6.3, comparison
 * with MCMC): each pattern's count divided by the total over all
 * patterns of its size.  Host arrays of n_patterns entries; patterns must
 * be pairwise non-isomorphic, connected, of one size, and hold every
 * connected graph of that size with more edges than one of them (all of
 * them, normally).  copies: edge-induced counts (agis_result.copies).
 * Outputs (each may be NULL): conc_edge = copies / sum(copies); induced =
 * vertex-induced counts, from copies(H) = sum_G s(H, G) induced(G) over
 * the patterns G with at least H's edges, s(H, G) = the copies of H as a
 * spanning subgraph of G (solved from the most edges down); conc_induced =
 * induced / sum(induced).  No GPU work; no context. */
int agis_concentrations(uint32_t n_patterns, const agis_pattern* patterns, const double* copies, double* conc_edge,
                        double* induced, double* conc_induced);

/* Runs the samples whose indices are listed in idx (device uint64[m]) and
 * writes one agis_record per index into out (device, m records).  At most
 * 2^24 indices per call. */
int agis_dump_samples(agis_ctx* ctx, const agis_graph* g, const agis_tables* t, const agis_pattern* p,
                      const uint8_t* order, uint64_t seed, const agis_run_params* params, const uint64_t* idx,
                      uint64_t m, agis_record* out);

/* Memory requests of individual samples, for the roofline of the sampler
 * (the random-gather bound of Algorithm 3's steps): runs the samples listed
 * in idx (device uint64[m], at most 2^24) through the production paths of
 * the sampling kernel -- the same choices as agis_estimate with the same
 * params (pass AGIS_RUN_ROWTAB_ON or _OFF to match what the estimate used)
 * -- and writes per sample four counters into out (device uint64[m][4]):
 * bytes its global loads asked for, bytes its global stores wrote (the
 * wave's candidate scratch and the weight slot), the 64-byte segments those
 * accesses touched (an access spanning consecutive lanes counts each
 * segment once; the merge-free upper bound of the lines it moves), and its
 * wave-level memory requests.  LDS accesses are not counted. */
int agis_meter_samples(agis_ctx* ctx, const agis_graph* g, const agis_tables* t, const agis_pattern* p,
                       const uint8_t* order, uint64_t seed, const agis_run_params* params, const uint64_t* idx,
                       uint64_t m, uint64_t* out);

/* Random-gather microbenchmark (the ceiling the sampler's memory traffic is
 * measured against): waves_per_cu (4..32, a multiple of 4) resident waves
 * on every compute unit each run `rounds` rounds; in a round every group of
 * seg_bytes / 16 lanes reads one random seg_bytes-aligned segment of
 * seg_bytes bytes (one 16-byte word per lane; seg_bytes 4 or 8: every lane
 * one item) from buffer (device, `bytes` bytes, 16-byte aligned, >= 1 KiB;
 * its contents only steer the dependent chains).  dependent = 0: addresses
 * from a counter, up to 8 reads in flight per lane; dependent = 1: each
 * read's address depends on the previous read's value (a chain of
 * dependent loads, like a search).  seg_bytes: a power of two in [4, 1024].
 * sink: device, 8 KiB (folded values, never read back).  *seconds: kernel
 * time (HIP events on the context's stream); *useful_bytes: bytes read. */
int agis_gather_bench(agis_ctx* ctx, const void* buffer, uint64_t bytes, uint32_t seg_bytes, int32_t dependent,
                      uint32_t waves_per_cu, uint32_t rounds, uint64_t seed, void* sink, double* seconds,
                      double* useful_bytes);

/* ---- Learned proposal ------------------------------------------------
 * A small MLP predicts, for a vertex v and the position of a weighted
 * step, the log2 of the number of successful extensions when v is picked
 * there -- the quantity the ideal distribution is proportional to
 * (Theorem 1, Sec. 4.1).  It is trained on extension counts estimated by
 * the sampler itself and its predictions become Q16 log2 pick tables
 * (AGIS_MODE_LEARNED); the importance factors keep the estimate unbiased
 * (Theorem 2) whatever the network predicts.
 * Network: x (8) -> 64 GELU -> 64 GELU -> 1, GELU(a) = a Phi(a) (exact erf
 * form).  x = (log2(1 + d(v)), log2(1 + S2(v)), log2(1 + C_v C(d(v), 2)),
 * log2(1 + h(v))) and a one-hot of the step position class {1, 2, 3, >= 4},
 * where h(v) = largest h with at least h neighbours of degree >= h (an
 * upper bound of the core number).  Parameters: float[4801] =
 * W1[64][8], b1[64], W2[64][64] (W2[j][i]: output j, input i), b2[64],
 * w3[64], b3. */
int agis_mlp_param_count(void);

/* Per-vertex features into feats (device float[n][4], the 4 scalars above). */
int agis_features(agis_ctx* ctx, const agis_tables* t, float* feats);

/* Training targets: runs samples 0..n_samples-1 of the pattern (mode and
 * beta from params) and, for every step i of each sample, adds to
 * sums[i][v_i] (device double[k][n]) the product of the factors of the
 * steps after i -- an unbiased estimate of the successful extensions of
 * the prefix ending at v_i, 0 when the sample failed later -- and 1 to
 * counts[i][v_i] (device uint32[k][n]).  Both are cleared first.  The sums
 * use FP64 atomics, so their last bits depend on the order of arrival. */
int agis_learn_targets(agis_ctx* ctx, const agis_graph* g, const agis_tables* t, const agis_pattern* p,
                       const uint8_t* order, uint64_t n_samples, uint64_t seed, const agis_run_params* params,
                       double* sums, uint32_t* counts);

/* Training rows from targets: for every step i in step_mask (bit i) and
 * every vertex v with counts[i][v] >= min_count (and >= 1), one row (vtx v,
 * cls = position class min(i, 3), target log2(1 + sums/counts), weight
 * counts), steps ascending then vertices ascending.  sums/counts: device,
 * as written by agis_learn_targets (k steps, n vertices); base: NULL, or
 * device int32[k][n] Q16 log weights the network corrects (residual
 * targets: rows whose base is the certain-zero marker are skipped; with
 * B = 2^(base / 2^16) and, per step, kappa = sum(sums) / sum(counts * B)
 * over the kept rows (1 if either sum is 0), the row target becomes
 * log2((sums / (kappa B) + 1) / (counts + 1)), i.e. the mean completion
 * count with kappa B as one pseudo-observation, relative to kappa B);
 * outputs: device
 * arrays of capacity k * n; *rows (host) receives the row count. */
int agis_learn_rows(agis_ctx* ctx, const double* sums, const uint32_t* counts, uint32_t k, uint64_t n,
                    uint32_t step_mask, uint32_t min_count, const int32_t* base, uint32_t* vtx, uint8_t* cls,
                    float* target, float* weight, uint64_t* rows);

/* Gradient of L = sum_r w_r (y_r - target_r)^2 / weight_sum over `rows`
 * training rows (device arrays: vtx uint32, cls uint8 position class,
 * target float, weight float; feats from agis_features) at `params`
 * (device float[4801]), in FP32 with a fixed summation order.  grad:
 * device float[4801]; loss: device float[1] or NULL. */
int agis_mlp_grad(agis_ctx* ctx, const float* params, const float* feats, const uint32_t* vtx, const uint8_t* cls,
                  const float* target, const float* weight, uint64_t rows, float weight_sum, float* grad, float* loss);

/* Adam (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on minibatches
 * of `batch` rows of a per-epoch shuffle (host generator seeded with
 * shuffle_seed), for `epochs` epochs; updates params in place.
 * loss_per_epoch: host float[epochs] or NULL. */
int agis_mlp_train(agis_ctx* ctx, float* params, const float* feats, const uint32_t* vtx, const uint8_t* cls,
                   const float* target, const float* weight, uint64_t rows, uint32_t epochs, uint32_t batch,
                   float lr, uint64_t shuffle_seed, float* loss_per_epoch);

/* f_approx Q16 log2 weight (Eq. probability_function in the library's
 * integer encoding) of every vertex for a step signature (b, f1, ie, f2),
 * INT32_MIN where d(v) - b < f1.  out: device int32[n]. */
int agis_step_log_weights(agis_ctx* ctx, const agis_tables* t, uint32_t b, uint32_t f1, uint32_t ie, uint32_t f2,
                          int32_t* out);

/* Inference for every vertex at one position class (0..3): BF16 matrix-core
 * products with FP32 accumulation for the 64 x 64 layer, FP32 elsewhere.
 * lt: device int32[n] = round(2^16 y), the Q16 log2 pick table consumed by
 * AGIS_MODE_LEARNED (certain zeros are still decided by degree at pick
 * time), or base[v] + round(2^16 y) when base (device int32[n], e.g. the
 * step's agis_step_log_weights) is given -- a learned correction of
 * f_approx; the output is first clamped to [y_min, y_max] (e.g. the range
 * of the training targets, against extrapolation to unseen degrees;
 * -INFINITY and INFINITY for none); y: device float[n] (the unclamped
 * output) or NULL. */
int agis_mlp_infer(agis_ctx* ctx, const float* params, const float* feats, uint64_t n, uint32_t position_class,
                   const int32_t* base, float y_min, float y_max, int32_t* lt, float* y);

/* Host copies of the library's Q16 tables (4096 entries each), its Philox
 * block function and its bounded draw -- for host-side tests. */
int agis_fixed_point_tables(int32_t* logtab, uint32_t* exp2tab);
int agis_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

#ifdef __cplusplus
}
#endif

#endif /* AGIS_H */
