/*
 * AGIS CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, single-threaded, deliberately unoptimised implementation of the
 * structure-informed neighbour sampler of the paper (Algorithm 3,
 * "Structure-Informed Neighbor Sampling"), its proposal tables
 * (Sec. 4.4 "Preprocessing Data Graphs"), the approximate extension count
 * (Eq. probability_function, Sec. 4.2.3) and the estimator statistics of
 * Algorithm 1 ("Online Convergence Detection").  It exists so that the GPU
 * library can be checked against it sample by sample.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the GPU
 * library never links or calls it, and it shares no code with the library.
 *
 * Conventions fixed by this implementation (the paper leaves them open):
 *  - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 *    random numbers: as easy as 1, 2, 3", SC'11), counter
 *    (c0, c1, c2, attempt<<4 | tag), key = 64-bit seed.  A bounded draw in
 *    [0, range) uses Lemire's multiply-and-reject method ("Fast random
 *    integer generation in an interval", ACM TOMACS 2019) on the 64-bit word
 *    (out[1]<<32 | out[0]); a rejected attempt moves to attempt+1.
 *  - Sampling draw of step i (0-based) of sample s for pattern id p:
 *    c0 = s & 0xffffffff, c1 = s >> 32, c2 = p, tag = i.
 *  - Clustering-coefficient trial t of vertex v: c0 = v, c1 = t, c2 = 0,
 *    tag 0 for the first neighbour position, tag 1 for the second.
 *  - Proposal weights are integers computed in a Q16 fixed-point log2
 *    domain (see log2fx and weight_from_log below), so that the sampler's
 *    choices are exactly reproducible; unbiasedness (Theorem 2) is kept
 *    because the importance factor uses the same integer weights.
 */

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXK 8
#define ORC_CERTAIN_ZERO INT32_MIN

/* ------------------------------------------------------------------ */
/* Philox4x32-10, written from the round function published in SC'11. */
/* ------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        uint32_t n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

static uint64_t orc_word64(const uint32_t key[2], uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag,
                           uint32_t attempt) {
    uint32_t ctr[4] = {c0, c1, c2, (attempt << 4) | (tag & 0xFu)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return ((uint64_t)out[1] << 32) | (uint64_t)out[0];
}

/* Uniform integer in [0, range), range >= 1. */
uint64_t orc_bounded(const uint32_t key[2], uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag, uint64_t range) {
    uint64_t threshold = (0 - range) % range; /* 2^64 mod range */
    for (uint32_t attempt = 0;; ++attempt) {
        uint64_t x = orc_word64(key, c0, c1, c2, tag, attempt);
        unsigned __int128 m = (unsigned __int128)x * (unsigned __int128)range;
        uint64_t low = (uint64_t)m;
        if (low >= threshold) return (uint64_t)(m >> 64);
    }
}

/* ------------------------------------------------------------------ */
/* Q16 fixed-point log2 / exp2                                          */
/* ------------------------------------------------------------------ */

static int32_t LOGTAB[4096];
static uint32_t EXP2TAB[4096];
static int tables_ready = 0;

static void init_fixed_point(void) {
    if (tables_ready) return;
    for (int j = 0; j < 4096; ++j) {
        LOGTAB[j] = (int32_t)llround(65536.0 * log2(1.0 + (double)j / 4096.0));
        EXP2TAB[j] = (uint32_t)llround(2147483648.0 * exp2(-(double)j / 4096.0));
    }
    tables_ready = 1;
}

void orc_fixed_point_tables(int32_t* logtab, uint32_t* exp2tab) {
    init_fixed_point();
    memcpy(logtab, LOGTAB, sizeof(LOGTAB));
    memcpy(exp2tab, EXP2TAB, sizeof(EXP2TAB));
}

/* log2(x) in Q16 for x >= 1: integer part from the leading bit, fraction
 * from a 4096-entry table indexed by the next 12 bits. */
int32_t orc_log2fx(uint64_t x) {
    init_fixed_point();
    int p = 63 - __builtin_clzll(x);
    uint32_t m;
    if (p >= 12)
        m = (uint32_t)((x >> (p - 12)) & 0xFFFu);
    else
        m = (uint32_t)((x << (12 - p)) & 0xFFFu);
    return (int32_t)(p << 16) + LOGTAB[m];
}

/* Integer pick weight of a candidate whose log weight is lw, when the
 * largest log weight among the candidates is lmax: 2^31 * 2^((lw-lmax)/2^16),
 * rounded down through the table, never below 1. */
uint32_t orc_weight_from_log(int32_t lmax, int32_t lw) {
    init_fixed_point();
    uint32_t delta = (uint32_t)(lmax - lw);
    uint32_t sh = delta >> 16;
    uint32_t fr = (delta & 0xFFFFu) >> 4;
    uint32_t q = sh >= 32 ? 0u : (EXP2TAB[fr] >> sh);
    return q < 1u ? 1u : q;
}

/* ------------------------------------------------------------------ */
/* Graph and per-vertex proposal tables (Sec. 4.4)                      */
/* ------------------------------------------------------------------ */

typedef struct {
    uint64_t n, nnz;
    const uint64_t* off;
    const uint32_t* nbr;
} orc_graph;

typedef struct {
    const uint32_t* deg;
    const uint64_t* s2;    /* sum of neighbour degrees */
    const int32_t* la;     /* log2 average neighbour degree, Q16 */
    const int32_t* lc;     /* log2 clustering coefficient, Q16, clamped */
} orc_tables;

static int contains(const uint32_t* list, uint64_t len, uint32_t x) {
    uint64_t lo = 0, hi = len;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (list[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < len && list[lo] == x;
}

/* Table entries of vertex v (Sec. 4.4): degree, S2 = sum of the neighbour
 * degrees, the C_v trials (hits out of trials) and the Q16 logs LA and LC.
 * exact_cv = 1: hits = number of edges among N(v), trials = C(d, 2).
 * exact_cv = 0: d(v) sampled ordered pairs of distinct neighbours. */
static void tables_of_vertex(const uint64_t* off, const uint32_t* nbr, const uint64_t* aoff, const uint32_t* anbr,
                             uint64_t v, const uint32_t key[2], int32_t lc_min, int exact_cv, uint32_t* deg_v,
                             uint64_t* s2_v, uint64_t* hits_v, uint64_t* trials_v, int32_t* la_v, int32_t* lc_v) {
    uint64_t d = off[v + 1] - off[v];
    const uint32_t* row = nbr + off[v];
    uint64_t s = 0;
    for (uint64_t e = 0; e < d; ++e) s += off[row[e] + 1] - off[row[e]];
    uint64_t h = 0, t = 0;
    if (d >= 2) {
        if (exact_cv) {
            for (uint64_t a = 0; a < d; ++a) {
                const uint32_t* ra = anbr + aoff[row[a]];
                uint64_t da = aoff[row[a] + 1] - aoff[row[a]];
                for (uint64_t b = a + 1; b < d; ++b)
                    if (contains(ra, da, row[b])) ++h;
            }
            t = d * (d - 1) / 2;
        } else {
            for (uint64_t trial = 0; trial < d; ++trial) {
                uint64_t a = orc_bounded(key, (uint32_t)v, (uint32_t)trial, 0, 0, d);
                uint64_t b = orc_bounded(key, (uint32_t)v, (uint32_t)trial, 0, 1, d - 1);
                if (b >= a) ++b;
                uint32_t x = row[a], y = row[b];
                if (contains(anbr + aoff[x], aoff[x + 1] - aoff[x], y)) ++h;
            }
            t = d;
        }
    }
    *deg_v = (uint32_t)d;
    *s2_v = s;
    *hits_v = h;
    *trials_v = t;
    /* log2(S2 / d) is undefined at S2 = 0, which only an oriented graph has
     * (out-neighbours without out-neighbours): 0 there, as for d = 0 */
    *la_v = (d >= 1 && s > 0) ? orc_log2fx(s) - orc_log2fx(d) : 0;
    if (d < 2 || h == 0) {
        *lc_v = lc_min;
    } else {
        int32_t c = orc_log2fx(h) - orc_log2fx(t);
        *lc_v = c > lc_min ? c : lc_min;
    }
}

/* Fills deg, s2, hits, trials, la, lc for every vertex. */
void orc_build_tables(const uint64_t* off, const uint32_t* nbr, uint64_t n, uint32_t cv_seed_lo,
                      uint32_t cv_seed_hi, int32_t lc_min, int exact_cv, uint32_t* deg, uint64_t* s2,
                      uint64_t* hits, uint64_t* trials, int32_t* la, int32_t* lc) {
    init_fixed_point();
    uint32_t key[2] = {cv_seed_lo, cv_seed_hi};
    for (uint64_t v = 0; v < n; ++v)
        tables_of_vertex(off, nbr, off, nbr, v, key, lc_min, exact_cv, &deg[v], &s2[v], &hits[v], &trials[v], &la[v],
                         &lc[v]);
}

/* The same for an oriented graph (off, nbr: out-neighbours), with the
 * adjacency of two out-neighbours decided in the undirected graph (aoff,
 * anbr). */
void orc_build_tables_oriented(const uint64_t* off, const uint32_t* nbr, uint64_t n, const uint64_t* aoff,
                               const uint32_t* anbr, uint32_t cv_seed_lo, uint32_t cv_seed_hi, int32_t lc_min,
                               int exact_cv, uint32_t* deg, uint64_t* s2, uint64_t* hits, uint64_t* trials, int32_t* la,
                               int32_t* lc) {
    init_fixed_point();
    uint32_t key[2] = {cv_seed_lo, cv_seed_hi};
    for (uint64_t v = 0; v < n; ++v)
        tables_of_vertex(off, nbr, aoff, anbr, v, key, lc_min, exact_cv, &deg[v], &s2[v], &hits[v], &trials[v],
                         &la[v], &lc[v]);
}

/* Degree orientation (the DAG of the clique optimisation): keep v -> w iff
 * (d(v), v) < (d(w), w).  off_out: n + 1 entries; nbr_out: capacity nnz / 2;
 * rows stay in ascending id order.  Returns the number of kept edges. */
uint64_t orc_orient(const uint64_t* off, const uint32_t* nbr, uint64_t n, uint64_t* off_out, uint32_t* nbr_out) {
    uint64_t p = 0;
    off_out[0] = 0;
    for (uint64_t v = 0; v < n; ++v) {
        uint64_t dv = off[v + 1] - off[v];
        for (uint64_t e = off[v]; e < off[v + 1]; ++e) {
            uint32_t w = nbr[e];
            uint64_t dw = off[w + 1] - off[w];
            if (dv < dw || (dv == dw && v < w)) nbr_out[p++] = w;
        }
        off_out[v + 1] = p;
    }
    return p;
}

/* The same entries for the listed vertices only (entry j for vs[j]), for
 * graphs whose whole table takes the oracle too long. */
void orc_tables_at(const uint64_t* off, const uint32_t* nbr, const uint64_t* vs, uint64_t count, uint32_t cv_seed_lo,
                   uint32_t cv_seed_hi, int32_t lc_min, int exact_cv, uint32_t* deg, uint64_t* s2, uint64_t* hits,
                   uint64_t* trials, int32_t* la, int32_t* lc) {
    init_fixed_point();
    uint32_t key[2] = {cv_seed_lo, cv_seed_hi};
    for (uint64_t j = 0; j < count; ++j)
        tables_of_vertex(off, nbr, off, nbr, vs[j], key, lc_min, exact_cv, &deg[j], &s2[j], &hits[j], &trials[j],
                         &la[j], &lc[j]);
}

/* ------------------------------------------------------------------ */
/* Compiled pattern plan (produced by the Python pattern compiler)      */
/* ------------------------------------------------------------------ */

typedef struct {
    uint32_t k;
    uint32_t pattern_id;
    uint8_t bmask[ORC_MAXK];    /* bit j: position j (< i) is joined to position i */
    uint8_t f1[ORC_MAXK];       /* |F1| */
    uint8_t ie[ORC_MAXK];       /* |I_effective| */
    uint8_t f2[ORC_MAXK];       /* |F2| */
    uint8_t decision[ORC_MAXK]; /* D(i): 1 = f_approx / learned, 0 = f_uniform */
    uint8_t oriented;           /* 1: sampling a clique on the degree-oriented graph */
} orc_plan;

/* A step draws from weights when it is an f_approx step with forward
 * structure; with |F1| = 0 every candidate has weight C(d-b, 0) = 1, so the
 * step is a uniform draw and is executed as one. */
static int step_weighted(const orc_plan* P, int i) { return P->decision[i] && P->f1[i] > 0; }

/* Log weight (Q16) of candidate v at step i, or ORC_CERTAIN_ZERO when v
 * cannot extend to an embedding because d(v) - |B| < |F1|.
 * lt: learned log-weight table for this step (NULL = f_approx). */
static int32_t log_weight(const orc_tables* T, const orc_plan* P, int i, uint32_t v, const int32_t* lt) {
    /* on the oriented graph no backward vertex is an out-neighbour of v:
     * all d(v) out-neighbours are open to the later clique vertices */
    uint32_t b = P->oriented ? 0u : (uint32_t)__builtin_popcount(P->bmask[i]);
    uint32_t d = T->deg[v];
    uint32_t f1 = P->f1[i];
    if (d < b + f1) return ORC_CERTAIN_ZERO;
    if (lt) return lt[v];
    int32_t l = 0;
    for (uint32_t t = 0; t < f1; ++t) l += orc_log2fx((uint64_t)(d - b - t));  /* T[F1] = C(d-b, f1) * f1! */
    /* (a term with a zero exponent is 1: its table is not read) */
    if (P->ie[i]) l += (int32_t)P->ie[i] * T->lc[v]; /* T[I1] = C_v^|I_eff| */
    if (P->f2[i]) l += (int32_t)P->f2[i] * T->la[v]; /* T[F2] = (S2/d)^|F2| */
    return l;
}

/* f_approx log weight of every vertex at step i (certain zeros marked), the
 * base a learned correction is added to. */
void orc_log_weights(const orc_tables* T, const orc_plan* P, int i, uint64_t n, int32_t* out) {
    for (uint64_t v = 0; v < n; ++v) out[v] = log_weight(T, P, i, (uint32_t)v, NULL);
}

/* Step-1 proposal over the whole vertex set: fills q1[v] and the inclusive
 * prefix pre1[v]; returns the total. */
uint64_t orc_step1_table(const orc_graph* G, const orc_tables* T, const orc_plan* P, const int32_t* lt,
                         uint32_t* q1, uint64_t* pre1) {
    int32_t lmax = ORC_CERTAIN_ZERO;
    for (uint64_t v = 0; v < G->n; ++v) {
        int32_t l = log_weight(T, P, 0, (uint32_t)v, lt);
        if (l != ORC_CERTAIN_ZERO && l > lmax) lmax = l;
    }
    uint64_t run = 0;
    for (uint64_t v = 0; v < G->n; ++v) {
        int32_t l = log_weight(T, P, 0, (uint32_t)v, lt);
        uint32_t q = (l == ORC_CERTAIN_ZERO) ? 0u : orc_weight_from_log(lmax, l);
        q1[v] = q;
        run += q;
        pre1[v] = run;
    }
    return run;
}

/* ------------------------------------------------------------------ */
/* One sample (Algorithm 3)                                             */
/* ------------------------------------------------------------------ */

typedef struct {
    uint32_t v[ORC_MAXK];
    uint64_t num[ORC_MAXK];
    uint64_t den[ORC_MAXK];
    double x;
    int32_t steps;      /* number of steps that picked a vertex */
    int32_t fail_step;  /* -1 on success, else the step whose candidate set was empty */
} orc_record;

typedef struct {
    const orc_graph* G;
    const orc_tables* T;
    const orc_plan* P;
    const int32_t* const* lt;  /* per-step learned tables, or NULL */
    const uint32_t* q1;
    const uint64_t* pre1;
    uint64_t Q1;
    uint32_t key[2];
    uint32_t* cand;   /* scratch, >= max degree entries */
    int32_t* candl;   /* scratch, >= max degree entries */
} orc_sampler;

static const int32_t* step_lt(const orc_sampler* S, int i) { return S->lt ? S->lt[i] : NULL; }

/* Candidate set of step i >= 1: the intersection I of the neighbour lists of
 * the matched backward vertices, in ascending id order.  Writes I into
 * cand (the caller removes already-matched vertices).  Returns |I|. */
static uint64_t intersect_backward(const orc_sampler* S, int i, const uint32_t* tau) {
    const orc_graph* G = S->G;
    uint8_t bm = S->P->bmask[i];
    int j0 = __builtin_ctz(bm);
    uint32_t base = tau[j0];
    uint64_t cnt = 0;
    for (uint64_t e = G->off[base]; e < G->off[base + 1]; ++e) {
        uint32_t x = G->nbr[e];
        int all = 1;
        for (int j = j0 + 1; j < i; ++j) {
            if (!(bm >> j & 1)) continue;
            uint32_t w = tau[j];
            if (!contains(G->nbr + G->off[w], G->off[w + 1] - G->off[w], x)) { all = 0; break; }
        }
        if (all) S->cand[cnt++] = x;
    }
    return cnt;
}

static int in_tau(const uint32_t* tau, int i, uint32_t x) {
    for (int j = 0; j < i; ++j)
        if (tau[j] == x) return 1;
    return 0;
}

double orc_sample_one(const orc_sampler* S, uint64_t s, orc_record* rec) {
    const orc_graph* G = S->G;
    const orc_plan* P = S->P;
    uint32_t c0 = (uint32_t)s, c1 = (uint32_t)(s >> 32), c2 = P->pattern_id;
    uint32_t tau[ORC_MAXK];
    uint64_t num[ORC_MAXK], den[ORC_MAXK];
    double x = 1.0;
    int fail = -1;
    int i;
    for (i = 0; i < (int)P->k; ++i) {
        if (i == 0) {
            if (step_weighted(P, 0)) {
                if (S->Q1 == 0) { fail = 0; break; }
                uint64_t r = orc_bounded(S->key, c0, c1, c2, 0, S->Q1);
                uint64_t lo = 0, hi = G->n; /* first v with pre1[v] > r */
                while (lo < hi) {
                    uint64_t mid = lo + (hi - lo) / 2;
                    if (S->pre1[mid] > r) hi = mid; else lo = mid + 1;
                }
                tau[0] = (uint32_t)lo;
                num[0] = S->Q1;
                den[0] = S->q1[lo];
            } else {
                if (G->nnz == 0) { fail = 0; break; }
                uint64_t r = orc_bounded(S->key, c0, c1, c2, 0, G->nnz);
                uint64_t lo = 0, hi = G->n; /* first v with off[v+1] > r */
                while (lo < hi) {
                    uint64_t mid = lo + (hi - lo) / 2;
                    if (G->off[mid + 1] > r) hi = mid; else lo = mid + 1;
                }
                tau[0] = (uint32_t)lo;
                num[0] = G->nnz;
                den[0] = G->off[lo + 1] - G->off[lo];
            }
            x = (double)num[0] / (double)den[0];
            continue;
        }
        uint64_t isize = intersect_backward(S, i, tau);
        if (step_weighted(P, i)) {
            const int32_t* lt = step_lt(S, i);
            int32_t lmax = ORC_CERTAIN_ZERO;
            for (uint64_t c = 0; c < isize; ++c) {
                int32_t l = log_weight(S->T, P, i, S->cand[c], lt);
                S->candl[c] = l;
                if (l != ORC_CERTAIN_ZERO && l > lmax) lmax = l;
            }
            uint64_t Q = 0;
            for (uint64_t c = 0; c < isize; ++c) {
                if (in_tau(tau, i, S->cand[c]) || S->candl[c] == ORC_CERTAIN_ZERO) continue;
                Q += orc_weight_from_log(lmax, S->candl[c]);
            }
            if (Q == 0) { fail = i; break; }
            uint64_t r = orc_bounded(S->key, c0, c1, c2, (uint32_t)i, Q);
            uint64_t run = 0;
            uint32_t pick = 0, qpick = 0;
            for (uint64_t c = 0; c < isize; ++c) {
                if (in_tau(tau, i, S->cand[c]) || S->candl[c] == ORC_CERTAIN_ZERO) continue;
                uint32_t q = orc_weight_from_log(lmax, S->candl[c]);
                run += q;
                if (run > r) { pick = S->cand[c]; qpick = q; break; }
            }
            tau[i] = pick;
            num[i] = Q;
            den[i] = qpick;
        } else {
            uint64_t m = 0;
            for (uint64_t c = 0; c < isize; ++c)
                if (!in_tau(tau, i, S->cand[c])) S->cand[m++] = S->cand[c];
            if (m == 0) { fail = i; break; }
            uint64_t r = orc_bounded(S->key, c0, c1, c2, (uint32_t)i, m);
            tau[i] = S->cand[r];
            num[i] = m;
            den[i] = 1;
        }
        x = x * ((double)num[i] / (double)den[i]);
    }
    if (fail >= 0) x = 0.0;
    if (rec) {
        memset(rec, 0, sizeof(*rec));
        for (int j = 0; j < i && j < ORC_MAXK; ++j) {
            rec->v[j] = tau[j];
            rec->num[j] = num[j];
            rec->den[j] = den[j];
        }
        rec->x = x;
        rec->steps = i;
        rec->fail_step = fail;
    }
    return x;
}

static uint64_t max_degree(const orc_graph* G) {
    uint64_t m = 0;
    for (uint64_t v = 0; v < G->n; ++v) {
        uint64_t d = G->off[v + 1] - G->off[v];
        if (d > m) m = d;
    }
    return m;
}

typedef struct {
    uint64_t n;
    double mean;
    double m2;
    uint64_t nonzero;
} orc_stats;

/* Shared setup of the public entry points below. */
static int make_sampler(orc_sampler* S, orc_graph* G, orc_tables* T, const orc_plan* P, const uint64_t* off,
                        const uint32_t* nbr, uint64_t n, uint64_t nnz, const uint32_t* deg, const uint64_t* s2,
                        const int32_t* la, const int32_t* lc, const int32_t* const* lt, const uint32_t* q1,
                        const uint64_t* pre1, uint64_t Q1, uint64_t seed) {
    init_fixed_point();
    G->n = n; G->nnz = nnz; G->off = off; G->nbr = nbr;
    T->deg = deg; T->s2 = s2; T->la = la; T->lc = lc;
    S->G = G; S->T = T; S->P = P; S->lt = lt;
    S->q1 = q1; S->pre1 = pre1; S->Q1 = Q1;
    S->key[0] = (uint32_t)seed; S->key[1] = (uint32_t)(seed >> 32);
    uint64_t md = max_degree(G) + 1;
    S->cand = (uint32_t*)malloc(md * sizeof(uint32_t));
    S->candl = (int32_t*)malloc(md * sizeof(int32_t));
    return (S->cand && S->candl) ? 0 : -1;
}

static void free_sampler(orc_sampler* S) {
    free(S->cand);
    free(S->candl);
}

/* Runs samples [start, start+count) in index order: Welford accumulation
 * into *st (which may already hold earlier samples); optional per-sample
 * outputs xs (count doubles) and records recs (count records). */
int orc_run(const uint64_t* off, const uint32_t* nbr, uint64_t n, uint64_t nnz, const uint32_t* deg,
            const uint64_t* s2, const int32_t* la, const int32_t* lc, const orc_plan* P,
            const int32_t* const* lt, const uint32_t* q1, const uint64_t* pre1, uint64_t Q1, uint64_t seed,
            uint64_t start, uint64_t count, orc_stats* st, double* xs, orc_record* recs) {
    orc_graph G; orc_tables T; orc_sampler S;
    if (make_sampler(&S, &G, &T, P, off, nbr, n, nnz, deg, s2, la, lc, lt, q1, pre1, Q1, seed)) return -1;
    for (uint64_t j = 0; j < count; ++j) {
        double xv = orc_sample_one(&S, start + j, recs ? &recs[j] : NULL);
        if (xs) xs[j] = xv;
        st->n += 1;
        double d = xv - st->mean;
        st->mean += d / (double)st->n;
        st->m2 += d * (xv - st->mean);
        if (xv != 0.0) st->nonzero += 1;
    }
    free_sampler(&S);
    return 0;
}

/* Same as orc_run but for an explicit list of sample indices. */
int orc_run_indices(const uint64_t* off, const uint32_t* nbr, uint64_t n, uint64_t nnz, const uint32_t* deg,
                    const uint64_t* s2, const int32_t* la, const int32_t* lc, const orc_plan* P,
                    const int32_t* const* lt, const uint32_t* q1, const uint64_t* pre1, uint64_t Q1,
                    uint64_t seed, const uint64_t* idx, uint64_t count, orc_record* recs) {
    orc_graph G; orc_tables T; orc_sampler S;
    if (make_sampler(&S, &G, &T, P, off, nbr, n, nnz, deg, s2, la, lc, lt, q1, pre1, Q1, seed)) return -1;
    for (uint64_t j = 0; j < count; ++j) orc_sample_one(&S, idx[j], &recs[j]);
    free_sampler(&S);
    return 0;
}

/* Distribution of step i given the matched prefix tau[0..i-1], as the
 * sampler would draw it: candidates in draw order and their integer
 * weights.  Step 0 lists every vertex (weights q1 when weighted, else d(v),
 * i.e. edge-uniform).  Returns the number of candidates written. */
uint64_t orc_step_distribution(const uint64_t* off, const uint32_t* nbr, uint64_t n, uint64_t nnz,
                               const uint32_t* deg, const uint64_t* s2, const int32_t* la, const int32_t* lc,
                               const orc_plan* P, const int32_t* const* lt, const uint32_t* q1, int i,
                               const uint32_t* tau, uint32_t* out_v, uint64_t* out_w) {
    orc_graph G; orc_tables T; orc_sampler S;
    if (make_sampler(&S, &G, &T, P, off, nbr, n, nnz, deg, s2, la, lc, lt, q1, NULL, 0, 0)) return 0;
    uint64_t m = 0;
    if (i == 0) {
        for (uint64_t v = 0; v < n; ++v) {
            out_v[m] = (uint32_t)v;
            out_w[m] = step_weighted(P, 0) ? q1[v] : (off[v + 1] - off[v]);
            ++m;
        }
    } else {
        uint64_t isize = intersect_backward(&S, i, tau);
        int32_t lmax = ORC_CERTAIN_ZERO;
        const int32_t* l_t = step_lt(&S, i);
        if (step_weighted(P, i)) {
            for (uint64_t c = 0; c < isize; ++c) {
                int32_t l = log_weight(&T, P, i, S.cand[c], l_t);
                S.candl[c] = l;
                if (l != ORC_CERTAIN_ZERO && l > lmax) lmax = l;
            }
        }
        for (uint64_t c = 0; c < isize; ++c) {
            if (in_tau(tau, i, S.cand[c])) continue;
            out_v[m] = S.cand[c];
            if (step_weighted(P, i))
                out_w[m] = S.candl[c] == ORC_CERTAIN_ZERO ? 0 : orc_weight_from_log(lmax, S.candl[c]);
            else
                out_w[m] = 1;
            ++m;
        }
    }
    free_sampler(&S);
    return m;
}

/* ------------------------------------------------------------------ */
/* Literal real-valued f_approx (Eq. probability_function), for pins     */
/* and for measuring what the integer encoding costs in variance.       */
/* ------------------------------------------------------------------ */

static double binom_real(double nn, int k) {
    if (nn < k) return 0.0;
    double r = 1.0;
    for (int t = 0; t < k; ++t) r = r * (nn - t) / (double)(t + 1);
    return r;
}

/* The three terms of Eq. probability_function for a vertex of degree d,
 * clustering coefficient cv and neighbour-degree sum s2. */
void orc_literal_terms(uint64_t d, uint32_t b, uint32_t f1, uint32_t ie, uint32_t f2, double cv, uint64_t s2,
                       double* t_f1, double* t_i1, double* t_f2) {
    *t_f1 = binom_real((double)d - (double)b, (int)f1);
    *t_i1 = pow(cv, (double)ie);
    *t_f2 = d ? pow((double)s2 / (double)d, (double)f2) : 0.0;
}

/* Literal weights of step i for the candidates of the given prefix, with a
 * per-vertex clustering coefficient array cv (e.g. the exact one).  Same
 * candidate order as orc_step_distribution; uniform steps get weight 1,
 * and step 0 when not weighted gets d(v). */
uint64_t orc_step_distribution_literal(const uint64_t* off, const uint32_t* nbr, uint64_t n, uint64_t nnz,
                                       const uint32_t* deg, const uint64_t* s2, const double* cv,
                                       const orc_plan* P, int i, const uint32_t* tau, uint32_t* out_v,
                                       double* out_w) {
    orc_graph G; orc_tables T; orc_sampler S;
    if (make_sampler(&S, &G, &T, P, off, nbr, n, nnz, deg, s2, NULL, NULL, NULL, NULL, NULL, 0, 0)) return 0;
    uint32_t b = P->oriented ? 0u : (uint32_t)__builtin_popcount(P->bmask[i]);
    uint64_t m = 0;
    if (i == 0) {
        for (uint64_t v = 0; v < n; ++v) {
            out_v[m] = (uint32_t)v;
            if (step_weighted(P, 0)) {
                double a, c, e;
                orc_literal_terms(deg[v], 0, P->f1[0], P->ie[0], P->f2[0], cv[v], s2[v], &a, &c, &e);
                out_w[m] = a * c * e;
            } else {
                out_w[m] = (double)deg[v];
            }
            ++m;
        }
    } else {
        uint64_t isize = intersect_backward(&S, i, tau);
        for (uint64_t c = 0; c < isize; ++c) {
            uint32_t v = S.cand[c];
            if (in_tau(tau, i, v)) continue;
            out_v[m] = v;
            if (step_weighted(P, i)) {
                double a, cc, e;
                orc_literal_terms(deg[v], b, P->f1[i], P->ie[i], P->f2[i], cv[v], s2[v], &a, &cc, &e);
                out_w[m] = a * cc * e;
            } else {
                out_w[m] = 1.0;
            }
            ++m;
        }
    }
    free_sampler(&S);
    return m;
}

/* ------------------------------------------------------------------ */
/* Exact counting judges (the plain definition of C(G, P), Sec. 2.1)    */
/* ------------------------------------------------------------------ */

/* Number of injective edge-preserving maps of the pattern into the graph,
 * by backtracking over the pattern vertices in the given order (each
 * prefix of which must be connected).  Candidates of a non-first vertex
 * are the common neighbours of its matched pattern neighbours; the last
 * level is counted rather than enumerated. */
static uint64_t bt_count(const orc_graph* G, const uint8_t* adjmask, const uint8_t* order, uint32_t k, uint32_t i,
                         uint32_t* m) {
    uint32_t u = order[i];
    uint8_t back = 0; /* positions j < i adjacent to u */
    for (uint32_t j = 0; j < i; ++j)
        if (adjmask[u] >> order[j] & 1) back |= (uint8_t)(1u << j);
    uint64_t total = 0;
    if (i == 0) {
        for (uint64_t v = 0; v < G->n; ++v) {
            m[0] = (uint32_t)v;
            total += (k == 1) ? 1 : bt_count(G, adjmask, order, k, 1, m);
        }
        return total;
    }
    int j0 = __builtin_ctz(back);
    uint32_t base = m[j0];
    for (uint64_t e = G->off[base]; e < G->off[base + 1]; ++e) {
        uint32_t x = G->nbr[e];
        int ok = 1;
        for (uint32_t j = 0; j < i && ok; ++j) {
            if (m[j] == x) ok = 0;
            else if ((back >> j & 1) && j != (uint32_t)j0) {
                uint32_t w = m[j];
                if (!contains(G->nbr + G->off[w], G->off[w + 1] - G->off[w], x)) ok = 0;
            }
        }
        if (!ok) continue;
        if (i + 1 == k) {
            total += 1;
        } else {
            m[i] = x;
            total += bt_count(G, adjmask, order, k, i + 1, m);
        }
    }
    return total;
}

uint64_t orc_count_embeddings(const uint64_t* off, const uint32_t* nbr, uint64_t n, uint64_t nnz,
                              const uint8_t* adjmask, const uint8_t* order, uint32_t k) {
    orc_graph G = {n, nnz, off, nbr};
    uint32_t m[ORC_MAXK];
    if (k == 0) return 0;
    return bt_count(&G, adjmask, order, k, 0, m);
}

/* n_(v) for every v: the embeddings whose first matched pattern vertex
 * (order[0]) maps to v -- the normaliser of the ideal first-step
 * distribution f_ideal(v | ()) (Sec. 3 and the analysis of the approximate
 * distribution).  out[v] for v < n; returns their sum. */
uint64_t orc_rooted_counts(const uint64_t* off, const uint32_t* nbr, uint64_t n, uint64_t nnz,
                           const uint8_t* adjmask, const uint8_t* order, uint32_t k, uint64_t* out) {
    orc_graph G = {n, nnz, off, nbr};
    uint32_t m[ORC_MAXK];
    uint64_t total = 0;
    for (uint64_t v = 0; v < n; ++v) {
        m[0] = (uint32_t)v;
        out[v] = (k <= 1) ? (k == 1) : bt_count(&G, adjmask, order, k, 1, m);
        total += out[v];
    }
    return total;
}

/* Number of k-cliques (copies) by ordered listing over the degree-oriented
 * graph: an edge points from the endpoint with smaller (degree, id) to the
 * larger one; each clique is counted once at its smallest vertex. */
static uint64_t clique_rec(const orc_graph* G, const uint32_t* cand, uint64_t ncand, uint32_t left,
                           uint32_t* buf, uint64_t bufcap) {
    if (left == 0) return 1;
    if (left == 1) return ncand;
    uint64_t total = 0;
    for (uint64_t a = 0; a < ncand; ++a) {
        uint32_t x = cand[a];
        uint32_t* next = buf;
        uint64_t nn = 0;
        const uint32_t* rx = G->nbr + G->off[x];
        uint64_t dx = G->off[x + 1] - G->off[x];
        for (uint64_t b = a + 1; b < ncand; ++b)
            if (contains(rx, dx, cand[b])) next[nn++] = cand[b];
        if (nn + 1 >= left) total += clique_rec(G, next, nn, left - 1, buf + nn, bufcap - nn);
    }
    return total;
}

uint64_t orc_count_cliques(const uint64_t* off, const uint32_t* nbr, uint64_t n, uint64_t nnz, uint32_t k) {
    orc_graph G = {n, nnz, off, nbr};
    uint64_t md = max_degree(&G) + 1;
    uint32_t* out = (uint32_t*)malloc(md * sizeof(uint32_t));
    uint32_t* buf = (uint32_t*)malloc(md * (uint64_t)(k + 1) * sizeof(uint32_t));
    uint64_t total = 0;
    for (uint64_t v = 0; v < n; ++v) {
        uint64_t dv = off[v + 1] - off[v];
        uint64_t no = 0;
        for (uint64_t e = off[v]; e < off[v + 1]; ++e) {
            uint32_t x = nbr[e];
            uint64_t dx = off[x + 1] - off[x];
            if (dx > dv || (dx == dv && x > v)) out[no++] = x; /* already ascending by id */
        }
        if (k == 1) { total += 1; continue; }
        total += clique_rec(&G, out, no, k - 1, buf, md * (uint64_t)(k + 1));
    }
    free(out);
    free(buf);
    return total;
}

/* ------------------------------------------------------------------ */
/* OpenMP flavour: the same functions, the work split across host      */
/* threads (one sampler per thread, as the paper's CPU implementation   */
/* runs its samplers).  Every result equals the single-threaded one:    */
/* table entries and records are per vertex and per sample, and the     */
/* statistics of contiguous index blocks are merged in block order.     */
/* ------------------------------------------------------------------ */
#include <omp.h>

/* orc_build_tables over all vertices on `threads` threads (0 = OpenMP's
 * default).  Returns the number of threads used. */
int orc_build_tables_parallel(const uint64_t* off, const uint32_t* nbr, uint64_t n, uint32_t cv_seed_lo,
                              uint32_t cv_seed_hi, int32_t lc_min, int exact_cv, int threads, uint32_t* deg,
                              uint64_t* s2, uint64_t* hits, uint64_t* trials, int32_t* la, int32_t* lc) {
    init_fixed_point();
    uint32_t key[2] = {cv_seed_lo, cv_seed_hi};
    int used = 1;
    int nt = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel num_threads(nt)
    {
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 4096)
        for (int64_t v = 0; v < (int64_t)n; ++v)
            tables_of_vertex(off, nbr, off, nbr, (uint64_t)v, key, lc_min, exact_cv, &deg[v], &s2[v], &hits[v],
                             &trials[v], &la[v], &lc[v]);
    }
    return used;
}

/* Merges statistics b into a (Chan et al.'s pairwise update). */
static void merge_stats(orc_stats* a, const orc_stats* b) {
    if (b->n == 0) return;
    if (a->n == 0) {
        *a = *b;
        return;
    }
    double na = (double)a->n, nb = (double)b->n, tot = na + nb;
    double delta = b->mean - a->mean;
    a->mean = a->mean + delta * (nb / tot);
    a->m2 = a->m2 + b->m2 + delta * delta * (na * nb / tot);
    a->n += b->n;
    a->nonzero += b->nonzero;
}

/* orc_run over samples [start, start + count) on `threads` threads: thread
 * t runs the t-th of `threads` contiguous blocks in index order with its own
 * sampler, and the blocks' statistics are merged in block order into *st.
 * Returns the number of threads used, or -1 when a scratch allocation
 * failed. */
int orc_run_parallel(const uint64_t* off, const uint32_t* nbr, uint64_t n, uint64_t nnz, const uint32_t* deg,
                     const uint64_t* s2, const int32_t* la, const int32_t* lc, const orc_plan* P,
                     const int32_t* const* lt, const uint32_t* q1, const uint64_t* pre1, uint64_t Q1, uint64_t seed,
                     uint64_t start, uint64_t count, int threads, orc_stats* st) {
    int nt = threads > 0 ? threads : omp_get_max_threads();
    orc_stats* part = (orc_stats*)calloc((size_t)nt, sizeof(orc_stats));
    int* bad = (int*)calloc((size_t)nt, sizeof(int));
    if (!part || !bad) {
        free(part);
        free(bad);
        return -1;
    }
#pragma omp parallel num_threads(nt)
    {
        int t = omp_get_thread_num();
        int tn = omp_get_num_threads();
        uint64_t lo = count * (uint64_t)t / (uint64_t)tn, hi = count * (uint64_t)(t + 1) / (uint64_t)tn;
        if (tn != nt) bad[t] = 1; /* fewer threads than asked: the blocks would not cover the range */
        else if (hi > lo)
            bad[t] = orc_run(off, nbr, n, nnz, deg, s2, la, lc, P, lt, q1, pre1, Q1, seed, start + lo, hi - lo,
                             &part[t], NULL, NULL) != 0;
    }
    int rc = nt;
    for (int t = 0; t < nt; ++t) {
        if (bad[t]) rc = -1;
        merge_stats(st, &part[t]);
    }
    free(part);
    free(bad);
    return rc;
}

/* orc_run_indices on `threads` threads (records are per sample). */
int orc_run_indices_parallel(const uint64_t* off, const uint32_t* nbr, uint64_t n, uint64_t nnz,
                             const uint32_t* deg, const uint64_t* s2, const int32_t* la, const int32_t* lc,
                             const orc_plan* P, const int32_t* const* lt, const uint32_t* q1, const uint64_t* pre1,
                             uint64_t Q1, uint64_t seed, const uint64_t* idx, uint64_t count, int threads,
                             orc_record* recs) {
    int nt = threads > 0 ? threads : omp_get_max_threads();
    int bad = 0;
#pragma omp parallel num_threads(nt) reduction(| : bad)
    {
        int t = omp_get_thread_num();
        int tn = omp_get_num_threads();
        uint64_t lo = count * (uint64_t)t / (uint64_t)tn, hi = count * (uint64_t)(t + 1) / (uint64_t)tn;
        if (hi > lo)
            bad |= orc_run_indices(off, nbr, n, nnz, deg, s2, la, lc, P, lt, q1, pre1, Q1, seed, idx + lo, hi - lo,
                                   recs + lo) != 0;
    }
    return bad ? -1 : nt;
}

/* orc_count_cliques with the vertices (each clique counted at its smallest
 * vertex in the degree order) spread over `threads` threads. */
uint64_t orc_count_cliques_parallel(const uint64_t* off, const uint32_t* nbr, uint64_t n, uint64_t nnz, uint32_t k,
                                    int threads) {
    orc_graph G = {n, nnz, off, nbr};
    uint64_t md = max_degree(&G) + 1;
    uint64_t total = 0;
    int nt = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel num_threads(nt) reduction(+ : total)
    {
        uint32_t* out = (uint32_t*)malloc(md * sizeof(uint32_t));
        uint32_t* buf = (uint32_t*)malloc(md * (uint64_t)(k + 1) * sizeof(uint32_t));
#pragma omp for schedule(dynamic, 64)
        for (int64_t v = 0; v < (int64_t)n; ++v) {
            uint64_t dv = off[v + 1] - off[v];
            uint64_t no = 0;
            for (uint64_t e = off[v]; e < off[v + 1]; ++e) {
                uint32_t x = nbr[e];
                uint64_t dx = off[x + 1] - off[x];
                if (dx > dv || (dx == dv && x > (uint64_t)v)) out[no++] = x;
            }
            if (k == 1) {
                total += 1;
                continue;
            }
            total += clique_rec(&G, out, no, k - 1, buf, md * (uint64_t)(k + 1));
        }
        free(out);
        free(buf);
    }
    return total;
}
