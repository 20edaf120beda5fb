// Pattern compiler of the AGIS library (host code, integers only).
//
// For a matching order u_1..u_k and each step i it derives, on the
// remaining pattern P_i = P[{u_i..u_k}] (Sec. 4.2.2, Eq. Pi):
//   b  = |B|: pattern edges from u_i to already matched vertices;
//   f1 = |F1|: vertices at hop 1 of u_i inside P_i;
//   i1 = |I1|: edges among the hop-1 vertices; ie = |I_effective|, the edge
//        count of a spanning forest of the graph those edges induce;
//   f2 = |F2|: edges between hop-1 and hop-2 vertices (Sec. 4.2.3);
//   certainty(i) = 1 - (|E>=2| - |V>=2|) / |V_i|, with V>=2 the vertices of
//        P_i at distance >= 2 (and finite) from u_i and E>=2 the edges of
//        E_P touching V>=2 (Definition "Decision Function", Sec. 5.1).
// The order itself, when not given, is built greedily by Algorithm 2
// (Sec. 5.2): among the unmatched neighbours of the prefix (any vertex at
// the first step) take the one maximising |F1| + |I1|, smallest id on ties.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "agis.h"
#include "agis_internal.h"

namespace agis {
namespace {

struct StepInfo {
    int b, f1, i1, ie, f2;
    int cert_num, cert_den;
};

int popc(uint32_t x) { return __builtin_popcount(x); }

StepInfo analyse_step(const agis_pattern& p, const uint8_t* order, int i) {
    const int k = (int)p.k;
    uint32_t prefix = 0;
    for (int j = 0; j < i; ++j) prefix |= 1u << order[j];
    const uint32_t all = (1u << k) - 1u;
    const uint32_t rem = all & ~prefix;
    const int u = order[i];
    StepInfo s{};
    s.b = popc(p.adj[u] & prefix);
    // breadth-first distances from u inside P_i
    int dist[kMaxK];
    for (int w = 0; w < k; ++w) dist[w] = -1;
    dist[u] = 0;
    uint32_t frontier = 1u << u, seen = frontier;
    for (int h = 1; frontier; ++h) {
        uint32_t next = 0;
        for (int w = 0; w < k; ++w)
            if (frontier >> w & 1u) next |= p.adj[w];
        next &= rem & ~seen;
        for (int w = 0; w < k; ++w)
            if (next >> w & 1u) dist[w] = h;
        seen |= next;
        frontier = next;
    }
    uint32_t h1 = 0, h2 = 0, ge2 = 0;
    for (int w = 0; w < k; ++w) {
        if (dist[w] == 1) h1 |= 1u << w;
        if (dist[w] == 2) h2 |= 1u << w;
        if (dist[w] >= 2) ge2 |= 1u << w;
    }
    s.f1 = popc(h1);
    // I1 and its spanning forest (union-find over the hop-1 vertices)
    int parent[kMaxK];
    for (int w = 0; w < k; ++w) parent[w] = w;
    auto find = [&](int x) {
        while (parent[x] != x) x = parent[x];
        return x;
    };
    int e_ge2 = 0;
    for (int a = 0; a < k; ++a) {
        for (int c = a + 1; c < k; ++c) {
            if (!(p.adj[a] >> c & 1u)) continue;
            const bool a1 = h1 >> a & 1u, c1 = h1 >> c & 1u;
            const bool a2 = h2 >> a & 1u, c2 = h2 >> c & 1u;
            if (a1 && c1) {
                ++s.i1;
                int ra = find(a), rc = find(c);
                if (ra != rc) {
                    parent[ra] = rc;
                    ++s.ie;
                }
            }
            if ((a1 && c2) || (a2 && c1)) ++s.f2;
            if ((ge2 >> a & 1u) || (ge2 >> c & 1u)) ++e_ge2;
        }
    }
    const int vi = popc(rem);
    s.cert_den = vi;
    s.cert_num = vi - (e_ge2 - popc(ge2));
    return s;
}

bool connected(const agis_pattern& p) {
    const uint32_t all = (1u << p.k) - 1u;
    uint32_t seen = 1u, frontier = 1u;
    while (frontier) {
        uint32_t next = 0;
        for (uint32_t w = 0; w < p.k; ++w)
            if (frontier >> w & 1u) next |= p.adj[w];
        next &= all & ~seen;
        seen |= next;
        frontier = next;
    }
    return seen == all;
}

uint32_t count_automorphisms(const agis_pattern& p) {
    int perm[kMaxK];
    for (uint32_t i = 0; i < p.k; ++i) perm[i] = (int)i;
    uint32_t cnt = 0;
    do {
        bool ok = true;
        for (uint32_t a = 0; a < p.k && ok; ++a)
            for (uint32_t c = 0; c < p.k && ok; ++c)
                if ((p.adj[a] >> c & 1u) && !(p.adj[perm[a]] >> perm[c] & 1u)) ok = false;
        if (ok) ++cnt;
    } while (std::next_permutation(perm, perm + p.k));
    return cnt;
}

}  // namespace

int compile_plan(const agis_pattern* p, const uint8_t* order_in, int mode, int beta_num, int beta_den,
                 agis_plan* out, std::string* err) {
    if (!p || !out) {
        *err = "null pattern or output";
        return AGIS_E_INVALID_ARG;
    }
    if (p->k < 2 || p->k > (uint32_t)kMaxK) {
        *err = "pattern size must be in [2, 8]";
        return AGIS_E_PATTERN;
    }
    const int k = (int)p->k;
    for (int a = 0; a < k; ++a) {
        if (p->adj[a] >> a & 1u) {
            *err = "pattern has a self-loop";
            return AGIS_E_PATTERN;
        }
        if (p->adj[a] >> k) {
            *err = "pattern adjacency names a vertex >= k";
            return AGIS_E_PATTERN;
        }
        for (int c = 0; c < k; ++c)
            if ((p->adj[a] >> c & 1u) != (p->adj[c] >> a & 1u)) {
                *err = "pattern adjacency is not symmetric";
                return AGIS_E_PATTERN;
            }
    }
    if (!connected(*p)) {
        *err = "pattern is not connected";
        return AGIS_E_PATTERN;
    }
    if (mode < AGIS_MODE_UNIFORM || mode > AGIS_MODE_LEARNED) {
        *err = "unknown mode";
        return AGIS_E_INVALID_ARG;
    }
    if (beta_den < 0) {
        *err = "beta denominator must be >= 0";
        return AGIS_E_INVALID_ARG;
    }
    uint8_t order[kMaxK];
    if (order_in) {
        uint32_t seen = 0;
        for (int i = 0; i < k; ++i) {
            if (order_in[i] >= k || (seen >> order_in[i] & 1u)) {
                *err = "order is not a permutation of the pattern vertices";
                return AGIS_E_ORDER;
            }
            seen |= 1u << order_in[i];
            order[i] = order_in[i];
        }
    } else {
        uint32_t used = 0;
        for (int i = 0; i < k; ++i) {
            uint32_t cands = 0;
            if (i == 0) {
                cands = (1u << k) - 1u;
            } else {
                for (int j = 0; j < i; ++j) cands |= p->adj[order[j]];
                cands &= ~used;
            }
            int best = -1, best_s = -1;
            for (int u = 0; u < k; ++u) {
                if (!(cands >> u & 1u)) continue;
                uint8_t trial[kMaxK];
                for (int j = 0; j < i; ++j) trial[j] = order[j];
                trial[i] = (uint8_t)u;
                int t = i + 1;
                for (int w = 0; w < k; ++w)
                    if (!(used >> w & 1u) && w != u) trial[t++] = (uint8_t)w;
                StepInfo s = analyse_step(*p, trial, i);
                if (s.f1 + s.i1 > best_s) {
                    best_s = s.f1 + s.i1;
                    best = u;
                }
            }
            order[i] = (uint8_t)best;
            used |= 1u << best;
        }
    }
    for (int i = 1; i < k; ++i) {
        uint32_t prefix = 0;
        for (int j = 0; j < i; ++j) prefix |= 1u << order[j];
        if (!(p->adj[order[i]] & prefix)) {
            *err = "order position " + std::to_string(i) + " has no matched neighbour";
            return AGIS_E_ORDER;
        }
    }
    std::memset(out, 0, sizeof(*out));
    out->k = (uint32_t)k;
    out->aut = count_automorphisms(*p);
    for (int i = 0; i < k; ++i) {
        StepInfo s = analyse_step(*p, order, i);
        out->order[i] = order[i];
        uint8_t bm = 0;
        for (int j = 0; j < i; ++j)
            if (p->adj[order[i]] >> order[j] & 1u) bm |= (uint8_t)(1u << j);
        out->bmask[i] = bm;
        out->b[i] = (uint8_t)s.b;
        out->f1[i] = (uint8_t)s.f1;
        out->i1[i] = (uint8_t)s.i1;
        out->ie[i] = (uint8_t)s.ie;
        out->f2[i] = (uint8_t)s.f2;
        out->cert_num[i] = s.cert_num;
        out->cert_den[i] = s.cert_den;
        int d;
        if (mode == AGIS_MODE_UNIFORM) {
            d = 0;
        } else if (mode == AGIS_MODE_ALWAYS) {
            d = 1;
        } else if (beta_den == 0) {
            d = beta_num > 0 ? 0 : 1;
        } else {
            // certainty >= beta  <=>  cert_num * beta_den >= beta_num * cert_den
            d = (int64_t)s.cert_num * beta_den >= (int64_t)beta_num * s.cert_den ? 1 : 0;
        }
        out->decision[i] = (uint8_t)d;
    }
    return AGIS_OK;
}

namespace {

// Canonical code of a graph on k <= 6 vertices given as a bitmask over the
// vertex pairs (a, b), a < b, in lexicographic order: the smallest pair mask
// over all relabellings.
uint32_t pair_index(int a, int b, int k) {
    // index of (a, b), a < b, among the pairs of k vertices in lexicographic order
    return (uint32_t)(a * (2 * k - a - 1) / 2 + (b - a - 1));
}

uint32_t canonical_code(uint32_t mask, int k) {
    int perm[8];
    for (int i = 0; i < k; ++i) perm[i] = i;
    uint32_t best = 0xFFFFFFFFu;
    do {
        uint32_t m = 0;
        for (int a = 0; a < k; ++a)
            for (int b = a + 1; b < k; ++b)
                if (mask >> pair_index(a, b, k) & 1u) {
                    const int x = std::min(perm[a], perm[b]), y = std::max(perm[a], perm[b]);
                    m |= 1u << pair_index(x, y, k);
                }
        best = std::min(best, m);
    } while (std::next_permutation(perm, perm + k));
    return best;
}

bool mask_connected(uint32_t mask, int k) {
    agis_pattern p{};
    p.k = (uint32_t)k;
    for (int a = 0; a < k; ++a)
        for (int b = a + 1; b < k; ++b)
            if (mask >> pair_index(a, b, k) & 1u) {
                p.adj[a] |= (uint8_t)(1u << b);
                p.adj[b] |= (uint8_t)(1u << a);
            }
    return connected(p);
}

}  // namespace

int connected_patterns(uint32_t k, agis_pattern* out, uint32_t cap, uint32_t* count, std::string* err) {
    if (k < 2 || k > 6) {
        *err = "connected patterns are enumerated for 2 <= k <= 6";
        return AGIS_E_INVALID_ARG;
    }
    const int kk = (int)k;
    const uint32_t npairs = (uint32_t)(kk * (kk - 1) / 2);
    std::vector<uint32_t> codes;
    for (uint32_t m = 0; m < (1u << npairs); ++m) {
        if ((uint32_t)__builtin_popcount(m) < k - 1 || !mask_connected(m, kk)) continue;
        const uint32_t c = canonical_code(m, kk);
        if (c == m) codes.push_back(c);  // each class once, at its canonical mask
    }
    std::sort(codes.begin(), codes.end(), [](uint32_t a, uint32_t b) {
        const int pa = __builtin_popcount(a), pb = __builtin_popcount(b);
        return pa != pb ? pa < pb : a < b;
    });
    *count = (uint32_t)codes.size();
    if (!out) return AGIS_OK;
    if (cap < codes.size()) {
        *err = "output array too small";
        return AGIS_E_INVALID_ARG;
    }
    for (size_t i = 0; i < codes.size(); ++i) {
        agis_pattern p{};
        p.k = k;
        for (int a = 0; a < kk; ++a)
            for (int b = a + 1; b < kk; ++b)
                if (codes[i] >> pair_index(a, b, kk) & 1u) {
                    p.adj[a] |= (uint8_t)(1u << b);
                    p.adj[b] |= (uint8_t)(1u << a);
                }
        out[i] = p;
    }
    return AGIS_OK;
}

int concentrations(uint32_t n, const agis_pattern* patterns, const double* copies, double* conc_edge, double* induced,
                   double* conc_induced, std::string* err) {
    if (n == 0 || !patterns || !copies) {
        *err = "null or empty pattern set";
        return AGIS_E_INVALID_ARG;
    }
    const int k = (int)patterns[0].k;
    if (k < 2 || k > 6) {
        *err = "concentrations need 2 <= k <= 6";
        return AGIS_E_INVALID_ARG;
    }
    std::vector<uint32_t> mask(n), code(n);
    for (uint32_t i = 0; i < n; ++i) {
        const agis_pattern& p = patterns[i];
        if ((int)p.k != k || !connected(p)) {
            *err = "every pattern must be connected and of the same size";
            return AGIS_E_PATTERN;
        }
        uint32_t m = 0;
        for (int a = 0; a < k; ++a)
            for (int b = a + 1; b < k; ++b)
                if (p.adj[a] >> b & 1u) m |= 1u << pair_index(a, b, k);
        mask[i] = m;
        code[i] = canonical_code(m, k);
        for (uint32_t j = 0; j < i; ++j)
            if (code[j] == code[i]) {
                *err = "patterns must be pairwise non-isomorphic";
                return AGIS_E_INVALID_ARG;
            }
    }
    auto index_of = [&](uint32_t c) -> int {
        for (uint32_t j = 0; j < n; ++j)
            if (code[j] == c) return (int)j;
        return -1;
    };
    // s[h][g]: copies of pattern h as a spanning subgraph of pattern g (edge
    // subsets of g isomorphic to h); the set must contain every connected
    // graph that is such a subgraph's supergraph on the same vertices, i.e. be
    // closed under adding edges
    const uint32_t npairs = (uint32_t)(k * (k - 1) / 2);
    for (uint32_t i = 0; i < n; ++i)
        for (uint32_t e = 0; e < npairs; ++e)
            if (!(mask[i] >> e & 1u) && index_of(canonical_code(mask[i] | (1u << e), k)) < 0) {
                *err = "the pattern set must hold every connected graph of its size with more edges";
                return AGIS_E_INVALID_ARG;
            }
    std::vector<double> s((size_t)n * n, 0.0);
    for (uint32_t g = 0; g < n; ++g) {
        // enumerate the edge subsets of pattern g
        std::vector<int> bits;
        for (uint32_t e = 0; e < npairs; ++e)
            if (mask[g] >> e & 1u) bits.push_back((int)e);
        for (uint32_t sub = 1; sub < (1u << bits.size()); ++sub) {
            uint32_t m = 0;
            for (size_t j = 0; j < bits.size(); ++j)
                if (sub >> j & 1u) m |= 1u << bits[j];
            if (!mask_connected(m, k)) continue;
            const int h = index_of(canonical_code(m, k));
            if (h >= 0) s[(size_t)h * n + g] += 1.0;
        }
    }
    // copies(h) = sum_g s[h][g] induced(g): solve from the most edges down
    std::vector<uint32_t> order(n);
    for (uint32_t i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(),
              [&](uint32_t a, uint32_t b) { return __builtin_popcount(mask[a]) > __builtin_popcount(mask[b]); });
    std::vector<double> ind(n, 0.0);
    for (uint32_t oi = 0; oi < n; ++oi) {
        const uint32_t h = order[oi];
        double v = copies[h];
        for (uint32_t g = 0; g < n; ++g)
            if (g != h) v -= s[(size_t)h * n + g] * ind[g];
        ind[h] = v / s[(size_t)h * n + h];
    }
    double se = 0.0, si = 0.0;
    for (uint32_t i = 0; i < n; ++i) {
        se += copies[i];
        si += ind[i];
    }
    for (uint32_t i = 0; i < n; ++i) {
        if (conc_edge) conc_edge[i] = se != 0.0 ? copies[i] / se : 0.0;
        if (induced) induced[i] = ind[i];
        if (conc_induced) conc_induced[i] = si != 0.0 ? ind[i] / si : 0.0;
    }
    return AGIS_OK;
}

}  // namespace agis
