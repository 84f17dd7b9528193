// Host planner (integer-exact).
//
//  * canonical edges: u < v, input order kept as the edge index; self-loops, duplicates
//    and out-of-range ids rejected (MaxCut on a simple graph, Sec. 2.4)
//  * generator check: a permutation of V mapping E onto E (automorphism, Sec. 2.6) that
//    keeps every edge weight bit for bit (weighted symmetries, Sec. 4)
//  * edge orbits by union-find over (e, sigma(e)) for every generator sigma and edge e;
//    the class representative is its smallest edge index and classes are numbered by
//    ascending representative (the paper lets the representative be arbitrary, Sec. 3)
//  * one light cone per class: the radius-p ball around the representative's endpoints
//    (reverse causal cone, Sec. 2.3) with u -> qubit 0, v -> qubit 1 and the rest ordered
//    by (distance, node id); every edge induced on the ball is a cone edge
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <system_error>
#include <thread>

namespace qaoa {
namespace {

[[noreturn]] void fail(int32_t st, const std::string& m) { throw PlanError{st, m}; }

constexpr int32_t kEINVAL = -1, kENOTAUT = -2, kECONE = -3;

// Sorted (key -> edge index) table for edge lookup by endpoints.
struct EdgeIndex {
    uint64_t n = 0;
    std::vector<uint64_t> key;
    std::vector<int64_t> idx;
    void build(int32_t nn, const std::vector<int32_t>& u, const std::vector<int32_t>& v) {
        n = static_cast<uint64_t>(nn);
        const size_t m = u.size();
        std::vector<std::pair<uint64_t, int64_t>> kv(m);
        for (size_t i = 0; i < m; ++i) kv[i] = {static_cast<uint64_t>(u[i]) * n + static_cast<uint64_t>(v[i]), (int64_t)i};
        std::sort(kv.begin(), kv.end());
        key.resize(m);
        idx.resize(m);
        for (size_t i = 0; i < m; ++i) { key[i] = kv[i].first; idx[i] = kv[i].second; }
    }
    int64_t find(int32_t a, int32_t b) const {
        if (a > b) std::swap(a, b);
        const uint64_t k = static_cast<uint64_t>(a) * n + static_cast<uint64_t>(b);
        auto it = std::lower_bound(key.begin(), key.end(), k);
        if (it == key.end() || *it != k) return -1;
        return idx[it - key.begin()];
    }
};

// Union-find whose root is always the smallest index of its set.
struct MinUnionFind {
    std::vector<int64_t> parent;
    explicit MinUnionFind(int64_t m) : parent(m) { for (int64_t i = 0; i < m; ++i) parent[i] = i; }
    int64_t find(int64_t x) {
        while (parent[x] != x) { parent[x] = parent[parent[x]]; x = parent[x]; }
        return x;
    }
    void unite(int64_t a, int64_t b) {
        a = find(a);
        b = find(b);
        if (a == b) return;
        if (a < b) parent[b] = a; else parent[a] = b;
    }
};

// Smallest denominator q <= qmax with |x - a/q| <= tol (continued-fraction convergents),
// or 0 if there is none.
int64_t rational_denominator(double x, int64_t qmax, double tol) {
    double r = std::fabs(x);
    int64_t h0 = 0, h1 = 1, k0 = 1, k1 = 0;   // convergents h/k
    for (int it = 0; it < 64; ++it) {
        const double a = std::floor(r);
        if (a > 9.0e15) break;
        const int64_t ai = static_cast<int64_t>(a);
        const int64_t h2 = ai * h1 + h0, k2 = ai * k1 + k0;
        if (k2 > qmax) break;
        h0 = h1; h1 = h2; k0 = k1; k1 = k2;
        if (std::fabs(std::fabs(x) - static_cast<double>(h1) / static_cast<double>(k1)) <= tol) return k1;
        const double frac = r - a;
        if (frac <= 0.0) break;
        r = 1.0 / frac;
    }
    return 0;
}

// Weights become integers wi in units of delta (w = delta * wi): the kernels keep cut
// values as small integers.  Integer weights use delta = 1; otherwise every weight must be
// a rational with a denominator of at most 2^20 (to 1e-13 relative), delta = g / L with L
// the least common denominator and g the gcd of the scaled weights.  Weights without such
// a unit (irrational ones, Gaussian couplings, ...) make the plan one of real weights.
void weight_units(HostPlan& P);

bool weight_units_or_real(HostPlan& P) {
    try {
        weight_units(P);
        return false;
    } catch (const PlanError&) {
        P.wi.assign(P.w.size(), 0);
        P.delta = 1.0;
        return true;
    }
}

void weight_units(HostPlan& P) {
    const int64_t m = static_cast<int64_t>(P.w.size());
    P.wi.assign(m, 1);
    P.delta = 1.0;
    bool integral = true;
    for (double x : P.w) integral = integral && x == std::floor(x) && std::fabs(x) <= 16777216.0;
    if (integral) {
        for (int64_t i = 0; i < m; ++i) P.wi[i] = static_cast<int32_t>(P.w[i]);
        return;
    }
    int64_t L = 1;
    for (int64_t i = 0; i < m; ++i) {
        const double x = P.w[i];
        const int64_t q = rational_denominator(x, int64_t{1} << 20, 1e-13 * std::max(1.0, std::fabs(x)));
        if (q == 0)
            fail(kEINVAL, "edge " + std::to_string(i) + ": weight is not a rational with a denominator of at most 2^20");
        L = L / std::gcd(L, q) * q;
        if (L > (int64_t{1} << 40)) fail(kEINVAL, "weights have no common unit (denominators too large)");
    }
    std::vector<int64_t> n(m);
    int64_t g = 0;
    for (int64_t i = 0; i < m; ++i) {
        n[i] = std::llround(P.w[i] * static_cast<double>(L));
        g = std::gcd(g, std::llabs(n[i]));
    }
    if (g == 0) g = 1;
    for (int64_t i = 0; i < m; ++i) {
        const int64_t v = n[i] / g;
        if (std::llabs(v) > (int64_t{1} << 24))
            fail(kEINVAL, "edge " + std::to_string(i) + ": weight is more than 2^24 units of the common weight unit");
        P.wi[i] = static_cast<int32_t>(v);
    }
    P.delta = static_cast<double>(g) / static_cast<double>(L);
}

}  // namespace

void build_host_plan(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev, const double* ew,
                     int32_t n_gen, const int32_t* gens, int32_t p, const PlanOptions& opt,
                     HostPlan& P) {
    if (n < 1) fail(kEINVAL, "n_nodes must be >= 1");
    if (m < 0) fail(kEINVAL, "n_edges must be >= 0");
    if (m > 0 && (!eu || !ev)) fail(kEINVAL, "edge arrays are NULL");
    if (p < 1) fail(kEINVAL, "p must be >= 1");
    if (p > 1024) fail(kEINVAL, "p must be <= 1024 (launch grids carry 2p + 1 values per point)");
    if (n_gen < 0 || (n_gen > 0 && !gens)) fail(kEINVAL, "bad generator array");
    if (opt.max_cone_qubits < 2 || opt.max_cone_qubits > 30) fail(kEINVAL, "max_cone_qubits must be in [2, 30]");
    if (opt.k_lds_max != 14) fail(kEINVAL, "k_lds_max must be 14 (cones above it are kept in device memory)");

    P = HostPlan{};
    P.n = n;
    P.m = m;
    P.p = p;
    P.u.resize(m);
    P.v.resize(m);
    P.w.assign(m, 1.0);
    P.unit = (ew == nullptr);
    for (int64_t i = 0; i < m; ++i) {
        int32_t a = eu[i], b = ev[i];
        if (a < 0 || a >= n || b < 0 || b >= n) fail(kEINVAL, "edge " + std::to_string(i) + ": node id out of range");
        if (a == b) fail(kEINVAL, "edge " + std::to_string(i) + ": self-loop");
        if (a > b) std::swap(a, b);
        P.u[i] = a;
        P.v[i] = b;
        if (ew) {
            const double x = ew[i];
            if (!std::isfinite(x)) fail(kEINVAL, "edge " + std::to_string(i) + ": non-finite weight");
            P.w[i] = x;
            if (x != 1.0) P.unit = false;
        }
    }
    P.realw = weight_units_or_real(P);
    EdgeIndex index;
    index.build(n, P.u, P.v);
    for (int64_t i = 1; i < m; ++i)
        if (index.key[i] == index.key[i - 1]) fail(kEINVAL, "duplicate edge (" + std::to_string(index.key[i] / index.n) + "," + std::to_string(index.key[i] % index.n) + ")");

    // ---- CSR adjacency with edge ids (neighbours in edge order)
    std::vector<int64_t> off(static_cast<size_t>(n) + 1, 0);
    for (int64_t e = 0; e < m; ++e) { off[P.u[e] + 1]++; off[P.v[e] + 1]++; }
    for (int32_t i = 0; i < n; ++i) off[i + 1] += off[i];
    std::vector<int32_t> nbr(2 * m);
    std::vector<int64_t> nbr_e(2 * m);
    {
        std::vector<int64_t> pos(off.begin(), off.end() - 1);
        for (int64_t e = 0; e < m; ++e) {
            nbr[pos[P.u[e]]] = P.v[e]; nbr_e[pos[P.u[e]]++] = e;
            nbr[pos[P.v[e]]] = P.u[e]; nbr_e[pos[P.v[e]]++] = e;
        }
    }
    // edge id of {a, b}: a scan of the shorter neighbour list, the sorted index for long ones
    auto edge_of = [&](int32_t a, int32_t b) -> int64_t {
        if (off[a + 1] - off[a] > off[b + 1] - off[b]) std::swap(a, b);
        if (off[a + 1] - off[a] > 32) return index.find(a, b);
        for (int64_t j = off[a]; j < off[a + 1]; ++j)
            if (nbr[j] == b) return nbr_e[j];
        return -1;
    };

    // ---- generators: verify, then union every edge with its image
    MinUnionFind uf(m);
    std::vector<char> seen(n);
    for (int32_t g = 0; g < n_gen; ++g) {
        const int32_t* s = gens + static_cast<int64_t>(g) * n;
        std::fill(seen.begin(), seen.end(), 0);
        for (int32_t i = 0; i < n; ++i) {
            if (s[i] < 0 || s[i] >= n || seen[s[i]]) fail(kENOTAUT, "generator " + std::to_string(g) + " is not a permutation of the nodes");
            seen[s[i]] = 1;
        }
        for (int64_t e = 0; e < m; ++e) {
            const int64_t f = edge_of(s[P.u[e]], s[P.v[e]]);
            if (f < 0) fail(kENOTAUT, "generator " + std::to_string(g) + " maps edge " + std::to_string(e) + " to a non-edge");
            if (std::memcmp(&P.w[e], &P.w[f], sizeof(double)) != 0)
                fail(kENOTAUT, "generator " + std::to_string(g) + " does not preserve the weight of edge " + std::to_string(e));
            if (opt.reduce) uf.unite(e, f);
        }
    }
    P.edge_orbit.resize(m);
    for (int64_t e = 0; e < m; ++e) {
        const int64_t r = uf.find(e);
        if (r == e) {
            P.edge_orbit[e] = static_cast<int32_t>(P.rep.size());
            P.rep.push_back(e);
            P.size.push_back(0);
            P.W.push_back(0.0);
        } else {
            P.edge_orbit[e] = P.edge_orbit[r];
        }
        P.size[P.edge_orbit[e]] += 1;
        P.W[P.edge_orbit[e]] += P.w[e];
        P.total_weight += P.w[e];
    }

    // ---- light cones.  Every cone depends only on the graph, so the orbits are split into
    // contiguous ranges over threads; a failure reports the lowest failing orbit, as a
    // serial walk would.
    const int32_t kmax = opt.max_cone_qubits;
    const int64_t M = static_cast<int64_t>(P.rep.size());
    P.cones.resize(static_cast<size_t>(M));
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int64_t nt = M >= 4096 ? std::min<int64_t>({16, hw, M / 1024}) : 1;
    std::vector<int64_t> fail_at(static_cast<size_t>(nt), -1);
    std::vector<PlanError> fail_err(static_cast<size_t>(nt));
    std::vector<char> no_mem(static_cast<size_t>(nt), 0);
    std::vector<char> wide(static_cast<size_t>(nt), 0);   // a cone's integer cut range above 255
    auto extract_range = [&](int64_t t) {
        std::vector<int32_t> mark(n, -1), dist(n, 0), loc(n, -1), ball;
        ball.reserve(static_cast<size_t>(kmax) + 1);
        const int64_t o_end = (t + 1) * M / nt;
        for (int64_t o = t * M / nt; o < o_end; ++o) {
            const int64_t e0 = P.rep[o];
            const int32_t a0 = P.u[e0], b0 = P.v[e0];
            const int32_t stamp = static_cast<int32_t>(o);
            ball.assign({a0, b0});
            mark[a0] = mark[b0] = stamp;
            dist[a0] = dist[b0] = 0;
            size_t lo = 0;
            for (int32_t d = 1; d <= p; ++d) {
                const size_t hi = ball.size();
                for (size_t q = lo; q < hi; ++q) {
                    const int32_t x = ball[q];
                    for (int64_t j = off[x]; j < off[x + 1]; ++j) {
                        const int32_t y = nbr[j];
                        if (mark[y] != stamp) {
                            mark[y] = stamp;
                            dist[y] = d;
                            ball.push_back(y);
                            if (static_cast<int32_t>(ball.size()) > kmax) {
                                fail_at[t] = o;
                                fail_err[t] = PlanError{kECONE, "light cone of orbit " + std::to_string(o) + " (edge " +
                                                                     std::to_string(e0) + ") exceeds " +
                                                                     std::to_string(kmax) + " qubits"};
                                return;
                            }
                        }
                    }
                }
                lo = hi;
            }
            std::sort(ball.begin() + 2, ball.end(), [&](int32_t x, int32_t y) {
                return dist[x] != dist[y] ? dist[x] < dist[y] : x < y;
            });
            Cone& c = P.cones[o];
            c.k = static_cast<int32_t>(ball.size());
            c.nodes.assign(ball.begin(), ball.end());
            for (int32_t i = 0; i < c.k; ++i) loc[ball[i]] = i;
            int64_t cmin = 0, cmax = 0, ne = 0;
            for (int32_t i = 0; i < c.k; ++i) {
                const int32_t x = ball[i];
                for (int64_t j = off[x]; j < off[x + 1]; ++j)
                    if (mark[nbr[j]] == stamp && loc[nbr[j]] > i) ++ne;
            }
            c.ea.reserve(ne);
            c.eb.reserve(ne);
            c.ew.reserve(ne);
            c.wf.reserve(ne);
            double fmin = 0.0, fmax = 0.0;
            for (int32_t i = 0; i < c.k; ++i) {
                const int32_t x = ball[i];
                for (int64_t j = off[x]; j < off[x + 1]; ++j) {
                    const int32_t y = nbr[j];
                    if (mark[y] == stamp && loc[y] > i) {
                        c.ea.push_back(i);
                        c.eb.push_back(loc[y]);
                        const int32_t wi = P.wi[nbr_e[j]];
                        const double wr = P.w[nbr_e[j]];
                        c.ew.push_back(wi);
                        c.wf.push_back(wr);
                        if (wi < 0) cmin += wi; else cmax += wi;
                        if (wr < 0) fmin += wr; else fmax += wr;
                    }
                }
            }
            if (cmax - cmin > 255) wide[t] = 1;   // integer cut tables hold bytes: real weights instead
            c.cut_min = static_cast<int32_t>(std::max<int64_t>(cmin, INT32_MIN));
            c.cut_max = static_cast<int32_t>(std::min<int64_t>(cmax, INT32_MAX));
            c.cf_min = fmin;
            c.cf_max = fmax;
        }
    };
    // an allocation failure on a worker thread is carried to the caller's thread
    auto extract = [&](int64_t t) {
        try {
            extract_range(t);
        } catch (const std::bad_alloc&) {
            no_mem[t] = 1;
        }
    };
    if (nt == 1) {
        extract(0);
    } else {
        std::vector<std::thread> pool;
        int64_t started = 1;
        try {
            for (int64_t t = 1; t < nt; ++t) {
                pool.emplace_back(extract, t);
                started = t + 1;
            }
        } catch (const std::system_error&) {
            // no more threads: the remaining ranges run here
        }
        for (int64_t t = started; t < nt; ++t) extract(t);
        extract(0);
        for (auto& th : pool) th.join();
    }
    for (int64_t t = 0; t < nt; ++t)
        if (no_mem[t]) throw std::bad_alloc();
    for (int64_t t = 0; t < nt; ++t)
        if (fail_at[t] >= 0) throw fail_err[t];   // ranges are ascending: the first is the lowest
    for (int64_t t = 0; t < nt; ++t) P.realw = P.realw || wide[t];
    P.cut_min = 0;
    P.cut_max = 0;
    if (P.realw) {
        P.delta = 1.0;
    } else {
        for (const Cone& c : P.cones) {
            P.cut_min = std::min<int32_t>(P.cut_min, c.cut_min);
            P.cut_max = std::max<int32_t>(P.cut_max, c.cut_max);
        }
    }
    P.n_inst = 1;
    P.inst_node = {0, n};
    P.inst_edge = {0, m};
    P.inst_orbit = {0, M};
    P.inst_delta = {P.delta};
}

void merge_host_plans(std::vector<HostPlan>& parts, HostPlan& P) {
    if (parts.empty()) fail(kEINVAL, "no instances");
    P = HostPlan{};
    P.p = parts[0].p;
    P.n_inst = static_cast<int32_t>(parts.size());
    P.inst_node.assign(1, 0);
    P.inst_edge.assign(1, 0);
    P.inst_orbit.assign(1, 0);
    P.unit = true;
    P.delta = parts[0].delta;
    int64_t n_total = 0;
    for (const HostPlan& h : parts) n_total += h.n;
    if (n_total > INT32_MAX) fail(kEINVAL, "the instances hold more than 2^31 - 1 nodes in all");
    for (int32_t j = 0; j < P.n_inst; ++j) {
        HostPlan& h = parts[j];
        if (h.p != P.p) fail(kEINVAL, "instance " + std::to_string(j) + ": every instance needs the same p");
        const int32_t n0 = P.n;
        const int64_t e0 = P.m, o0 = static_cast<int64_t>(P.rep.size());
        P.n += h.n;
        P.m += h.m;
        for (int64_t e = 0; e < h.m; ++e) {
            P.u.push_back(h.u[e] + n0);
            P.v.push_back(h.v[e] + n0);
            P.edge_orbit.push_back(static_cast<int32_t>(h.edge_orbit[e] + o0));
        }
        P.w.insert(P.w.end(), h.w.begin(), h.w.end());
        P.wi.insert(P.wi.end(), h.wi.begin(), h.wi.end());
        for (size_t o = 0; o < h.rep.size(); ++o) {
            P.rep.push_back(h.rep[o] + e0);
            P.size.push_back(h.size[o]);
            P.W.push_back(h.W[o]);
        }
        for (Cone& c : h.cones) {
            for (int32_t& x : c.nodes) x += n0;
            c.inst = j;
            P.cones.push_back(std::move(c));
        }
        P.total_weight += h.total_weight;
        P.cut_min = std::min(P.cut_min, h.cut_min);
        P.cut_max = std::max(P.cut_max, h.cut_max);
        P.unit = P.unit && h.unit;
        P.realw = P.realw || h.realw;
        if (h.delta != P.delta) P.delta = 0.0;   // no single unit: see inst_delta
        P.inst_node.push_back(P.n);
        P.inst_edge.push_back(P.m);
        P.inst_orbit.push_back(static_cast<int64_t>(P.rep.size()));
        P.inst_delta.push_back(h.delta);
        h = HostPlan{};
    }
    if (static_cast<int64_t>(P.rep.size()) > INT32_MAX) fail(kEINVAL, "more than 2^31 - 1 orbits in all");
    if (P.realw) {
        // one instance with real weights: every cone takes the real-weight path (a launch
        // covers cones of all instances), weights used as they are
        P.delta = 1.0;
        P.cut_min = P.cut_max = 0;
        std::fill(P.inst_delta.begin(), P.inst_delta.end(), 1.0);
    }
}

}  // namespace qaoa
