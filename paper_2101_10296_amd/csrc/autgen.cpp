// Automorphism generators of a weighted graph, for graphs whose symmetry is not known by
// construction (the paper takes its symmetry group from an automorphism solver, Sec. 2.6,
// Sec. 5).  Individualisation and refinement:
//
//  * colour refinement: a vertex's new colour is the rank of (its colour, the sorted
//    multiset of (neighbour colour, edge weight class)) among all vertices, repeated until
//    no class splits.  Ranks are assigned in sorted signature order, so isomorphic branches
//    of the search produce the same colours on corresponding vertices;
//  * the first (reference) path individualises, at every level, the smallest-id vertex of
//    the smallest non-singleton class, until the colouring is discrete;
//  * bottom-up along that path, every other vertex y of the level's target class that is
//    not yet in the orbit of the reference vertex (under the generators found at deeper
//    levels, which fix the path above) is individualised instead, and the search below it
//    looks for a discrete colouring whose vertex-by-colour matching with the reference leaf
//    is an automorphism (edges and weights preserved).  Branches whose refinement trace
//    (classes after every round) differs from the reference are cut.
//
// Every returned permutation is a verified automorphism; with the search complete they
// generate the automorphism group.  A time limit or a leaf budget can end the search early;
// the generators found so far still generate a subgroup, which the orbit reduction accepts.
#include <algorithm>
#include <chrono>
#include <cstdint>
#include <map>
#include <numeric>
#include <string>
#include <vector>

namespace qaoa {

namespace {

struct AGraph {
    int32_t n = 0;
    std::vector<int64_t> off;       // CSR
    std::vector<int32_t> nbr;
    std::vector<int32_t> wcls;      // weight class of each adjacency entry
    std::vector<std::pair<int64_t, int32_t>> edges;   // sorted (u * n + v, weight class), u < v
};

struct Colouring {
    std::vector<int32_t> col;       // colour of every vertex, 0 .. ncol-1
    int32_t ncol = 0;
    std::vector<int32_t> trace;     // number of classes after every refinement round
};

class Searcher {
  public:
    Searcher(const AGraph& g, int64_t leaf_budget, double seconds)
        : g_(g), budget_(leaf_budget), t0_(std::chrono::steady_clock::now()), limit_(seconds) {}

    bool timed_out() const {
        const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
        return dt > limit_;
    }

    // Refine c in place; with ref != nullptr stop early (return false) once the number of
    // classes after some round differs from ref.
    bool refine(Colouring& c, const std::vector<int32_t>* ref) const {
        const int32_t n = g_.n;
        std::vector<std::vector<uint64_t>> sig(n);
        std::vector<int32_t> order(n);
        c.trace.clear();
        for (int round = 0;; ++round) {
            for (int32_t v = 0; v < n; ++v) {
                auto& s = sig[v];
                s.clear();
                s.push_back(static_cast<uint64_t>(c.col[v]));
                for (int64_t j = g_.off[v]; j < g_.off[v + 1]; ++j)
                    s.push_back((static_cast<uint64_t>(c.col[g_.nbr[j]]) << 24) | static_cast<uint64_t>(g_.wcls[j]));
                std::sort(s.begin() + 1, s.end());
            }
            std::iota(order.begin(), order.end(), 0);
            std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
                if (sig[a] != sig[b]) return sig[a] < sig[b];
                return a < b;
            });
            std::vector<int32_t> nc(n);
            int32_t k = 0;
            for (int32_t i = 0; i < n; ++i) {
                if (i > 0 && sig[order[i]] != sig[order[i - 1]]) ++k;
                nc[order[i]] = k;
            }
            const int32_t ncol = n ? k + 1 : 0;
            c.trace.push_back(ncol);
            if (ref && (static_cast<int32_t>(c.trace.size()) > static_cast<int32_t>(ref->size()) ||
                        (*ref)[c.trace.size() - 1] != ncol))
                return false;
            const bool stable = ncol == c.ncol;
            c.col.swap(nc);
            c.ncol = ncol;
            if (stable) break;
        }
        if (ref && c.trace.size() != ref->size()) return false;
        return true;
    }

    // The smallest non-singleton class (smallest colour on ties); -1 if discrete.
    int32_t target(const Colouring& c) const {
        std::vector<int32_t> size(c.ncol, 0);
        for (int32_t x : c.col) size[x]++;
        int32_t best = -1;
        for (int32_t k = 0; k < c.ncol; ++k)
            if (size[k] > 1 && (best < 0 || size[k] < size[best])) best = k;
        return best;
    }

    std::vector<int32_t> members(const Colouring& c, int32_t colour) const {
        std::vector<int32_t> out;
        for (int32_t v = 0; v < g_.n; ++v)
            if (c.col[v] == colour) out.push_back(v);
        return out;
    }

    Colouring individualise(const Colouring& c, int32_t x, const std::vector<int32_t>* ref) const {
        Colouring d;
        d.col.resize(g_.n);
        for (int32_t v = 0; v < g_.n; ++v) d.col[v] = 2 * c.col[v] + (v == x ? 0 : 1);
        d.ncol = -1;   // forces at least one renumbering round
        if (!refine(d, ref)) d.ncol = -2;
        return d;
    }

    bool is_automorphism(const std::vector<int32_t>& perm) const {
        for (const auto& e : g_.edges) {
            const int32_t a = perm[e.first / g_.n], b = perm[e.first % g_.n];
            const int64_t key = static_cast<int64_t>(std::min(a, b)) * g_.n + std::max(a, b);
            auto it = std::lower_bound(g_.edges.begin(), g_.edges.end(), std::make_pair(key, int32_t{-1}));
            if (it == g_.edges.end() || it->first != key || it->second != e.second) return false;
        }
        return true;
    }

    // Search below c (a branch whose levels so far matched the reference) for a leaf whose
    // matching with the reference leaf is an automorphism.
    bool descend(const Colouring& c, size_t depth, const std::vector<Colouring>& path, const std::vector<int32_t>& ref_leaf,
                 std::vector<int32_t>& perm) {
        if (timed_out() || leaves_ >= budget_) return false;
        const int32_t t = target(c);
        if (t < 0) {
            ++leaves_;
            // colour -> vertex in this leaf; the reference leaf's vertex of colour k maps there
            std::vector<int32_t> at(g_.n);
            for (int32_t v = 0; v < g_.n; ++v) at[c.col[v]] = v;
            perm.assign(g_.n, 0);
            for (int32_t v = 0; v < g_.n; ++v) perm[v] = at[ref_leaf[v]];
            return is_automorphism(perm);
        }
        if (depth + 1 >= path.size()) return false;
        const std::vector<int32_t>& ref = path[depth + 1].trace;
        for (int32_t y : members(c, t)) {
            Colouring d = individualise(c, y, &ref);
            if (d.ncol < 0) continue;
            if (descend(d, depth + 1, path, ref_leaf, perm)) return true;
        }
        return false;
    }

    int64_t leaves_ = 0;

  private:
    const AGraph& g_;
    int64_t budget_;
    std::chrono::steady_clock::time_point t0_;
    double limit_;
};

// Vertex invariant for the root colouring: the sizes of the spheres at distances 1..R and
// the number of edges inside the radius-R ball (both preserved by automorphisms).  Regular
// graphs are not split by colour refinement alone; this separates the vertices near short
// cycles, so the first target class is small.  Skipped (all zero) once the balls would cost
// more than `cap` visits in total.
std::vector<std::vector<int64_t>> ball_invariant(const AGraph& g, int R, int64_t cap) {
    const int32_t n = g.n;
    std::vector<std::vector<int64_t>> inv(n);
    std::vector<int32_t> dist(n, -1);
    std::vector<int32_t> queue;
    int64_t work = 0;
    for (int32_t s = 0; s < n; ++s) {
        queue.assign(1, s);
        dist[s] = 0;
        std::vector<int64_t> sphere(R + 1, 0);
        int64_t inner = 0;
        for (size_t h = 0; h < queue.size(); ++h) {
            const int32_t x = queue[h];
            for (int64_t j = g.off[x]; j < g.off[x + 1]; ++j) {
                const int32_t y = g.nbr[j];
                ++work;
                if (dist[y] < 0 && dist[x] < R) {
                    dist[y] = dist[x] + 1;
                    sphere[dist[y]]++;
                    queue.push_back(y);
                }
                if (dist[y] >= 0 && x < y) ++inner;
            }
        }
        for (int32_t x : queue) dist[x] = -1;
        inv[s] = sphere;
        inv[s][0] = inner;
        if (work > cap) {
            for (auto& v : inv) v.assign(1, 0);
            return inv;
        }
    }
    return inv;
}

struct UnionFind {
    std::vector<int32_t> p;
    explicit UnionFind(int32_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
    int32_t find(int32_t x) {
        while (p[x] != x) x = p[x] = p[p[x]];
        return x;
    }
    void unite(int32_t a, int32_t b) {
        a = find(a);
        b = find(b);
        if (a != b) p[std::max(a, b)] = std::min(a, b);
    }
};

}  // namespace

// Returns 0 on success, -1 on bad input (msg set).  gens receives the generators (each a
// permutation of 0..n-1); complete is set when the search ran to the end.
int32_t find_generators(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev, const double* ew, int32_t max_gens,
                        double seconds, int64_t leaf_budget, std::vector<std::vector<int32_t>>& gens, bool& complete,
                        std::string& msg) {
    gens.clear();
    complete = false;
    if (n < 1 || m < 0 || (m > 0 && (!eu || !ev)) || max_gens < 0) {
        msg = "bad graph or limits";
        return -1;
    }
    AGraph g;
    g.n = n;
    std::map<double, int32_t> wclass;
    std::vector<int32_t> wc(m, 0);
    for (int64_t i = 0; i < m; ++i) {
        if (eu[i] < 0 || eu[i] >= n || ev[i] < 0 || ev[i] >= n || eu[i] == ev[i]) {
            msg = "edge " + std::to_string(i) + ": bad endpoints";
            return -1;
        }
        if (ew && !(ew[i] == ew[i] && ew[i] - ew[i] == 0.0)) {
            msg = "edge " + std::to_string(i) + ": non-finite weight";
            return -1;
        }
        if (ew) wclass.emplace(ew[i], 0);
    }
    int32_t k = 0;
    for (auto& kv : wclass) kv.second = k++;
    g.off.assign(static_cast<size_t>(n) + 1, 0);
    for (int64_t i = 0; i < m; ++i) {
        wc[i] = ew ? wclass[ew[i]] : 0;
        g.off[eu[i] + 1]++;
        g.off[ev[i] + 1]++;
        const int32_t a = std::min(eu[i], ev[i]), b = std::max(eu[i], ev[i]);
        g.edges.emplace_back(static_cast<int64_t>(a) * n + b, wc[i]);
    }
    std::sort(g.edges.begin(), g.edges.end());
    for (size_t i = 1; i < g.edges.size(); ++i)
        if (g.edges[i].first == g.edges[i - 1].first) {
            msg = "duplicate edge";
            return -1;
        }
    for (int32_t v = 0; v < n; ++v) g.off[v + 1] += g.off[v];
    g.nbr.resize(2 * m);
    g.wcls.resize(2 * m);
    {
        std::vector<int64_t> pos(g.off.begin(), g.off.end() - 1);
        for (int64_t i = 0; i < m; ++i) {
            g.nbr[pos[eu[i]]] = ev[i];
            g.wcls[pos[eu[i]]++] = wc[i];
            g.nbr[pos[ev[i]]] = eu[i];
            g.wcls[pos[ev[i]]++] = wc[i];
        }
    }

    Searcher S(g, leaf_budget, seconds);
    // reference path
    std::vector<Colouring> path(1);
    {
        const auto inv = ball_invariant(g, 4, int64_t{1} << 26);
        std::vector<int32_t> order(n);
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return inv[a] != inv[b] ? inv[a] < inv[b] : a < b; });
        path[0].col.assign(n, 0);
        int32_t k = 0;
        for (int32_t i = 0; i < n; ++i) {
            if (i > 0 && inv[order[i]] != inv[order[i - 1]]) ++k;
            path[0].col[order[i]] = k;
        }
        path[0].ncol = -1;
    }
    S.refine(path[0], nullptr);
    std::vector<int32_t> xs;   // reference vertex chosen at each level
    for (;;) {
        const int32_t t = S.target(path.back());
        if (t < 0) break;
        const int32_t x = S.members(path.back(), t).front();
        xs.push_back(x);
        path.push_back(S.individualise(path.back(), x, nullptr));
    }
    const std::vector<int32_t> ref_leaf = path.back().col;

    // generators, bottom-up along the path; those found at depth >= d fix x_1 .. x_d
    bool cut_short = false;
    for (int d = static_cast<int>(xs.size()) - 1; d >= 0; --d) {
        UnionFind uf(n);
        for (const auto& gnr : gens)
            for (int32_t v = 0; v < n; ++v) uf.unite(v, gnr[v]);
        const int32_t t = S.target(path[d]);
        for (int32_t y : S.members(path[d], t)) {
            if (y == xs[d] || uf.find(y) == uf.find(xs[d])) continue;
            if (static_cast<int32_t>(gens.size()) >= max_gens || S.timed_out()) {
                cut_short = true;
                break;
            }
            Colouring c = S.individualise(path[d], y, &path[d + 1].trace);
            if (c.ncol < 0) continue;
            std::vector<int32_t> perm;
            if (S.descend(c, d + 1, path, ref_leaf, perm)) {
                gens.push_back(perm);
                for (int32_t v = 0; v < n; ++v) uf.unite(v, perm[v]);
            } else if (S.timed_out() || S.leaves_ >= leaf_budget) {
                cut_short = true;
            }
        }
        if (cut_short) break;
    }
    complete = !cut_short;
    return 0;
}

}  // namespace qaoa
