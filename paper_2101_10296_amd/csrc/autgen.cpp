// Automorphism generators of a weighted graph, for graphs whose symmetry is not known by
// construction (the paper takes its symmetry group from an automorphism solver, Sec. 2.6,
// Sec. 5).  Individualisation and refinement:
//
//  * colour refinement: a vertex's new colour is the rank of (its colour, a 64-bit hash of
//    the sorted multiset of (neighbour colour, edge weight class)) among all vertices,
//    with the multisets themselves compared where two differ under one hash, repeated until
//    no class splits.  The ranks depend only on the colour data, so isomorphic branches of
//    the search produce the same colours on corresponding vertices;
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

// splitmix64 finaliser: the signature hash of a refinement round (an isomorphism-invariant
// function of the colour data, so ranks by hash are canonical)
inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

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
        // colours 0 .. ncol-1 in the order of the input values (canonical)
        {
            std::vector<int32_t> vals(c.col);
            std::sort(vals.begin(), vals.end());
            vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
            for (int32_t& x : c.col) x = static_cast<int32_t>(std::lower_bound(vals.begin(), vals.end(), x) - vals.begin());
            c.ncol = static_cast<int32_t>(vals.size());
        }
        std::vector<std::vector<int32_t>> cells(c.ncol);
        std::vector<int32_t> pos(n);
        for (int32_t v = 0; v < n; ++v) {
            pos[v] = static_cast<int32_t>(cells[c.col[v]].size());
            cells[c.col[v]].push_back(v);
        }
        std::vector<uint64_t> keys(static_cast<size_t>(g_.off[n]));   // sorted neighbour keys, CSR by g_.off
        std::vector<uint64_t> h(n);
        std::vector<int32_t> seen(n, -1), cand(n), changed;
        std::iota(cand.begin(), cand.end(), 0);
        auto sign = [&](int32_t v) {
            const int64_t o = g_.off[v], d = g_.off[v + 1] - o;
            uint64_t* k = keys.data() + o;
            for (int64_t j = 0; j < d; ++j)
                k[j] = (static_cast<uint64_t>(c.col[g_.nbr[o + j]]) << 24) | static_cast<uint64_t>(g_.wcls[o + j]);
            std::sort(k, k + d);
            uint64_t x = 0x9e3779b97f4a7c15ull ^ static_cast<uint64_t>(d);
            for (int64_t j = 0; j < d; ++j) x = mix64(x ^ k[j]);
            h[v] = x;
        };
        // signature order: hash, then the key lists (exact), so a hash collision never merges
        auto cmp = [&](int32_t a, int32_t b) -> int {
            if (h[a] != h[b]) return h[a] < h[b] ? -1 : 1;
            const auto a0 = keys.begin() + g_.off[a], a1 = keys.begin() + g_.off[a + 1];
            const auto b0 = keys.begin() + g_.off[b], b1 = keys.begin() + g_.off[b + 1];
            if (std::lexicographical_compare(a0, a1, b0, b1)) return -1;
            if (std::lexicographical_compare(b0, b1, a0, a1)) return 1;
            return 0;
        };
        c.trace.clear();
        for (int32_t round = 0;; ++round) {
            // Synchronous rounds: a vertex's signature is recomputed only if it or a neighbour
            // changed colour in the previous round (the first round computes every vertex).
            // Colour ids are stable: a splitting class keeps its id for the part whose
            // signature is unchanged (or, if all of it was recomputed, for the first part in
            // signature order); the other parts get new ids in signature order.
            for (int32_t v : cand) {
                sign(v);
                seen[v] = round;
            }
            std::sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) {
                if (c.col[a] != c.col[b]) return c.col[a] < c.col[b];
                const int r = cmp(a, b);
                return r != 0 ? r < 0 : a < b;
            });
            // one unchanged member per touched class, signed before any colour moves
            std::vector<std::pair<int32_t, int32_t>> runs;   // [begin, end) of each class in cand
            std::vector<int32_t> rep;
            for (size_t i0 = 0; i0 < cand.size();) {
                size_t i1 = i0;
                while (i1 < cand.size() && c.col[cand[i1]] == c.col[cand[i0]]) ++i1;
                const auto& cell = cells[c.col[cand[i0]]];
                int32_t r = -1;
                if (cell.size() > i1 - i0)
                    for (int32_t v : cell)
                        if (seen[v] != round) {
                            r = v;
                            break;
                        }
                if (r >= 0) sign(r);
                runs.push_back({static_cast<int32_t>(i0), static_cast<int32_t>(i1)});
                rep.push_back(r);
                i0 = i1;
            }
            changed.clear();
            for (size_t t = 0; t < runs.size(); ++t) {
                const int32_t X = c.col[cand[runs[t].first]];
                const int32_t r = rep[t];
                for (int32_t i0 = runs[t].first; i0 < runs[t].second;) {
                    int32_t i1 = i0 + 1;
                    while (i1 < runs[t].second && cmp(cand[i1], cand[i0]) == 0) ++i1;
                    // the part keeping X: the unchanged members' signature, else the first part
                    const bool keep = (r >= 0) ? cmp(cand[i0], r) == 0 : i0 == runs[t].first;
                    if (!keep) {
                        const int32_t id = c.ncol++;
                        cells.emplace_back();
                        for (int32_t i = i0; i < i1; ++i) {
                            const int32_t v = cand[i];
                            auto& from = cells[X];
                            const int32_t last = from.back();
                            from[pos[v]] = last;
                            pos[last] = pos[v];
                            from.pop_back();
                            pos[v] = static_cast<int32_t>(cells[id].size());
                            cells[id].push_back(v);
                            c.col[v] = id;   // this round's signatures are all computed already
                            changed.push_back(v);
                        }
                    }
                    i0 = i1;
                }
            }
            c.trace.push_back(c.ncol);
            if (ref && (static_cast<int32_t>(c.trace.size()) > static_cast<int32_t>(ref->size()) ||
                        (*ref)[c.trace.size() - 1] != c.ncol))
                return false;
            if (changed.empty()) break;
            cand.clear();
            const int32_t mark = -2 - round;   // fresh marker (seen[] holds rounds >= 0)
            auto add = [&](int32_t v) {
                if (seen[v] != mark) {
                    seen[v] = mark;
                    cand.push_back(v);
                }
            };
            for (int32_t v : changed) {
                add(v);
                for (int64_t j = g_.off[v]; j < g_.off[v + 1]; ++j) add(g_.nbr[j]);
            }
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
