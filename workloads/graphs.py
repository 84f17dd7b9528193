"""Seeded graph families with automorphism generators known by construction.

Every family returns a :class:`Graph` whose edge list is canonical (u < v) and sorted
lexicographically, so that the same edge index means the same edge on every side.
The generators are permutations of the node set (row g maps node i to
``generators[g, i]``); they generate a subgroup of Aut(G) (Sec. 2.6 of the paper
defines automorphisms as node permutations that preserve the edge set).

Families and the generators they carry:

* random d-regular (pairing model): none (trivial group; random regular graphs are
  almost surely asymmetric, Sec. 2.6)
* circulant C_n(S): rotation i -> i+1 and reflection i -> -i (mod n)
* L x L torus: translation (x, y) -> (x+1, y) and quarter turn (x, y) -> (y, -x)
* L x L x L torus: translation along x and the coordinate cycle (x, y, z) -> (y, z, x)
* hypercube Q_d: every coordinate flip, the swap of coordinates 0 and 1, and the
  cyclic shift of coordinates
* complete graph K_n: the transposition (0 1) and the n-cycle
* rook graph K_n x K_n: row transposition, row cycle and the transpose (i, j) -> (j, i)
* Paley graph on a prime q = 1 (mod 4): x -> x+1 and x -> g^2 x (g a primitive root)
* star K_{1,m}: a transposition and a cycle of the leaves
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Graph:
    name: str
    n: int
    edges: np.ndarray                  # int32 [m, 2], u < v, lexicographically sorted
    weights: np.ndarray | None = None  # float64 [m] or None (unit weights)
    generators: np.ndarray = field(default_factory=lambda: np.zeros((0, 0), np.int32))

    @property
    def m(self) -> int:
        return int(self.edges.shape[0])

    def gens(self) -> np.ndarray:
        g = np.asarray(self.generators, dtype=np.int32)
        if g.size == 0:
            return np.zeros((0, self.n), np.int32)
        return g.reshape(-1, self.n)


def _canon(n: int, pairs) -> np.ndarray:
    a = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    u = np.minimum(a[:, 0], a[:, 1])
    v = np.maximum(a[:, 0], a[:, 1])
    if np.any(u == v):
        raise ValueError("self-loop in generated graph")
    key = u * n + v
    key = np.unique(key)
    if key.size != a.shape[0]:
        raise ValueError("duplicate edge in generated graph")
    return np.stack([key // n, key % n], axis=1).astype(np.int32)


def random_regular(n: int, d: int, seed: int) -> Graph:
    """Random d-regular graph from the pairing model.

    The draw is ``pts = repeat(arange(n), d)``, shuffled by ``default_rng(seed)``,
    consecutive entries paired; any self-loop or multi-edge restarts the whole draw
    (same generator, continuing its stream).
    """
    if (n * d) % 2:
        raise ValueError("n*d must be even")
    rng = np.random.default_rng(seed)
    while True:
        pts = np.repeat(np.arange(n, dtype=np.int64), d)
        rng.shuffle(pts)
        a, b = pts[0::2], pts[1::2]
        if np.any(a == b):
            continue
        u, v = np.minimum(a, b), np.maximum(a, b)
        key = u * n + v
        if np.unique(key).size != key.size:
            continue
        key.sort()
        edges = np.stack([key // n, key % n], axis=1).astype(np.int32)
        return Graph(f"rand{d}reg-n{n}-s{seed}", n, edges)


def circulant(n: int, steps) -> Graph:
    steps = [int(s) for s in steps]
    if any(s <= 0 or 2 * s >= n for s in steps):
        raise ValueError("circulant steps must satisfy 0 < s < n/2")
    i = np.arange(n)
    pairs = np.concatenate([np.stack([i, (i + s) % n], 1) for s in steps])
    rot = ((i + 1) % n).astype(np.int32)
    ref = ((-i) % n).astype(np.int32)
    return Graph(f"C{n}({','.join(map(str, steps))})", n, _canon(n, pairs),
                 generators=np.stack([rot, ref]))


def torus2d(L: int) -> Graph:
    if L < 3:
        raise ValueError("L >= 3")
    x, y = np.divmod(np.arange(L * L), L)
    idx = lambda xx, yy: (xx % L) * L + (yy % L)  # noqa: E731
    pairs = np.concatenate([np.stack([idx(x, y), idx(x + 1, y)], 1),
                            np.stack([idx(x, y), idx(x, y + 1)], 1)])
    tr = idx(x + 1, y).astype(np.int32)
    rot = idx(y, -x).astype(np.int32)
    return Graph(f"torus{L}x{L}", L * L, _canon(L * L, pairs), generators=np.stack([tr, rot]))


def torus3d(L: int) -> Graph:
    if L < 3:
        raise ValueError("L >= 3")
    n = L ** 3
    x, rem = np.divmod(np.arange(n), L * L)
    y, z = np.divmod(rem, L)
    idx = lambda a, b, c: ((a % L) * L + (b % L)) * L + (c % L)  # noqa: E731
    pairs = np.concatenate([np.stack([idx(x, y, z), idx(x + 1, y, z)], 1),
                            np.stack([idx(x, y, z), idx(x, y + 1, z)], 1),
                            np.stack([idx(x, y, z), idx(x, y, z + 1)], 1)])
    tr = idx(x + 1, y, z).astype(np.int32)
    cyc = idx(y, z, x).astype(np.int32)
    return Graph(f"torus{L}^3", n, _canon(n, pairs), generators=np.stack([tr, cyc]))


def hypercube(d: int) -> Graph:
    n = 1 << d
    x = np.arange(n)
    pairs = np.concatenate([np.stack([x, x ^ (1 << i)], 1)[(x >> i) & 1 == 0] for i in range(d)])
    gens = [(x ^ (1 << i)).astype(np.int32) for i in range(d)]
    if d >= 2:
        b0, b1 = x & 1, (x >> 1) & 1
        gens.append(((x & ~3) | (b0 << 1) | b1).astype(np.int32))
        # cyclic shift of coordinates: bit i -> bit i+1 (mod d)
        gens.append((((x << 1) | (x >> (d - 1))) & (n - 1)).astype(np.int32))
    return Graph(f"Q{d}", n, _canon(n, pairs), generators=np.stack(gens))


def complete(n: int) -> Graph:
    iu, ju = np.triu_indices(n, 1)
    i = np.arange(n)
    t = i.copy()
    t[0], t[1] = 1, 0
    cyc = (i + 1) % n
    return Graph(f"K{n}", n, _canon(n, np.stack([iu, ju], 1)),
                 generators=np.stack([t, cyc]).astype(np.int32))


def rook(L: int) -> Graph:
    """Rook graph K_L x K_L: (i, j) ~ (i', j') when they share exactly one coordinate."""
    n = L * L
    pairs = []
    for r in range(L):
        a, b = np.triu_indices(L, 1)
        pairs.append(np.stack([r * L + a, r * L + b], 1))
        pairs.append(np.stack([a * L + r, b * L + r], 1))
    i, j = np.divmod(np.arange(n), L)
    ti = i.copy()
    ti[i == 0], ti[i == 1] = 1, 0
    g_tr = (ti * L + j).astype(np.int32)
    g_cy = (((i + 1) % L) * L + j).astype(np.int32)
    g_t = (j * L + i).astype(np.int32)
    return Graph(f"rook{L}", n, _canon(n, np.concatenate(pairs)), generators=np.stack([g_tr, g_cy, g_t]))


def _primitive_root(q: int) -> int:
    phi = q - 1
    fac, m, f = [], phi, 2
    while f * f <= m:
        if m % f == 0:
            fac.append(f)
            while m % f == 0:
                m //= f
        f += 1
    if m > 1:
        fac.append(m)
    for g in range(2, q):
        if all(pow(g, phi // f, q) != 1 for f in fac):
            return g
    raise ValueError("no primitive root")


def paley(q: int) -> Graph:
    if q % 4 != 1:
        raise ValueError("Paley graph needs q = 1 mod 4 (prime q)")
    sq = np.zeros(q, bool)
    sq[(np.arange(1, q) ** 2) % q] = True
    a, b = np.triu_indices(q, 1)
    keep = sq[(b - a) % q]
    g = _primitive_root(q)
    x = np.arange(q)
    return Graph(f"paley{q}", q, _canon(q, np.stack([a[keep], b[keep]], 1)),
                 generators=np.stack([(x + 1) % q, (g * g * x) % q]).astype(np.int32))


def star(m: int) -> Graph:
    """Star K_{1,m}: hub 0 joined to leaves 1..m; generators permute the leaves."""
    e = np.stack([np.zeros(m, np.int64), np.arange(1, m + 1)], 1)
    n = m + 1
    i = np.arange(n)
    gens = []
    if m >= 2:
        t = i.copy()
        t[1], t[2] = 2, 1
        cyc = np.where(i == 0, 0, (i % m) + 1)
        gens = [t, cyc]
    return Graph(f"star{m}", n, _canon(n, e), generators=np.asarray(gens, np.int32).reshape(-1, n))


def spider_pair(a: int, b: int) -> Graph:
    """Two hubs 0 and 1 joined by an edge; hub 0 carries a legs of length 2, hub 1 carries b
    legs of length 2, and the last leg of hub 1 ends in two leaves instead of one.

    The radius-2 light cone of the edge (0, 1) holds 2 + 2a + 2b + 1 qubits; generators
    permute the legs of each hub and swap the two forked leaves.
    """
    if a < 2 or b < 3:
        raise ValueError("spider_pair needs a >= 2, b >= 3")
    e = [(0, 1)]
    nxt = 2
    legs0, legs1 = [], []
    for _ in range(a):
        e += [(0, nxt), (nxt, nxt + 1)]
        legs0.append((nxt, nxt + 1))
        nxt += 2
    for _ in range(b - 1):
        e += [(1, nxt), (nxt, nxt + 1)]
        legs1.append((nxt, nxt + 1))
        nxt += 2
    x = nxt
    e += [(1, x), (x, x + 1), (x, x + 2)]
    n = x + 3
    i = np.arange(n)

    def legs_swap(legs):          # exchange the first two legs
        s = i.copy()
        (c0, l0), (c1, l1) = legs[0], legs[1]
        s[c0], s[l0], s[c1], s[l1] = c1, l1, c0, l0
        return s

    def legs_cycle(legs):         # leg j -> leg j + 1
        s = i.copy()
        for j, (c, l) in enumerate(legs):
            s[c], s[l] = legs[(j + 1) % len(legs)]
        return s

    swap = i.copy()
    swap[x + 1], swap[x + 2] = x + 2, x + 1
    gens = [legs_swap(legs0), legs_cycle(legs0), legs_swap(legs1), legs_cycle(legs1), swap]
    return Graph(f"spider{a},{b}", n, _canon(n, np.array(e)), generators=np.asarray(gens, np.int32))


def single_edge() -> Graph:
    return Graph("K2", 2, np.array([[0, 1]], np.int32), generators=np.array([[1, 0]], np.int32))


def triangle() -> Graph:
    return Graph("K3", 3, np.array([[0, 1], [0, 2], [1, 2]], np.int32),
                 generators=np.array([[1, 2, 0], [1, 0, 2]], np.int32))


def relabel(g: Graph, perm: np.ndarray) -> Graph:
    """Graph with node i renamed perm[i]; edges re-canonicalised and re-sorted.

    Returns the relabelled graph and, through ``edge_map``, where each old edge went.
    Generators are conjugated so that they remain automorphisms.
    """
    perm = np.asarray(perm, np.int64)
    e = perm[g.edges.astype(np.int64)]
    u, v = e.min(1), e.max(1)
    key = u * g.n + v
    order = np.argsort(key, kind="stable")
    edges = np.stack([u[order], v[order]], 1).astype(np.int32)
    w = None if g.weights is None else np.asarray(g.weights)[order]
    inv = np.empty_like(perm)
    inv[perm] = np.arange(g.n)
    gens = g.gens()
    newg = perm[gens[:, inv]] if gens.shape[0] else gens
    out = Graph(g.name + "-relabel", g.n, edges, w, np.asarray(newg, np.int32))
    out.edge_map = np.empty(g.m, np.int64)  # type: ignore[attr-defined]
    out.edge_map[order] = np.arange(g.m)    # type: ignore[attr-defined]
    return out


def degree_root_weights(g: Graph) -> np.ndarray:
    """Edge weights sqrt(deg u + deg v): irrational for most edges (no common unit) and kept
    by every automorphism, so a weighted instance with the graph's own edge-colour symmetry."""
    deg = np.bincount(g.edges.ravel(), minlength=g.n)
    return np.sqrt((deg[g.edges[:, 0]] + deg[g.edges[:, 1]]).astype(np.float64))
