"""Reverse causal cone of a MaxCut edge term (oracle step O3).

Sec. 2.3: conjugating Z_u Z_v by the last mixer leaves support {u, v}; each phase
layer adds every qubit that shares a Hamiltonian term with the current support.
After p layers the support is the ball B_p of radius p (graph distance) around
{u, v}.  The cone simulated here is the subgraph induced by B_p with every induced
edge present at every layer and a mixer on every qubit at every layer; gates outside
the minimal cone commute through the observable and cancel, so this is exact.

Qubit order inside the cone (the paper is silent): u -> 0, v -> 1, the remaining
ball vertices sorted by (distance, vertex id).
"""
from __future__ import annotations


def light_cone(adj, u: int, v: int, p: int):
    """Return (nodes, local_edges, local_edge_ids).

    ``nodes[i]`` is the graph vertex of cone qubit i; ``local_edges`` is a list of
    (a, b) qubit pairs with a < b, ``local_edge_ids`` the graph edge index of each.
    """
    dist = {u: 0, v: 0}
    frontier = [u, v]
    for d in range(1, p + 1):
        nxt = set()
        for x in frontier:
            for y, _ in adj[x]:
                if y not in dist:
                    nxt.add(y)
        for y in nxt:
            dist[y] = d
        frontier = sorted(nxt)
    rest = sorted((x for x in dist if x not in (u, v)), key=lambda x: (dist[x], x))
    nodes = [u, v] + rest
    local = {x: i for i, x in enumerate(nodes)}
    edges, ids = [], []
    seen = set()
    for x in nodes:
        for y, eid in adj[x]:
            if y in local and eid not in seen:
                seen.add(eid)
                a, b = local[x], local[y]
                edges.append((min(a, b), max(a, b)))
                ids.append(eid)
    return nodes, edges, ids
