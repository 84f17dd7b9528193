"""Host-side checks of the byte accounting bench.py reports for cones held in device memory.

The closed form of the algorithmic state bytes per (cone, point) item is checked against a
pass-by-pass count of the adjoint pass program, and the total of the 20-30-qubit workload
(random 3-regular n = 200, p = 3, 8 points) against the cone sizes the oracle's light-cone
extraction gives for that graph (Sec. 2.3), so the GB/s figures can be recomputed from the
cone sizes alone.
"""
import collections

import pytest

import bench
from oracle.cones import light_cone
from oracle.problem import adjacency, canonical_edges
from workloads.graphs import random_regular


def test_pass_groups():
    # group 0 holds 13 stored qubits, every further group up to 9
    for kh in range(14, 32):
        g, left = 1, kh - 13
        while left > 0:
            g, left = g + 1, left - 9
        assert bench.hbm_groups(kh) == g
    assert (bench.hbm_groups(22), bench.hbm_groups(23), bench.hbm_groups(29)) == (2, 3, 3)


def program_sweeps(k, p, ckpt):
    """State sweeps (one read or one write of the stored half) of the adjoint pass program.

    Forward: layers 1 .. p - 1 each visit every group, in alternating order, so the last
    group of a layer is the first of the next and one pass serves both.  Layer 1 starts with
    a generating pass that only writes; every other pass reads and writes the state, the last
    one fused with phase p, the final mixer and the turn of the adjoint (it reads psi and
    writes lambda).  Reverse: every forward pass but the final one is undone in reverse
    order; undoing the generating pass reads lambda only, every other undo reads psi and
    lambda and writes lambda, and psi too unless it reads psi from a stored checkpoint.
    """
    groups = bench.hbm_groups(k - 1)
    visits = (p - 1) * groups
    shared = p - 2                      # layer boundaries served by one pass
    forward = ["gen"] + ["rw"] * (visits - shared - 1)
    n = 1 + 2 * (len(forward) - 1)      # the generating pass writes; the others read and write
    for kind in reversed(forward[:-1]):
        n += 1 if kind == "gen" else (3 if ckpt else 4)
    return n


@pytest.mark.parametrize("k", [16, 20, 23, 24, 27, 30])
@pytest.mark.parametrize("p", [2, 3, 4])
@pytest.mark.parametrize("ckpt", [False, True])
def test_bytes_per_item_match_the_pass_program(k, p, ckpt):
    n = float(1 << (k - 1))
    assert bench.hbm_bytes_per_item(k, p, True, ckpt) == 8.0 * n * program_sweeps(k, p, ckpt)


def test_config5ii_total_bytes():
    # every edge is its own orbit (no generators): 300 cones; the k >= 15 classes are the
    # device-memory ones, all of them here
    g = random_regular(200, 3, 502)
    u, v, _ = canonical_edges(g.n, g.edges, None)
    adj = adjacency(g.n, u, v)
    ks = [len(light_cone(adj, int(a), int(b), 3)[0]) for a, b in zip(u, v)]
    hist = collections.Counter(ks)
    assert hist == {20: 6, 22: 1, 23: 3, 24: 14, 25: 12, 26: 24, 27: 18, 28: 47, 29: 52, 30: 123}
    points = 8
    unc = sum(bench.hbm_bytes_per_item(k, 3, True, False) for k in ks) * points
    ck = sum(bench.hbm_bytes_per_item(k, 3, True, True) for k in ks) * points
    # the algorithmic_GB figures of the two bench objects (uncompute, stored checkpoints)
    assert round(unc / 1e9, 2) == 124808.13
    assert round(ck / 1e9, 2) == 107789.25
