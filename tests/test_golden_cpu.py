"""Integrity of the stored oracle values in tests/golden/oracle_cases.json (CPU).

The cheap case is recomputed in full; for the expensive ones the graph recipe must still
give the stored orbits and weights, the stored energy must be the orbit-weighted sum of the
stored terms, and one small orbit's term is recomputed.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

PATH = os.path.join(os.path.dirname(__file__), "golden", "oracle_cases.json")


def cases(kind="cases"):
    with open(PATH) as f:
        return json.load(f).get(kind, [])


@pytest.mark.parametrize("c", cases(), ids=lambda c: c["name"])
def test_stored_case_consistent(c):
    g = getattr(W, c["family"])(*c["args"])
    gens = g.gens() if c["reduce"] else None
    w = getattr(W, c["weights"])(g) if c.get("weights") else None
    ref = oracle.plan(g.n, g.edges, w, gens, c["p"], reduce=c["reduce"], max_k=30)
    assert [int(x) for x in ref["rep"]] == c["rep"]
    np.testing.assert_array_equal(ref["W"], c["W"])
    ga, be = W.draw_angles(c["points"], c["p"], c["seed"])
    if c["zz"] is None:   # terms not stored: the energy at the first point, recomputed
        E, _ = oracle.energy(ref, ga[:1], be[:1])
        np.testing.assert_allclose(E, c["energy"][:1], rtol=0, atol=1e-9)
        return
    zz = np.array(c["zz"])
    np.testing.assert_allclose(np.array(c["energy"]), (np.array(c["W"])[None] * (1 - zz) / 2).sum(1),
                               rtol=0, atol=1e-12)
    small = [m for m, cone in enumerate(ref["cones"]) if cone["k"] <= 12]
    if len(small) == len(ref["cones"]):
        E, dg, db, zz2 = oracle.energy_grad(ref, ga, be)
        np.testing.assert_allclose(E, c["energy"], rtol=0, atol=1e-12)
        np.testing.assert_allclose(dg, c["dgamma"], rtol=0, atol=1e-12)
        np.testing.assert_allclose(db, c["dbeta"], rtol=0, atol=1e-12)
    else:
        m = small[0] if small else int(np.argmin([cone["k"] for cone in ref["cones"]]))
        sub = dict(ref, cones=[ref["cones"][m]], rep=ref["rep"][[m]], W=ref["W"][[m]])
        _, zzm = oracle.energy(sub, ga, be)
        np.testing.assert_allclose(zzm[:, 0], zz[:, m], rtol=0, atol=1e-12)


@pytest.mark.parametrize("c", cases("term_cases") + cases("term_grad_cases"), ids=lambda c: c["name"])
def test_stored_terms_match_their_cones(c):
    # the stored edges still have cones of the stored sizes in the workload's graph, and the
    # stored values are expectations (|zz| <= 1) of the right shape
    (g, p), = W.workload(c["workload"])[0]
    ref = oracle.plan(g.n, g.edges, None, None, p, reduce=False, max_k=30)
    assert [ref["cones"][e]["k"] for e in c["edges"]] == c["k"]
    zz = np.array(c["zz"])
    assert zz.size == c["points"] * len(c["edges"]) and np.abs(zz).max() <= 1.0
    if "dzz" in c:
        assert np.array(c["dzz"]).shape == (len(c["edges"]), c["points"], 2 * p)
