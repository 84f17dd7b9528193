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


def cases():
    with open(PATH) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("c", cases(), ids=lambda c: c["name"])
def test_stored_case_consistent(c):
    g = getattr(W, c["family"])(*c["args"])
    gens = g.gens() if c["reduce"] else None
    ref = oracle.plan(g.n, g.edges, None, gens, c["p"], reduce=c["reduce"], max_k=30)
    assert [int(x) for x in ref["rep"]] == c["rep"]
    np.testing.assert_array_equal(ref["W"], c["W"])
    zz = np.array(c["zz"])
    np.testing.assert_allclose(np.array(c["energy"]), (np.array(c["W"])[None] * (1 - zz) / 2).sum(1),
                               rtol=0, atol=1e-12)
    ga, be = W.draw_angles(c["points"], c["p"], c["seed"])
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
