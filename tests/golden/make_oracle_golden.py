"""Write oracle_cases.json: FP64 oracle values for workloads whose oracle run takes minutes.

The GPU tests compare the HIP path against these stored values instead of re-running the
oracle.  Only ``oracle`` and the seeded ``workloads`` generators are called here; rerun
this script after any change to the oracle's arithmetic:

    python tests/golden/make_oracle_golden.py [--jobs N] [case names...]

Named cases replace their stored entries; the other stored cases are kept.  Each task is
one oracle call on one angle point (full cases) or one cone (term cases), so the points
and cones run in parallel processes; results are only stacked, never combined.
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

# Full cases: energy, per-orbit <Z_u Z_v> and gradient of every orbit.
# name -> (graph family, its arguments, p, reduce, number of angle points, angle seed
#          [, name of the workloads function giving the edge weights])
CASES = {
    "c1_rand3_n16_p1": ("random_regular", [16, 3, 0], 1, False, 1, 100),
    # two pass groups of stored qubits (23-qubit cone: 22 stored qubits) at p = 2
    "spider5_5_p2": ("spider_pair", [5, 5], 2, True, 2, 601),
    # two pass groups at p = 3 (20-, 21- and 22-qubit cones)
    "C60_1_2_3_p3": ("circulant", [60, [1, 2, 3]], 3, True, 1, 602),
    # three pass groups (25-qubit cones: 24 stored qubits) at p = 2 (one such cone) and
    # p = 3 (four such cones)
    "spider5_6_p2": ("spider_pair", [5, 6], 2, True, 2, 611),
    "spider5_6_p3": ("spider_pair", [5, 6], 3, True, 2, 612),
    # the same graph with weights sqrt(deg u + deg v) (no common unit, kept by the
    # generators: real cut values) at p = 2
    "spider5_6_p2_rootw": ("spider_pair", [5, 6], 2, True, 2, 613, "degree_root_weights"),
    # random 3-regular n = 1000, p = 2 (1500 cones of 10-14 qubits): energy and gradient at
    # all 64 angle points of that workload (its per-term values are not stored)
    "c3_rand3_n1000_p2_all": ("random_regular", [1000, 3, 3], 2, False, 64, 300),
}
NO_TERMS = {"c3_rand3_n1000_p2_all"}

# Term cases: forward <Z_u Z_v> of selected edges of an unreduced plan, at the first
# `points` angle points of a workload.  name -> (workload name, edge indices, points)
# random 3-regular n = 200, p = 3: the first two edges whose cones have 24, 25 and 26
# qubits (three pass groups of stored qubits) and edge 0, whose cone has 29 qubits.
TERM_CASES = {
    "c5ii_terms_k24_29": ("c5ii", [4, 21, 23, 65, 15, 16, 0], 1),
}
# Term-gradient cases: <Z_u Z_v> and its derivatives in (gamma_1..p, beta_1..p) of selected
# edges of an unreduced plan.  name -> (workload name, edge indices, points)
# random 3-regular n = 200, p = 3: the first edges whose cones have 24 and 25 qubits.
TERM_GRAD_CASES = {
    "c5ii_term_grads_k24_25": ("c5ii", [4, 23], 1),
}


def graph_of(family, args):
    return getattr(W, family)(*args)


def weights_of(name, g):
    spec = CASES[name]
    return getattr(W, spec[6])(g) if len(spec) > 6 else None


def _full_task(args):
    name, i = args
    fam, gargs, p, reduce, P, seed = CASES[name][:6]
    g = graph_of(fam, gargs)
    ref = oracle.plan(g.n, g.edges, weights_of(name, g), g.gens() if reduce else None, p, reduce=reduce, max_k=30)
    ga, be = W.draw_angles(P, p, seed)
    t = time.time()
    E, dg, db, zz = oracle.energy_grad(ref, ga[i:i + 1], be[i:i + 1])
    print(f"{name} point {i}: cones {[c['k'] for c in ref['cones']]}, {time.time() - t:.0f} s", flush=True)
    return E, dg, db, zz


def _term_task(args):
    name, e = args
    wl, _, P = TERM_CASES[name]
    (g, p), = W.workload(wl)[0]
    _, ga, be = W.workload(wl)
    ref = oracle.plan(g.n, g.edges, None, None, p, reduce=False, max_k=30)
    sub = dict(ref, cones=[ref["cones"][e]], rep=ref["rep"][[e]], W=ref["W"][[e]])
    t = time.time()
    _, zz = oracle.energy(sub, ga[:P], be[:P])
    print(f"{name} edge {e}: k = {ref['cones'][e]['k']}, {time.time() - t:.0f} s", flush=True)
    return ref["cones"][e]["k"], zz[:, 0]


def _term_grad_task(args):
    name, e = args
    wl, _, P = TERM_GRAD_CASES[name]
    (g, p), = W.workload(wl)[0]
    _, ga, be = W.workload(wl)
    ref = oracle.plan(g.n, g.edges, None, None, p, reduce=False, max_k=30)
    cone = ref["cones"][e]
    cut = oracle.cut_values(cone["k"], cone["edges"], cone["weights"])
    t = time.time()
    rows = [oracle.zz_and_grad(cone["k"], cut, ga[i], be[i]) for i in range(P)]
    print(f"{name} edge {e}: k = {cone['k']}, {time.time() - t:.0f} s", flush=True)
    return cone["k"], [r[0] for r in rows], [np.concatenate([r[1], r[2]]).tolist() for r in rows]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=1)
    ap.add_argument("names", nargs="*")
    a = ap.parse_args()
    names = a.names or list(CASES) + list(TERM_CASES) + list(TERM_GRAD_CASES)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_cases.json")
    stored = {"cases": [], "term_cases": [], "term_grad_cases": []}
    if os.path.exists(out):
        with open(out) as f:
            stored.update(json.load(f))
    tasks = [("full", (n, i)) for n in names if n in CASES for i in range(CASES[n][4])]
    tasks += [("term", (n, e)) for n in names if n in TERM_CASES for e in TERM_CASES[n][1]]
    tasks += [("tgrad", (n, e)) for n in names if n in TERM_GRAD_CASES for e in TERM_GRAD_CASES[n][1]]
    with mp.Pool(a.jobs) as pool:
        res = pool.map(_run_task, tasks, chunksize=1)
    done = dict(zip([t[1] for t in tasks], res))
    for n in names:
        if n in CASES:
            fam, gargs, p, reduce, P, seed = CASES[n][:6]
            g = graph_of(fam, gargs)
            ref = oracle.plan(g.n, g.edges, weights_of(n, g), g.gens() if reduce else None, p, reduce=reduce, max_k=30)
            parts = [done[(n, i)] for i in range(P)]
            case = dict(name=n, family=fam, args=gargs, p=p, reduce=reduce, points=P, seed=seed,
                        weights=CASES[n][6] if len(CASES[n]) > 6 else None,
                        rep=[int(x) for x in ref["rep"]], W=[float(x) for x in ref["W"]],
                        energy=np.concatenate([r[0] for r in parts]).tolist(),
                        zz=None if n in NO_TERMS else np.concatenate([r[3] for r in parts]).tolist(),
                        dgamma=np.concatenate([r[1] for r in parts]).tolist(),
                        dbeta=np.concatenate([r[2] for r in parts]).tolist())
            key = "cases"
        elif n in TERM_GRAD_CASES:
            wl, edges, P = TERM_GRAD_CASES[n]
            parts = [done[(n, e)] for e in edges]
            case = dict(name=n, workload=wl, edges=edges, points=P, k=[int(r[0]) for r in parts],
                        zz=[r[1] for r in parts], dzz=[r[2] for r in parts])
            key = "term_grad_cases"
        else:
            wl, edges, P = TERM_CASES[n]
            parts = [done[(n, e)] for e in edges]
            case = dict(name=n, workload=wl, edges=edges, points=P, k=[int(r[0]) for r in parts],
                        zz=np.stack([r[1] for r in parts], axis=1).tolist())
            key = "term_cases"
        stored[key] = [c for c in stored[key] if c["name"] != n] + [case]
    with open(out, "w") as f:
        json.dump({"generator": "tests/golden/make_oracle_golden.py", "cases": stored["cases"],
                   "term_cases": stored["term_cases"], "term_grad_cases": stored["term_grad_cases"]}, f, indent=1)
        f.write("\n")
    print("wrote", out)


def _run_task(t):
    kind, args = t
    return {"full": _full_task, "term": _term_task, "tgrad": _term_grad_task}[kind](args)


if __name__ == "__main__":
    main()
