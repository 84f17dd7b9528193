"""Write oracle_cases.json: FP64 oracle values for workloads whose oracle run takes minutes.

The GPU tests compare the HIP path against these stored values instead of re-running the
oracle.  Only ``oracle`` and the seeded ``workloads`` generators are called here; rerun
this script after any change to the oracle's arithmetic:

    python tests/golden/make_oracle_golden.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

# name -> (graph family, its arguments, p, reduce, number of angle points, angle seed)
CASES = {
    "c1_rand3_n16_p1": ("random_regular", [16, 3, 0], 1, False, 1, 100),
    # three pass groups (23-qubit cone) at p = 2
    "spider5_5_p2": ("spider_pair", [5, 5], 2, True, 2, 601),
    # two pass groups at p = 3 (20-, 21- and 22-qubit cones)
    "C60_1_2_3_p3": ("circulant", [60, [1, 2, 3]], 3, True, 1, 602),
}


def graph_of(family, args):
    return getattr(W, family)(*args)


def run(name):
    fam, args, p, reduce, P, seed = CASES[name]
    g = graph_of(fam, args)
    gens = g.gens() if reduce else None
    ref = oracle.plan(g.n, g.edges, None, gens, p, reduce=reduce, max_k=30)
    ga, be = W.draw_angles(P, p, seed)
    t = time.time()
    E, dg, db, zz = oracle.energy_grad(ref, ga, be)
    print(f"{name}: {len(ref['rep'])} orbits, cones {sorted(c['k'] for c in ref['cones'])}, "
          f"{time.time() - t:.0f} s", flush=True)
    return dict(name=name, family=fam, args=args, p=p, reduce=reduce, points=P, seed=seed,
                rep=[int(x) for x in ref["rep"]], W=[float(x) for x in ref["W"]],
                energy=E.tolist(), zz=np.asarray(zz).tolist(), dgamma=dg.tolist(), dbeta=db.tolist())


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_cases.json")
    cases = [run(n) for n in (sys.argv[1:] or CASES)]
    with open(out, "w") as f:
        json.dump({"generator": "tests/golden/make_oracle_golden.py", "cases": cases}, f, indent=1)
        f.write("\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
