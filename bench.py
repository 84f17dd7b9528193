"""Benchmark: symmetry-reduced light-cone QAOA energy + adjoint gradient on one MI355X.

Workload (default): the p=2 pair of graphs with a batch of 256 angle points each,
  (i)  circulant C_10000(1,2) with its dihedral generators (2 edge orbits), and
  (ii) a seeded random 3-regular graph with n=10000 (trivial group, 15000 cones of 10-14 qubits).
One step = plan both graphs (orbits + light cones + device tables) and evaluate the energy
and its gradient at all 256 points of each.  value = (graph, point) evaluations per second.

Prints one JSON line.  --gpus N with N > 1 is refused: the library drives one GPU (no sharding).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# HBM traffic of the device-memory pass kernels over their algorithmic bytes, from
# rocprofv3 FETCH_SIZE and WRITE_SIZE runs of `bench.py --hbm-only --hbm-points 1 --copy-gib 4`
# (counters scaled by a 4 GiB device copy; summary in profiles/).  Valid only for the kernel
# sources (and build flags) it was measured on: reported as null once they change.
HBM_TRAFFIC = {"sources_sha256": "fe95b2630654ddb90d6e5b9a8a14cbcbf6f76c4f49b29aeb2756a23dd7c1b9b1",
               "counted_over_algorithmic": 1.031,
               # the program with every cone-size class reading stored forward states
               # (checkpoint_mode 2, --checkpoint-mode 2 in the counter runs)
               "counted_over_algorithmic_ckpt": 1.035}


# Same for the 14-qubit workgroup-resident adjoint kernel: counted bytes per (cone, point)
# item (cut tables and phase rows read, five FP64 results written).
FUSED_TRAFFIC = {"sources_sha256": "a95bec3c946b07d2ac2745d366d5cc15b30f434ca46562838f583d13fd3ba120",
                 "bytes_per_item": 297.8}


def sources_sha256(files) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def hbm_sources_sha256() -> str:
    return sources_sha256(("paper_2101_10296_amd/csrc/hbm_impl.hpp", "paper_2101_10296_amd/csrc/hbm.hip",
                           "paper_2101_10296_amd/csrc/fused_impl.hpp", "paper_2101_10296_amd/build.py"))


def fused_sources_sha256() -> str:
    return sources_sha256(("paper_2101_10296_amd/csrc/fused_impl.hpp", "paper_2101_10296_amd/csrc/fused_k14.hip",
                           "paper_2101_10296_amd/build.py"))


def flops_model_8d(k: int, p: int) -> float:
    """Algorithmic FP32 flops of one forward + adjoint cone evaluation by the hot-path
    model: forward 2^k [p (6 + 3 k_int) + 6k (p - 1) + 12 + 3] (phase complex multiply and
    cut count, full mixers of layers 1..p-1, the last two-qubit mixer, the expectation);
    adjoint 3 x forward + 2^k p (8k + 8) (the inner products with sum_j X_j and C).
    Counted on the stored half of the state (2^(k-1) amplitudes: cones of k >= 3 qubits are
    invariant under flipping every qubit) with k_int = 0: cut values come from a table,
    not a popcount.
    """
    n = float(1 << (k - 1 if k >= 3 else k))
    fwd = p * 6 + 6 * k * (p - 1) + 12 + 3
    return n * (3 * fwd + p * (8 * k + 8))


def hbm_bytes_model_8d(k: int, p: int) -> float:
    """Bytes of the one-sweep-per-layer model of the adjoint on a cone held in device
    memory: 48 p bytes per stored amplitude (forward state stored once per layer, 16 p;
    backward reads and writes psi and lambda once per layer, 32 p)."""
    return 48.0 * p * float(1 << (k - 1))


def flops_fwd_adj(k: int, p: int) -> float:
    """Algorithmic FP32 flops of one forward + adjoint cone evaluation (k qubits, depth p).

    Mixer: 6 flop per amplitude per qubit (c*a - i*s*b); phase: 6 (complex multiply);
    <Z0 Z1>: 4; Im<lambda|X_j|psi>: 4 per amplitude per qubit; Im<lambda|C|psi>: 5.
    Forward: D_1|+> (2), p-1 full layers (6k + 6), last two-qubit mixer (12), zz (4).
    Adjoint (p >= 2): beta_p inner products (8), undo of the last mixer on lambda (12; psi
    before D_p is kept), p gamma inner products (5), D_p undone on lambda (6) and the other
    p-2 phases on two states (12), p-1 full layers undone on two states with their inner
    products (16k; the last stage of layer 1 leaves psi alone, which is not counted).
    p = 1: beta_1 (8), the last mixer undone on two states (24), gamma_1 (5).
    Per stored amplitude: cones of k >= 3 qubits keep only the half of the state with
    qubit k-1 = 0 (the state is invariant under flipping every qubit), 2^(k-1) amplitudes.
    """
    n = float(1 << (k - 1 if k >= 3 else k))
    fwd = 2 + (p - 1) * (6 * k + 6) + 12 + 4
    if p == 1:
        adj = 8 + 24 + 5
    else:
        adj = 8 + 12 + 5 * p + 6 + 12 * (p - 2) + 16 * k * (p - 1)
    return n * (fwd + adj)


def hbm_groups(kh: int) -> int:
    """Pass groups over the kh stored qubits of a cone held in device memory: qubits 0..12,
    then nine at a time."""
    return 1 + (kh - 13 + 8) // 9


def hbm_bytes_per_item(k: int, p: int, grad: bool, ckpt: bool = False) -> float:
    """Algorithmic HBM bytes of one (cone, point) item of the device-memory pass program.

    8 B per stored complex64 amplitude read or written; the stored half of the state has
    2^(k-1) amplitudes (qubit k-1 = 0).  Forward: the first pass writes the state, every
    later pass reads and writes it, the final pass only reads it (with the gradient it also
    writes lambda).  Reverse: every pass but the last reads and writes psi and lambda (with
    stored checkpoints, ckpt, it reads both and writes lambda only); the last (undoing the
    first forward pass) only reads lambda (psi there is regenerated from the cut values).
    p = 1 keeps no state.
    """
    if p == 1:
        return 0.0
    F = (p - 1) * (hbm_groups(k - 1) - 1)   # passes after the first (at least two groups)
    n = float(1 << (k - 1))
    if grad:
        return n * (8 + 16 * (F - 1) + 16 + 8 + (24 if ckpt else 32) * (F - 1))
    return n * (8 + 16 * (F - 1) + 8)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


_POOL_STATE = {}


def _pool_init(graphs, ga, be):
    import oracle
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass
    _POOL_STATE["plans"] = [oracle.plan(g.n, g.edges, None, gens, p, reduce=gens is not None)
                            for g, p, gens in graphs]
    _POOL_STATE["ga"], _POOL_STATE["be"] = ga, be


def _pool_term(args):
    import oracle
    gi, m = args
    pl = _POOL_STATE["plans"][gi]
    sub = dict(pl, cones=[pl["cones"][m]], rep=pl["rep"][[m]], W=pl["W"][[m]])
    oracle.energy_grad(sub, _POOL_STATE["ga"][:1], _POOL_STATE["be"][:1])
    return gi


def oracle_baseline_parallel(graphs, ga, be, budget_s: float, workers: int):
    """The same sampled oracle work spread over `workers` processes (one term per task),
    run for about budget_s seconds of wall time; per graph the extrapolated time is
    wall * M / terms_done.  Call before the GPU is initialised (the pool forks)."""
    import multiprocessing as mp
    import oracle
    Ms = [len(oracle.plan(g.n, g.edges, None, gens, p, reduce=gens is not None)["rep"]) for g, p, gens in graphs]
    ctx = mp.get_context("fork")
    total, desc = 0.0, []
    with ctx.Pool(workers, initializer=_pool_init, initargs=(graphs, ga, be)) as pool:
        pool.map(_pool_term, [(0, 0)] * workers)   # workers have built their plans
        for gi, M in enumerate(Ms):
            order = np.random.default_rng(0).permutation(M)
            done, t0 = 0, time.perf_counter()
            while done < M and time.perf_counter() - t0 < budget_s / len(graphs):
                chunk = [(gi, int(m)) for m in order[done:done + 4 * workers]]
                pool.map(_pool_term, chunk, chunksize=1)
                done += len(chunk)
            t = time.perf_counter() - t0
            total += t * M / done
            desc.append(f"{graphs[gi][0].name}: {done}/{M} terms at 1 point")
    return 1.0 / total * len(graphs), "; ".join(desc)


def oracle_baseline(graphs, ga, be, budget_s: float):
    """FP64 oracle (energy + forward-mode gradient) on a bounded sample of the workload.

    For each graph a fixed random sample of its terms is evaluated at one angle point and
    the time is extrapolated to all terms with t = t_sample * M / M_sample (the paper's
    estimator for runs that did not finish, Sec. 5).  Returns evaluations per second.
    """
    import oracle
    total = 0.0
    desc = []
    per_graph_budget = budget_s / len(graphs)
    for g, p, gens in graphs:
        pl = oracle.plan(g.n, g.edges, None, gens, p, reduce=gens is not None)
        M = len(pl["rep"])
        rng = np.random.default_rng(0)
        order = rng.permutation(M)
        done, t0 = 0, time.perf_counter()
        while done < M:
            m = int(order[done])
            sub = dict(pl, cones=[pl["cones"][m]], rep=pl["rep"][[m]], W=pl["W"][[m]])
            oracle.energy_grad(sub, ga[:1], be[:1])
            done += 1
            if time.perf_counter() - t0 > per_graph_budget:
                break
        t = time.perf_counter() - t0
        total += t * M / done
        desc.append(f"{g.name}: {done}/{M} terms at 1 point")
    return 1.0 / total * len(graphs), "; ".join(desc)


def hbm_measure(Q, torch, W, points: int, ckpt: int = 0) -> dict:
    """Large cones: random 3-regular n=200 at p=3 (300 cones of 20-30 qubits), energy and
    gradient at the first `points` angle points, through the device-memory pass kernels.
    The plan is built and evaluated once (device tables, state buffers), then timed on a
    second evaluation, as in a training loop.

    achieved = algorithmic state bytes (hbm_bytes_per_item x items, summed over cone sizes)
    over the HIP-event time of those kernel groups (passes, zero fill and tile reductions).
    """
    (g, p), = W.workload("c5ii")[0]
    _, ga, be = W.workload("c5ii")
    gt = torch.tensor(ga[:points], dtype=torch.float64, device="cuda")
    bt = torch.tensor(be[:points], dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    pl = Q.Plan(g.n, g.edges, p=p, profile=True, checkpoint_mode=ckpt)
    pl.energy_grad(gt, bt)          # first call: device tables and state buffers
    torch.cuda.synchronize()
    first = time.perf_counter() - t0
    t0 = time.perf_counter()
    pl.energy_grad(gt, bt)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = pl.info()
    stored = info["checkpointed_classes"] > 0
    byts, b8d, ms, by_k = 0.0, 0.0, 0.0, {}
    for k, items, t in pl.kernel_times():
        if k > 14:
            b = hbm_bytes_per_item(k, p, True, bool((info["checkpointed_k_mask"] >> k) & 1)) * items
            byts += b
            b8d += hbm_bytes_model_8d(k, p) * items
            ms += t
            by_k[k] = round(b / (t * 1e-3) / 1e9, 1)
    pl.close()
    gbs = byts / (ms * 1e-3) / 1e9
    traffic = None   # counted HBM bytes of the timed evaluation, if the counters are current
    all_stored = info["checkpointed_classes"] == len(by_k)
    if hbm_sources_sha256() == HBM_TRAFFIC["sources_sha256"] and (all_stored or not stored):
        traffic = round(byts * HBM_TRAFFIC["counted_over_algorithmic_ckpt" if stored else "counted_over_algorithmic"])
    return {"workload": f"random 3-regular n=200 (seed 502), p=3, {points} point(s), energy+gradient, "
                        "300 cones of 20-30 qubits in device memory",
            "adjoint": ("forward states read from stored checkpoints (checkpoint_mode %d, %d of %d cone-size "
                        "classes)" % (ckpt, info["checkpointed_classes"], len(by_k))) if stored
                       else "forward states recovered by inverse layers (checkpoint_mode 0)",
            "evals_per_s": round(points / wall, 4), "wall_s": round(wall, 3),
            "first_call_s_incl_plan_and_alloc": round(first, 3),
            "kernel_ms": round(ms, 2), "algorithmic_GB": round(byts / 1e9, 2),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic},
            "achieved_GBps_by_k": by_k,
            "one_sweep_per_layer_model": {"GB": round(b8d / 1e9, 2),
                                          "GBps": round(b8d / (ms * 1e-3) / 1e9, 1),
                                          "frac": round(b8d / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}}


def config4_measure(Q, torch, W) -> dict:
    """The 48-graph mix (tori, hypercubes, circulants C_n(1,2,5), random 3- and 4-regular
    graphs; p = 1 or 2; 32 angle points each), energy and gradient of every graph: one plan
    per depth over all graphs of that depth (each reduced by its own generators), so one
    call per depth evaluates every graph, with all cones of one size in one launch.  Plans
    are built once and reused (a training step over the 48 graphs).  busy = summed HIP-event
    kernel time over the wall time of the step; the device-memory classes of at least 18
    qubits at p = 2 are reported with their algorithmic bytes over their kernel time."""
    graphs, ga, be = W.workload("c4")
    plans = []
    t0 = time.perf_counter()
    for p in (1, 2):
        inst = [(g.n, g.edges, None, g.gens()) for g, pg in graphs if pg == p]
        gt = torch.tensor(np.ascontiguousarray(ga[:, :p]), dtype=torch.float64, device="cuda")
        bt = torch.tensor(np.ascontiguousarray(be[:, :p]), dtype=torch.float64, device="cuda")
        plans.append((Q.Plan.batch(inst, p, profile=True), gt, bt, p, len(inst)))
    plan_s = time.perf_counter() - t0
    for pl, gt, bt, _, _ in plans:
        pl.energy_grad(gt, bt)
    torch.cuda.synchronize()
    reps = 5
    kern_ms, hbm_b, hbm_ms, hist, launches = 0.0, 0.0, 0.0, {}, 0
    t0 = time.perf_counter()
    for _ in range(reps):
        for pl, gt, bt, p, _ in plans:
            pl.energy_grad(gt, bt)
        torch.cuda.synchronize()
        for pl, gt, bt, p, _ in plans:
            for k, items, ms in pl.kernel_times():
                kern_ms += ms
                if k >= 18 and p >= 2:
                    hbm_b += hbm_bytes_per_item(k, p, True) * items
                    hbm_ms += ms
                if k >= 2:
                    hist[k] = hist.get(k, 0) + items // reps
    wall = (time.perf_counter() - t0) / reps
    n_orb = sum(pl.n_orbits for pl, *_ in plans)
    for pl, *_ in plans:
        pl.close()
    evals = len(graphs) * ga.shape[0]
    return {"workload": "48 graphs (3 tori, Q_8, Q_10, 13 circulants C_n(1,2,5), 15 random 3-regular, "
                        "15 random 4-regular), p in {1, 2}, 32 points each, energy+gradient; one plan per "
                        "depth over its graphs, plans reused",
            "evals_per_s": round(evals / wall, 1), "ms_per_step": round(wall * 1e3, 3),
            "calls_per_step": len(plans), "orbits": n_orb, "plan_s": round(plan_s, 3),
            "gpu_busy_frac": round(kern_ms / reps / (wall * 1e3), 4),
            "items_by_k": {str(k): v for k, v in sorted(hist.items())},
            "hbm_k_ge_18_p2": {"GB": round(hbm_b / reps / 1e9, 3), "kernel_ms": round(hbm_ms / reps, 3),
                               "achieved_GBps": round(hbm_b / (hbm_ms * 1e-3) / 1e9, 1) if hbm_ms else None}}


def tuner_measure(Q, torch, W, gt, bt, graphs, reps: int = 3) -> dict:
    """The bench workload (both p = 2 graphs, 256 points, energy and gradient) with plans
    built once: default layouts against plans with the run-time tuner on (its first call
    times the candidates of every kernel class it meets; the timed calls use the choices)."""
    out = {}
    for tune in (False, True):
        plans = [Q.Plan(g.n, g.edges, p=pp, generators=gens, tune=tune) for g, pp, gens in graphs]
        for pl in plans:
            pl.energy_grad(gt, bt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for pl in plans:
                pl.energy_grad(gt, bt)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out["tuned" if tune else "default"] = {"ms_per_step": round(dt * 1e3, 3),
                                               "evals_per_s": round(len(graphs) * gt.shape[0] / dt, 1)}
        for pl in plans:
            pl.close()
    out["choices"] = [ln for ln in Q.tuning_report().splitlines() if ln]
    return out


def config5i_measure(Q, torch, W) -> dict:
    """Hypercube Q_12 at p = 1: one orbit, one 24-qubit cone; energy and gradient at 8 points
    (the p = 1 pass keeps no state: its roofline is the vector ALU)."""
    (g, p), = W.workload("c5i")[0]
    _, ga, be = W.workload("c5i")
    gt = torch.tensor(ga, dtype=torch.float64, device="cuda")
    bt = torch.tensor(be, dtype=torch.float64, device="cuda")
    pl = Q.Plan(g.n, g.edges, p=p, generators=g.gens(), profile=True)
    pl.energy_grad(gt, bt)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        pl.energy_grad(gt, bt)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    ms = sum(t for k, _, t in pl.kernel_times() if k == 24)
    pl.close()
    return {"workload": "hypercube Q_12 (4096 nodes, 24576 edges, 1 orbit), p=1, 8 points, energy+gradient",
            "evals_per_s": round(ga.shape[0] / wall, 2), "ms_per_call": round(wall * 1e3, 3),
            "kernel_ms_k24": round(ms, 3), "symmetry_reduction": g.m}


def replay_measure(Q, torch, W, calls: int = 200) -> dict:
    """Per-call time of a small training-loop evaluation (energy and gradient of C_10000(1,2)
    reduced to its two orbits, p=2, one angle point), eager launches against graph replay."""
    out = {}
    for name, g, p in (("C10000(1,2) p=2", W.circulant(10000, (1, 2)), 2),):
        ga, be = W.draw_angles(1, p, 77)
        gt = torch.tensor(ga, dtype=torch.float64, device="cuda")
        bt = torch.tensor(be, dtype=torch.float64, device="cuda")
        res = {}
        for mode in (False, True):
            pl = Q.Plan(g.n, g.edges, p=p, generators=g.gens(), graph=mode)
            o = (torch.empty(1, dtype=torch.float64, device="cuda"), torch.empty_like(gt), torch.empty_like(bt))
            for _ in range(3):
                pl.energy_grad(gt, bt, out=o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(calls):
                pl.energy_grad(gt, bt, out=o)
            torch.cuda.synchronize()
            res["replay_us" if mode else "eager_us"] = round((time.perf_counter() - t0) / calls * 1e6, 1)
            pl.close()
        out[name] = res
    return out


def training_measure(Q, torch, W, steps: int = 20) -> dict:
    """Multi-start Adam training: random 3-regular n=1000 (seed 3), p=2, 64 starts (seed 300),
    one batched energy + gradient call per step on a plan built once."""
    from paper_2101_10296_amd.train import adam_ascent
    (g, p), = W.workload("c3")[0]
    _, ga, be = W.workload("c3")
    gt = torch.tensor(ga, dtype=torch.float64, device="cuda")
    bt = torch.tensor(be, dtype=torch.float64, device="cuda")
    pl = Q.Plan(g.n, g.edges, p=p)
    adam_ascent(pl, gt, bt, steps=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, E, hist = adam_ascent(pl, gt, bt, steps=steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pl.close()
    return {"workload": "random 3-regular n=1000, p=2, 64 starts, Adam lr 0.02", "steps": steps,
            "steps_per_s": round(steps / dt, 2), "evals_per_s": round(steps * ga.shape[0] / dt, 1),
            "mean_cut_fraction_first_last": [round(float(hist[0].mean()) / g.m, 4),
                                              round(float(E.mean()) / g.m, 4)]}


def generator_measure(Q, W, torch) -> dict:
    """Automorphism generators found by the library's search (host) for the 100 x 100 torus,
    the paper's grid-w-2-100 row, and the edge orbits they give; then, as the paper counts
    it, the speedup of symmetry-reduced evaluation with the search time included over the
    unreduced evaluation, for cheap terms (C_10000(1,2,5), p = 1) and expensive ones
    (C_1000(1,2,5), p = 2, cones of 20-22 qubits)."""
    g = W.torus2d(100)
    t0 = time.perf_counter()
    gens, complete = Q.find_generators(g.n, g.edges)
    dt = time.perf_counter() - t0
    pl = Q.Plan(g.n, g.edges, p=1, generators=gens)
    n_orb = pl.info()["n_orbits"]
    pl.close()
    out = {"graph": "torus 100x100 (10000 nodes, 20000 edges)", "seconds": round(dt, 3),
           "generators": int(len(gens)), "complete": bool(complete), "edge_orbits": int(n_orb),
           "paper_t_aut_s_context": 58.70}

    def speedup(c, p, P, label):
        ga, be = W.draw_angles(P, p, 5)
        gt = torch.tensor(ga, dtype=torch.float64, device="cuda")
        bt = torch.tensor(be, dtype=torch.float64, device="cuda")

        def unreduced():
            p_ = Q.Plan(c.n, c.edges, p=p, reduce=False)
            r = p_.energy_grad(gt, bt)
            torch.cuda.synchronize()
            p_.close()
            return r

        def discovered():
            gs, _ = Q.find_generators(c.n, c.edges)
            p_ = Q.Plan(c.n, c.edges, p=p, generators=gs)
            r = p_.energy_grad(gt, bt)
            torch.cuda.synchronize()
            p_.close()
            return r

        unreduced(), discovered()   # warm-up
        t0 = time.perf_counter()
        Eu = unreduced()[0]
        t_unr = time.perf_counter() - t0
        t0 = time.perf_counter()
        Er = discovered()[0]
        t_red = time.perf_counter() - t0
        return {"graph": label, "unreduced_s": round(t_unr, 4), "search_plus_reduced_s": round(t_red, 4),
                "speedup": round(t_unr / t_red, 2), "max_abs_dE": float((Eu - Er).abs().max())}

    # cheap terms (p = 1, cones of at most 12 qubits) and expensive ones (p = 2, cones of
    # 20-22 qubits in device memory); plan and search included in both timings
    out["discovered_symmetry"] = [
        speedup(W.circulant(10000, (1, 2, 5)), 1, 64, "C_10000(1,2,5), p=1, 64 points, energy+gradient"),
        speedup(W.circulant(1000, (1, 2, 5)), 2, 2, "C_1000(1,2,5), p=2, 2 points, energy+gradient"),
    ]
    out["paper_median_speedup_context"] = 4.06
    return out


def rqaoa_measure(W) -> dict:
    """Recursive QAOA on random 3-regular n=200 (seed 502) at p=1 with fixed angles: one plan
    and one correlation evaluation per eliminated variable, down to 10 variables."""
    import numpy as np

    from paper_2101_10296_amd.rqaoa import rqaoa
    g = W.random_regular(200, 3, 502)
    t0 = time.perf_counter()
    z, cut, steps = rqaoa(g.n, g.edges, None, 1, lambda k, n: ([0.6], [0.4]), n_stop=10)
    dt = time.perf_counter() - t0
    return {"workload": "random 3-regular n=200, p=1, fixed angles, down to 10 variables",
            "steps": len(steps), "steps_per_s": round(len(steps) / dt, 1), "cut_fraction": round(cut / g.m, 4)}


def copy_measure(torch, gib: float) -> dict:
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    return {"bytes_each_way": n * 4, "ms": round(ms, 3), "GBps_read_plus_write": round(2 * n * 4 / ms / 1e6, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--hbm-points", type=int, default=8,
                    help="angle points of the large-cone (device-memory) measurement; 0 = skip")
    ap.add_argument("--hbm-only", action="store_true", help="only the large-cone measurement")
    ap.add_argument("--checkpoint-mode", type=int, default=0, help="adjoint mode of --hbm-only (0, 1, 2)")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="also time a device-to-device copy of this many GiB (counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "the library drives one GPU (no sharding across GPUs); --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2101_10296_amd as Q
    import workloads as W

    if a.hbm_only:
        out = {"hbm": hbm_measure(Q, torch, W, max(a.hbm_points, 1), ckpt=a.checkpoint_mode)}
        if a.copy_gib > 0:
            out["copy"] = copy_measure(torch, a.copy_gib)
        print(json.dumps(out), flush=True)
        return

    (g1, p), = W.workload("c2i")[0]
    (g2, _), = W.workload("c2ii")[0]
    _, ga, be = W.workload("c2i")
    P = ga.shape[0]
    graphs = [(g1, p, g1.gens()), (g2, p, None)]
    cpu_par = None
    if not a.no_cpu_baseline:
        # the oracle on all host cores first: the pool forks, so the GPU is not touched yet
        workers = max(1, min(16, os.cpu_count() or 1))
        v_par, sample_par = oracle_baseline_parallel(graphs, ga, be, a.cpu_budget, workers)
        cpu_par = (v_par, sample_par, workers)
    gt = torch.tensor(ga, dtype=torch.float64, device="cuda")
    bt = torch.tensor(be, dtype=torch.float64, device="cuda")

    def step(profile=False):
        out = []
        for g, pp, gens in graphs:
            pl = Q.Plan(g.n, g.edges, p=pp, generators=gens, profile=profile)
            E, dg, db = pl.energy_grad(gt, bt)
            out.append((pl, E, dg, db))
        return out

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    kernel_ms = {}
    t0 = time.perf_counter()
    for _ in range(a.steps):
        res = step(profile=True)
        torch.cuda.synchronize()
        for pl, *_ in res:
            for k, items, ms in pl.kernel_times():
                key = (pl.info()["n_orbits"], k)
                d = kernel_ms.setdefault(key, [0.0, 0, pl.p])
                d[0] += ms
                d[1] += items
            pl.close()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt / a.steps * 1e3
    evals = len(graphs) * P
    value = evals / (dt / a.steps)

    # dominant kernel: the cone-size group with the largest total time
    (norb, kdom), (ms_dom, items_dom, pdom) = max(((k, v) for k, v in kernel_ms.items() if k[1] >= 2),
                                                  key=lambda kv: kv[1][0])
    flop = flops_model_8d(kdom, pdom) * items_dom
    achieved = flop / (ms_dom * 1e-3) / 1e12
    executed = flops_fwd_adj(kdom, pdom) * items_dom / (ms_dom * 1e-3) / 1e12
    traffic = None   # counted HBM bytes per launch, if the counters are current for this kernel
    if kdom == 14 and fused_sources_sha256() == FUSED_TRAFFIC["sources_sha256"]:
        traffic = round(FUSED_TRAFFIC["bytes_per_item"] * items_dom / a.steps)
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
                "kernel": f"k_fused<K={kdom},grad>", "avg_launch_ms": round(ms_dom / a.steps, 4),
                "items_per_launch": items_dom // a.steps,
                "flop_per_item": flops_model_8d(kdom, pdom),
                "executed_model": {"flop_per_item": flops_fwd_adj(kdom, pdom), "TFLOPs": round(executed, 3),
                                   "frac": round(executed / PEAK_FP32_TFLOPS, 4)}}

    extra = {}
    if not a.no_plain:
        # plain path: same kernels, one (cone, point) item per launch, 2 points of graph (ii)
        plain = Q.Plan(g2.n, g2.edges, p=p, one_cone_at_a_time=True)
        plain.energy_grad(gt[:1], bt[:1])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plain.energy_grad(gt[:2], bt[:2])
        torch.cuda.synchronize()
        t_plain = (time.perf_counter() - t1) / 2
        batched = Q.Plan(g2.n, g2.edges, p=p)
        batched.energy_grad(gt, bt)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        batched.energy_grad(gt, bt)
        torch.cuda.synchronize()
        t_batched = (time.perf_counter() - t2) / P
        extra["plain_evals_per_s_rand3reg"] = round(1.0 / t_plain, 3)
        extra["batched_evals_per_s_rand3reg"] = round(1.0 / t_batched, 3)
        extra["speedup_vs_plain"] = round(t_plain / t_batched, 2)
        plain.close()
        batched.close()
        # symmetry speedup on the circulant: unreduced all-edge plan over the reduced one,
        # each timed over 100 calls (energy and gradient at all 256 points, plans reused)
        red = Q.Plan(g1.n, g1.edges, p=p, generators=g1.gens())
        unr = Q.Plan(g1.n, g1.edges, p=p, reduce=False)
        for pl in (red, unr):
            pl.energy_grad(gt, bt)
        torch.cuda.synchronize()
        ts = []
        for pl in (red, unr):
            t3 = time.perf_counter()
            for _ in range(100):
                pl.energy_grad(gt, bt)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t3) / 100)
        extra["symmetry_speedup_circulant"] = {"reduced_ms": round(ts[0] * 1e3, 4),
                                               "unreduced_ms": round(ts[1] * 1e3, 4),
                                               "speedup": round(ts[1] / ts[0], 1), "calls": 100}
        red.close()
        unr.close()
        extra["graph_replay"] = replay_measure(Q, torch, W)
        extra["training"] = training_measure(Q, torch, W)
        extra["generator_search"] = generator_measure(Q, W, torch)
        try:
            extra["rqaoa"] = rqaoa_measure(W)
        except Exception as ex:   # a contracted graph can outgrow the cone limit
            extra["rqaoa"] = {"error": str(ex)[:200]}

    line = {
        "metric": "QAOA energy+grad evals/s (batched adjoint vs plain); achieved HBM GB/s",
        "value": round(value, 3), "unit": "evals/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "p=2 energy+gradient: C_10000(1,2) reduced (2 orbits) + random 3-regular "
                               "n=10000 (15000 cones), 256 angle points each, plan included per step",
                   "points_per_graph": P, "p": p, "parallelism": "single GPU"},
        "roofline": roofline,
    }
    line.update(extra)
    if not a.no_plain:
        line["tuner"] = tuner_measure(Q, torch, W, gt, bt, graphs)
        line["config4"] = config4_measure(Q, torch, W)
        line["config5i"] = config5i_measure(Q, torch, W)
    if a.hbm_points > 0:
        line["hbm"] = hbm_measure(Q, torch, W, a.hbm_points)
        # the same workload with the adjoint reading stored forward states where the budget
        # allows (checkpoint_mode 2): time and bytes beside the uncompute program
        line["hbm_checkpointed"] = hbm_measure(Q, torch, W, a.hbm_points, ckpt=2)
        # context for the HBM fraction: what a plain 4 GiB device-to-device copy reaches here
        line["hbm"]["device_copy_GBps"] = copy_measure(torch, 4.0)["GBps_read_plus_write"]
    if a.copy_gib > 0:
        line["copy"] = copy_measure(torch, a.copy_gib)
    if not a.no_cpu_baseline:
        try:   # the oracle is element-wise numpy (one thread); pin any BLAS pool to one thread too
            from threadpoolctl import threadpool_limits
            with threadpool_limits(1):
                v, sample = oracle_baseline(graphs, ga, be, a.cpu_budget)
        except ImportError:
            v, sample = oracle_baseline(graphs, ga, be, a.cpu_budget)
        v_par, sample_par, workers = cpu_par
        line["cpu_baseline"] = {"value": round(v_par, 6), "unit": "evals/s", "cores": workers, "kind": "oracle",
                                "sample": sample_par + f" per graph, one term per task over {workers} processes "
                                          f"(FP64 numpy, {cpu_model()}, nproc {os.cpu_count()}, "
                                          "extrapolated to all terms)",
                                "one_core": {"value": round(v, 6), "cores": 1, "sample": sample}}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
