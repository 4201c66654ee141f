"""Benchmark: KIFMM particles/s for tree + forward + adjoint on one MI355X.

One step = one pass of the whole hot path over the clustered 1,048,576-charge
Laplace workload (60 % uniform + 40 % in 20 Gaussian clusters, p = 6, leaf 128,
adaptive octree): re-tree at the positions (keys, sort, octree, lists), the
forward evaluation (u, E) and the adjoint (dL/dq, dL/dx for given dL/du,
dL/dE).  Inputs are resident in HBM before the timed region starts.

Prints one JSON line.  The headline path is the split-bf16 M2L (all else
FP32); the plain FP32 path is measured beside it.  The roofline object is for
the kernel with the largest share of a forward evaluation, timed with HIP
events on the stream it is launched on.  The CPU baseline is the FP64 oracle
(test infrastructure) timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3, "bf16": 2500.0, "hbm": 8000.0}     # TFLOP/s, TFLOP/s, GB/s
P2P_FLOP_PER_PAIR = 20
METRIC = "FMM particles/sec fwd+adjoint at rel-L2<=1e-5; %FP32/MFMA peak vs plain FP32"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_path(Plan, w, pos, q, gu, gE, precision, steps, warmup):
    import torch
    plan = Plan(pos, w.kernel, w.p, w.leaf_size, w.adaptive, w.max_depth, precision=precision, root=w.root,
                profile=True)
    counts = plan.counts()
    phases = []

    def step(record):
        plan.rebuild(pos)
        u, E = plan.evaluate(q)
        if record:
            phases.append(plan.phase_times())
        gq, gx = plan.backward(q, gu, gE)
        return u, E, gq, gx

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step(True)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    # split of one step (untimed repetitions)
    torch.cuda.synchronize()
    a = time.perf_counter()
    plan.rebuild(pos)
    torch.cuda.synchronize()
    b = time.perf_counter()
    plan.evaluate(q)
    torch.cuda.synchronize()
    c = time.perf_counter()
    plan.backward(q, gu, gE)
    torch.cuda.synchronize()
    d = time.perf_counter()
    ph = {k: float(np.mean([p[k] for p in phases])) for k in phases[0]}
    res = dict(ms_per_step=1e3 * t, t_tree_ms=1e3 * (b - a), t_fwd_ms=1e3 * (c - b), t_adj_ms=1e3 * (d - c),
               phases_fwd_ms=ph, counts=counts, outputs=[o.detach() for o in out])
    plan.close()
    return res


def roofline(res, n, precision):
    ph = res["phases_fwd_ms"]
    c = res["counts"]
    cand = {"m2l": ph["m2l"], "p2p": ph["p2p"]}
    dom = max(cand, key=cand.get)
    if dom == "m2l":
        flops = 2.0 * n * n * c["v_pairs"]
        peak = PEAK["bf16"] if precision == "split_bf16" else PEAK["fp32"]
        ach = flops / (ph["m2l"] * 1e-3) / 1e12
        return dict(kernel="k_m2l", bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak,
                    traffic=None, per_launch_ms=ph["m2l"], work=f"2 n^2 x {c['v_pairs']} V pairs")
    flops = P2P_FLOP_PER_PAIR * c["p2p_pairs"]
    ach = flops / (ph["p2p"] * 1e-3) / 1e12
    return dict(kernel="k_p2p", bound="alu", achieved=ach, peak=PEAK["fp32"], unit="TFLOP/s",
                frac=ach / PEAK["fp32"], traffic=None, per_launch_ms=ph["p2p"],
                work=f"20 x {c['p2p_pairs']} pairs")


def cpu_baseline(seconds_target=20.0):
    """FP64 oracle forward + adjoint on a bounded sample of the same workload."""
    import workloads
    from oracle import kifmm
    n = 65536
    w = workloads.make(2, n=n)
    rng = np.random.default_rng(5)
    ub = rng.standard_normal(n)
    Eb = rng.standard_normal((n, 3))
    t0 = time.perf_counter()
    P = kifmm.plan(w.positions, w.kernel, w.p, w.leaf_size, w.adaptive, w.max_depth, w.root)
    kifmm.forward(P, w.charges)
    kifmm.vjp(P, w.charges, ub, Eb)
    t = time.perf_counter() - t0
    threads = os.environ.get("OMP_NUM_THREADS")
    cores = int(threads) if threads else (os.cpu_count() or 1)
    return dict(value=n / t, unit="particles/s", cores=cores, kind="oracle",
                sample=f"clustered workload generator at N={n} (same p, leaf, tree rules): "
                       f"tree+lists+forward+adjoint in FP64, {t:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None, help="override the number of charges")
    ap.add_argument("--paths", default="split_bf16,fp32")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import workloads
    from paper_2512_09478_amd import Plan
    w = workloads.make(2, n=args.n)
    n = w.n
    pos = torch.tensor(w.positions, dtype=torch.float64, device="cuda")
    q = torch.tensor(w.charges, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(77)
    gu = torch.tensor(workloads.round_f32(rng.standard_normal(n)), dtype=torch.float32, device="cuda")
    gE = torch.tensor(workloads.round_f32(rng.standard_normal((n, 3))), dtype=torch.float32, device="cuda")
    paths = {}
    for prec in args.paths.split(","):
        log(f"[bench] {prec}: N={n} steps={args.steps} warmup={args.warmup}")
        paths[prec] = run_path(Plan, w, pos, q, gu, gE, prec, args.steps, args.warmup)
        r = paths[prec]
        log(f"[bench] {prec}: {r['ms_per_step']:.3f} ms/step  tree {r['t_tree_ms']:.2f} fwd {r['t_fwd_ms']:.2f} "
            f"adj {r['t_adj_ms']:.2f}  phases {json.dumps({k: round(v, 3) for k, v in r['phases_fwd_ms'].items()})}")
    head = "split_bf16" if "split_bf16" in paths else next(iter(paths))
    H = paths[head]
    ops_n = H["counts"]["surface_points"]
    agree = {}
    if "fp32" in paths and "split_bf16" in paths:
        for name, i in (("u", 0), ("E", 1), ("qbar", 2), ("xbar", 3)):
            a = paths["split_bf16"]["outputs"][i].double()
            b = paths["fp32"]["outputs"][i].double()
            agree[name] = float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    out = {
        "metric": METRIC,
        "value": n / (H["ms_per_step"] * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": H["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (M2L bf16x3 split, FP32 accumulate)" if head == "split_bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": "clustered Laplace charges (60% uniform + 40% in 20 Gaussian clusters "
                               "sigma=0.02, N(0,1) charges mean removed), p=6, leaf 128, adaptive octree; "
                               "step = re-tree + forward + adjoint",
                   "n": n, "p": w.p, "leaf_size": w.leaf_size, "path": head},
        "roofline": roofline(H, ops_n, head),
        "paths": {k: {"particles_per_s": n / (v["ms_per_step"] * 1e-3), "ms_per_step": v["ms_per_step"],
                      "t_tree_ms": v["t_tree_ms"], "t_fwd_ms": v["t_fwd_ms"], "t_adj_ms": v["t_adj_ms"],
                      "phases_fwd_ms": v["phases_fwd_ms"], "roofline": roofline(v, ops_n, k)}
                  for k, v in paths.items()},
        "counts": H["counts"],
        "split_vs_fp32_rel_l2": agree,
    }
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
    for v in paths.values():
        v.pop("outputs", None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
