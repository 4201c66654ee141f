"""Benchmark: KIFMM particles/s for tree + forward + adjoint on one MI355X.

One step = one pass of the whole hot path over the clustered 1,048,576-charge
Laplace workload (60 % uniform + 40 % in 20 Gaussian clusters, p = 6, leaf 128,
adaptive octree): re-tree at the positions (keys, sort, octree, lists), the
forward evaluation (u, E) and the adjoint (dL/dq, dL/dx for given dL/du,
dL/dE).  Inputs are resident in HBM before the timed region starts.
``--workload k`` measures the other generators the same way (for the clump
workload the forward pass is the force and torque of the registered clumps
and the adjoint the gradient of a linear loss on them).

Prints one JSON line.  The headline path is the split-bf16 M2L (all else
FP32); the plain FP32 path is measured beside it.  The roofline object is for
the kernel with the most time per step, timed with HIP events that the
library records on the stream the kernel is launched on (read after the
timed region).  The line also carries the largest single-GPU workload (8.4M
Plummer masses, p = 8) on the headline path, the timing of the dipole,
field-gradient and Stokeslet sums on the headline workload (`--f4` adds their
oracle check), the oracle's check of the timed outputs on 256 sampled targets
(rel-L2 and worst element per output and path), and the CPU baseline: the
FP64 oracle (test infrastructure) timed on a bounded sample of the same
workload.
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
CSRC = os.path.join(ROOT, "paper_2512_09478_amd", "csrc")
KERNEL_SOURCE = {"k_m2l": "farfield.hip", "k_p2p": "nearfield.hip"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "kifmm_clustered_1M_p6_hbm_traffic.md")
# the counter summary of each path (the headline's split path in TRAFFIC_FILE)
TRAFFIC_FILES = {"split_bf16": TRAFFIC_FILE,
                 "fp32": os.path.join(ROOT, "profiles", "kifmm_clustered_1M_p6_fp32_hbm_traffic.md")}
CALIB_BYTES = 256 << 20     # the plain copy used to calibrate the byte counters
P2P_FLOP_PER_PAIR = 20
METRIC = "FMM particles/sec fwd+adjoint at rel-L2<=1e-5; %FP32/MFMA peak vs plain FP32"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


WORKLOADS = {
    1: "uniform Laplace charges in the unit cube, q ~ U[-1,1], p=4, leaf 64, uniform octree",
    2: "clustered Laplace charges (60% uniform + 40% in 20 Gaussian clusters sigma=0.02, N(0,1) charges "
       "mean removed), p=6, leaf 128, adaptive octree",
    3: "rigid clumps of 8 pebbles (cube corners, edge 0.6R, lognormal R, 30% packing), N(0,1) pebble charges, "
       "p=6, leaf 128, adaptive octree, per-clump force and torque",
    4: "uniform Laplace charges in the unit cube, q ~ N(0,1), p=6, leaf 128, adaptive octree",
    5: "Plummer sphere (a=0.1, r<=10a) of unit masses, gravity, p=8, leaf 256, adaptive octree depth<=12",
    6: "periodic unit cell: 50 co-oriented two-layer hexagonal platelets of 2x547 pebbles charged +1/-1, "
       "Laplace lattice sum (Ewald convention), p=6, leaf 64, adaptive octree",
}
CPU_SAMPLE = {1: 4096, 2: 131072, 3: 131072, 4: 131072, 5: 65536, 6: 8752}


def run_path(Plan, w, pos, q, gu, gE, precision, steps, warmup, move=0.0, m2l_rtol=0.0):
    """Time `steps` steps (re-tree + forward + adjoint) after `warmup` ones.
    The library records HIP events around every phase of every call on the
    streams the kernels run on; they are read after the timed region, so the
    timed steps never wait on the host."""
    import torch
    plan = Plan(pos, w.kernel, w.p, w.leaf_size, w.adaptive, w.max_depth, precision=precision, root=w.root,
                profile=True, periodic=w.periodic, m2l_rtol=m2l_rtol)
    lo, hi = None, None
    if move > 0:
        # particles drift between long-range calls (the DEM loop): each step
        # moves every position by N(0, move^2) per axis, kept inside the root
        pos = pos.clone()
        rlo = torch.tensor(w.root[0], dtype=torch.float64, device="cuda")
        lo, hi = rlo, rlo + w.root[1] * (1 - 2.0 ** -20)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(2512)
    counts = plan.counts()
    counts["m2l_rank"], counts["m2l_tile"] = plan.m2l_rank()
    clumps = None
    if w.clump_offsets is not None:
        # the clump workload: registered clumps, per-clump force and torque as
        # the forward pass, the gradient of a linear loss on them as the adjoint
        C = len(w.clump_offsets) - 1
        plan.set_clumps(torch.tensor(w.clump_offsets, device="cuda"))
        rng = np.random.default_rng(78)
        cen = torch.tensor(w.clump_centers, device="cuda")
        gF = torch.tensor(rng.standard_normal((C, 3)), device="cuda")
        gT = torch.tensor(rng.standard_normal((C, 3)), device="cuda")
        clumps = (cen, gF, gT)

    def drift():
        if move > 0:
            pos.add_(torch.randn(pos.shape, generator=gen, dtype=pos.dtype, device=pos.device), alpha=move)
            if w.periodic:
                # a particle leaving the cell re-enters through the opposite face
                pos.sub_(lo).remainder_(w.root[1]).add_(lo)
            torch.maximum(pos, lo, out=pos)
            torch.minimum(pos, hi, out=pos)

    def step():
        drift()
        plan.rebuild(pos)
        if clumps is not None:
            cen, gF, gT = clumps
            F, T = plan.clump_forces(q, cen)
            gq, gx, gX = plan.clump_forces_backward(q, cen, gF, gT)
            return F, T, gq, gx
        u, E = plan.evaluate(q)
        gq, gx = plan.backward(None, gu, gE)   # adjoint of the evaluation just made
        return u, E, gq, gx

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    # the phases of the timed calls (two per step: forward, then adjoint)
    ncalls = min(2 * steps, 64)
    calls = [plan.phase_times(back) for back in range(ncalls - 1, -1, -1)]
    phases, phases_adj = calls[0::2], calls[1::2]
    # split of a step (untimed repetitions, mean of five; moving particles
    # drift before each, outside the timed part)
    split = np.zeros(3)
    for _ in range(5):
        drift()
        torch.cuda.synchronize()
        a = time.perf_counter()
        plan.rebuild(pos)
        torch.cuda.synchronize()
        b = time.perf_counter()
        if clumps is not None:
            plan.clump_forces(q, clumps[0])
        else:
            plan.evaluate(q)
        torch.cuda.synchronize()
        c = time.perf_counter()
        if clumps is not None:
            plan.clump_forces_backward(q, clumps[0], clumps[1], clumps[2])
        else:
            plan.backward(None, gu, gE)
        torch.cuda.synchronize()
        d = time.perf_counter()
        split += (b - a, c - b, d - c)
    split /= 5
    ph = {k: float(np.mean([p[k] for p in phases])) for k in phases[0]}
    pha = {k: float(np.mean([p[k] for p in phases_adj])) for k in phases_adj[0]}
    res = dict(ms_per_step=1e3 * t, t_tree_ms=1e3 * split[0], t_fwd_ms=1e3 * split[1], t_adj_ms=1e3 * split[2],
               phases_fwd_ms=ph, phases_adj_ms=pha, counts=counts, outputs=[o.detach() for o in out],
               timed_launches=len(calls), builds=plan.build_stats())
    plan.close()
    return res


def source_digest(kernel):
    import hashlib
    with open(os.path.join(CSRC, KERNEL_SOURCE[kernel]), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def stored_traffic(kernel, precision, workload, n):
    """HBM bytes per launch from the committed counter summary, or None when
    there is none for this kernel, path and workload, or the kernel's source
    file changed since it was taken."""
    try:
        with open(TRAFFIC_FILES.get(precision, TRAFFIC_FILE)) as f:
            for line in f:
                if line.startswith("traffic_json: "):
                    rec = json.loads(line[len("traffic_json: "):])
                    if (rec["kernel"] == kernel and rec["precision"] == precision
                            and rec.get("workload") == workload and rec.get("n") == n
                            and rec["source_sha256_16"] == source_digest(kernel)):
                        return rec["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


def roofline(res, n, precision, workload, npts):
    """Roofline of the kernel with the most time per step: the M2L (one launch
    in the forward pass and one in the adjoint) or the forward P2P.  The
    per-launch time is the mean of that kernel's launches in a step, each
    measured by the library's HIP events on the stream it runs on."""
    ph, pa = res["phases_fwd_ms"], res["phases_adj_ms"]
    c = res["counts"]
    m2l_total = ph["m2l"] + pa["m2l"]
    if m2l_total >= ph["p2p"]:
        # the M2L as computed: 2 k^2 per V pair, k the rank of the operators
        # in use (the surface size n for the exact operators); the adjoint
        # launch does the same work for the adjoint sources
        k = c.get("m2l_rank", n)
        flops = 2.0 * k * k * c["v_pairs"]
        per = 0.5 * m2l_total
        peak = PEAK["bf16"] if precision == "split_bf16" else PEAK["fp32"]
        ach = flops / (per * 1e-3) / 1e12
        return dict(kernel="k_m2l", bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak,
                    traffic=stored_traffic("k_m2l", precision, workload, npts), per_launch_ms=per,
                    work=f"2 k^2 x {c['v_pairs']} V pairs, k = {k} (surface size {n})")
    return near_roofline(res, precision, workload, npts)


def near_roofline(res, precision, workload, npts):
    """Roofline of the forward near field (`k_p2p`, one launch per forward
    pass): 20 FLOP per pair against the FP32 vector peak, timed by the
    library's HIP events on the near-field stream."""
    ph, c = res["phases_fwd_ms"], res["counts"]
    flops = P2P_FLOP_PER_PAIR * c["p2p_pairs"]
    ach = flops / (ph["p2p"] * 1e-3) / 1e12
    return dict(kernel="k_p2p", bound="alu", achieved=ach, peak=PEAK["fp32"], unit="TFLOP/s",
                frac=ach / PEAK["fp32"], traffic=stored_traffic("k_p2p", precision, workload, npts),
                per_launch_ms=ph["p2p"],
                work=f"20 x {c['p2p_pairs']} pairs")


def cpu_baseline(k, m2l_rtol):
    """FP64 oracle forward + adjoint on a bounded sample of the same workload
    (with the same M2L basis cut-off as the timed GPU path)."""
    import workloads
    from oracle import kifmm
    w = workloads.make(k, n=CPU_SAMPLE[k])
    n = w.n
    rng = np.random.default_rng(5)
    ub = rng.standard_normal(n)
    Eb = rng.standard_normal((n, 3))
    t0 = time.perf_counter()
    P = kifmm.plan(w.positions, w.kernel, w.p, w.leaf_size, w.adaptive, w.max_depth, w.root,
                   periodic=w.periodic, m2l_rtol=m2l_rtol)
    kifmm.forward(P, w.charges)
    kifmm.vjp(P, w.charges, ub, Eb)
    t = time.perf_counter() - t0
    threads = os.environ.get("OMP_NUM_THREADS")
    cores = int(threads) if threads else (os.cpu_count() or 1)
    return dict(value=n / t, unit="particles/s", cores=cores, kind="oracle",
                sample=f"the same workload generator at N={n} (same p, leaf, tree rules): "
                       f"tree+lists+forward+adjoint in FP64, {t:.1f} s")


def oracle_check(w, paths, gu, gE, m2l_rtol, nsample=256):
    """The oracle as the checker of the timed outputs: the same plan (tree,
    lists, operators) in FP64, evaluated at `nsample` sampled targets, forward
    and adjoint; with the truncated M2L basis also the forward with the exact
    operators.  Per path and output: rel-L2 and the worst element
    (max |y - y_ref| / max |y_ref|) over the sample."""
    import dataclasses

    from oracle import kifmm
    from oracle.operators import Operators
    t0 = time.perf_counter()
    P = kifmm.plan(w.positions, w.kernel, w.p, w.leaf_size, w.adaptive, w.max_depth, w.root,
                   periodic=w.periodic, m2l_rtol=m2l_rtol)
    idx = np.sort(np.random.default_rng(21).choice(w.n, nsample, replace=False))
    ub = gu.double().cpu().numpy()
    Eb = gE.double().cpu().numpy()
    ref = {}
    ref["u"], ref["E"] = kifmm.forward(P, w.charges, targets=idx)
    ref["qbar"], ref["xbar"] = kifmm.vjp(P, w.charges, ub, Eb, targets=idx)
    if m2l_rtol > 0:
        PX = dataclasses.replace(P, ops=Operators(P.p, P.c, P.tree.s, P.tau, 0.0))
        ref["u_exact_m2l"], ref["E_exact_m2l"] = kifmm.forward(PX, w.charges, targets=idx)
    t = time.perf_counter() - t0

    def err(a, b):
        return {"rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                "worst": float(np.max(np.abs(a - b)) / np.max(np.abs(b)))}

    out = {"sample": f"{nsample} sampled targets of the timed plan; oracle {t:.1f} s",
           "tolerance": {"fp32": 1e-5, "split_bf16": 1e-4}}
    for prec, r in paths.items():
        got = dict(zip(("u", "E", "qbar", "xbar"), (o.double().cpu().numpy()[idx] for o in r["outputs"])))
        res = {k: err(got[k], ref[k]) for k in ("u", "E", "qbar", "xbar")}
        if m2l_rtol > 0:
            res["u_vs_exact_m2l"] = err(got["u"], ref["u_exact_m2l"])
            res["E_vs_exact_m2l"] = err(got["E"], ref["E_exact_m2l"])
        out[prec] = res
    return out


# the largest single-GPU workload, measured beside the headline
LARGEST = 5


def run_largest(Plan, steps, warmup, m2l_rtol):
    """The Plummer workload (8,388,608 unit masses, p = 8) on the headline path:
    ms per step (re-tree + forward + adjoint) and its dominant kernel."""
    import torch
    import workloads
    w = workloads.make(LARGEST)
    pos = torch.tensor(w.positions, dtype=torch.float64, device="cuda")
    q = torch.tensor(w.charges, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(77)
    gu = torch.tensor(workloads.round_f32(rng.standard_normal(w.n)), dtype=torch.float32, device="cuda")
    gE = torch.tensor(workloads.round_f32(rng.standard_normal((w.n, 3))), dtype=torch.float32, device="cuda")
    r = run_path(Plan, w, pos, q, gu, gE, "split_bf16", steps, warmup, 0.0, m2l_rtol)
    r.pop("outputs", None)
    return {"workload": WORKLOADS[LARGEST], "name": w.name, "n": w.n, "path": "split_bf16", "steps": steps,
            "warmup": warmup, "ms_per_step": r["ms_per_step"], "particles_per_s": w.n / (r["ms_per_step"] * 1e-3),
            "t_tree_ms": r["t_tree_ms"], "t_fwd_ms": r["t_fwd_ms"], "t_adj_ms": r["t_adj_ms"],
            "phases_fwd_ms": r["phases_fwd_ms"], "phases_adj_ms": r["phases_adj_ms"], "counts": r["counts"],
            "roofline": roofline(r, r["counts"]["surface_points"], "split_bf16", w.name, w.n)}


def run_f4(Plan, steps, warmup, m2l_rtol, paths=("split_bf16", "fp32"), check=True, nsample=256):
    """The sums beyond charges on the clustered workload (1,048,576 points,
    p = 6): point dipoles with charges (u, E), the same with dE/dx, and the
    Stokeslet velocity of point forces, alone and with the pressure.  Per
    path: ms per call on a fixed plan (no re-tree), then with `check` the
    oracle on the same plan at `nsample` sampled targets, and the Stokes
    velocity and pressure also against their direct sums there."""
    import torch
    import workloads
    w = workloads.make(2)
    n = w.n
    pos = torch.tensor(w.positions, dtype=torch.float64, device="cuda")
    q = torch.tensor(w.charges, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(81)
    # dipole moments of the size of a charge times a tenth of the mean spacing,
    # so charges and dipoles both carry weight in the sums
    m = workloads.round_f32(rng.standard_normal((n, 3)) * 0.1 * n ** (-1.0 / 3.0))
    f = workloads.round_f32(rng.standard_normal((n, 3)))
    mu = 0.7
    md = torch.tensor(m, dtype=torch.float32, device="cuda")
    fd = torch.tensor(f, dtype=torch.float32, device="cuda")
    calls = {"dipoles": lambda P: P.evaluate_dipoles(q, md),
             "gradient": lambda P: P.evaluate_gradient(q, md),
             "stokes": lambda P: (P.evaluate_stokes(fd, mu),),
             "stokes_pressure": lambda P: P.evaluate_stokes(fd, mu, pressure=True)}
    res, outs = {}, {}
    for prec in paths:
        plan = Plan(pos, w.kernel, w.p, w.leaf_size, w.adaptive, w.max_depth, precision=prec, root=w.root,
                    m2l_rtol=m2l_rtol)
        r = {}
        for name, fn in calls.items():
            for _ in range(warmup):
                fn(plan)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                o = fn(plan)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / steps
            r[name] = {"ms_per_call": t * 1e3, "points_per_s": n / t}
            if check:
                outs[(prec, name)] = [x.double().cpu().numpy() for x in o]
            log(f"[bench] f4 {prec} {name}: {t * 1e3:.3f} ms/call")
        res[prec] = r
        plan.close()
    out = {"workload": WORKLOADS[2] + "; dipoles N(0,1)*0.1*N^(-1/3) per axis, forces N(0,1) per axis, "
                                      f"viscosity {mu}; call = one evaluation on a fixed plan",
           "n": n, "steps": steps, "warmup": warmup, "m2l_rtol": m2l_rtol, "timing": res,
           "outputs": {"dipoles": "u, E", "gradient": "u, E, dE/dx", "stokes": "velocity",
                       "stokes_pressure": "velocity, pressure"}}
    if not check:
        return out
    from oracle import kifmm, stokes
    t0 = time.perf_counter()
    P = kifmm.plan(w.positions, w.kernel, w.p, w.leaf_size, w.adaptive, w.max_depth, w.root,
                   periodic=w.periodic, m2l_rtol=m2l_rtol)
    idx = np.sort(np.random.default_rng(21).choice(n, nsample, replace=False))
    uo, Eo, Go = kifmm.forward_dipoles(P, w.charges, m, targets=idx, grad=True)
    vo, vmag, po = stokes.kifmm(P, f, mu, targets=idx, terms=True, frame="leaf", pressure=True)
    t_oracle = time.perf_counter() - t0
    # how much the four-potential combination, about each target's leaf
    # centre as the library forms it, amplifies relative errors of its far
    # fields: the far terms' magnitudes over the velocity
    kappa = float(np.linalg.norm(vmag) / np.linalg.norm(vo))
    vd = stokes.direct(w.positions, f, mu, targets=idx, chunk=4)
    pd = stokes.pressure_direct(w.positions, f, targets=idx, chunk=4)

    def err(a, b):
        return {"rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                "worst": float(np.max(np.abs(a - b)) / np.max(np.abs(b)))}

    acc = {"sample": f"{nsample} sampled targets of the timed plan; oracle {t_oracle:.1f} s",
           "tolerance": {"fp32": 1e-5, "split_bf16": 1e-4}}
    for prec in paths:
        d = outs[(prec, "dipoles")]
        g = outs[(prec, "gradient")]
        s = outs[(prec, "stokes")][0]
        sp = outs[(prec, "stokes_pressure")]
        acc[prec] = {"dipoles": {"u": err(d[0][idx], uo), "E": err(d[1][idx], Eo)},
                     "gradient": {"u": err(g[0][idx], uo), "E": err(g[1][idx], Eo), "dE/dx": err(g[2][idx], Go)},
                     "stokes": {"velocity": err(s[idx], vo), "velocity_vs_direct_sum": err(s[idx], vd)},
                     "stokes_pressure": {"velocity": err(sp[0][idx], vo), "pressure": err(sp[1][idx], po),
                                         "pressure_vs_direct_sum": err(sp[1][idx], pd)}}
    acc["oracle_stokes_vs_direct_sum"] = err(vo, vd)
    acc["oracle_pressure_vs_direct_sum"] = err(po, pd)
    acc["stokes_amplification"] = kappa
    acc["stokes_tolerance"] = {"fp32": 2e-5, "split_bf16": 1e-4,
                               "reading": "the far fields carry about stokes_amplification of the velocity and "
                                          "are accurate to about 1e-5 of their own size in FP32 (the charge "
                                          "sums' field, 7 % far, meets 6e-7 overall)"}
    out["accuracy_vs_oracle"] = acc
    return out


# the workload --counter-run evaluates (its name and size, as recorded with the counters)
COUNTER_WORKLOAD = ("clustered_1M_p6", 1_048_576)
# M2L basis cut-off of the timed configuration (singular values below 1e-6
# sigma_1 of the stacked offset operators dropped; the full-size parity tests
# use the same)
M2L_RTOL = 1e-6


def counter_run(precision):
    """Short run for counter collection: set-up, two forward evaluations, then
    a plain copy of CALIB_BYTES (one elementwise kernel reading and writing
    CALIB_BYTES) that calibrates the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    import workloads
    from paper_2512_09478_amd import Plan
    w = workloads.make(2)
    pos = torch.tensor(w.positions, dtype=torch.float64, device="cuda")
    q = torch.tensor(w.charges, dtype=torch.float32, device="cuda")
    plan = Plan(pos, w.kernel, w.p, w.leaf_size, w.adaptive, w.max_depth, precision=precision, root=w.root,
                m2l_rtol=M2L_RTOL)
    for _ in range(2):
        plan.evaluate(q)
    torch.cuda.synchronize()
    a = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.neg(a, out=b)
    torch.cuda.synchronize()
    log(f"[bench] counter run done: {plan.counts()}")
    counts = plan.counts()
    counts["m2l_rank"], counts["m2l_tile"] = plan.m2l_rank()
    print(json.dumps({"counts": counts, "precision": precision}), flush=True)
    plan.close()


def short_name(name):
    import re
    name = re.sub(r"kifmm::\(anonymous namespace\)::", "", name)
    return name.split("(")[0]


TRACE_TITLE = ("clustered 1,048,576 charges, p = 6, leaf 128, M2L in the truncated basis (rank 116, cut-off 1e-6) "
               "(bench step: re-tree + forward + adjoint, split-bf16 and FP32 paths)")


def summarize_trace(db, out, cmd, title=TRACE_TITLE):
    """Per-kernel (and per grid size) duration table from a rocprofv3 database."""
    import sqlite3
    c = sqlite3.connect(db)
    rows = c.execute("select name, grid_x, count(*), sum(duration)/1e6, avg(duration)/1e3, min(duration)/1e3, "
                     "max(duration)/1e3, vgpr_count, accum_vgpr_count, lds_size from kernels "
                     "group by name, grid_x order by sum(duration) desc limit 40").fetchall()
    tot = c.execute("select sum(duration)/1e6 from kernels").fetchone()[0]
    with open(out, "w") as f:
        f.write(f"# Kernel trace: {title}\n\n")
        f.write(f"Command (repository root on an MI355X):\n\n```\n{cmd}\n```\n\n")
        f.write(f"Total kernel time {tot:.1f} ms. Rows are per kernel and grid size (the forward and adjoint "
                "M2L differ in grid).\n\n")
        f.write("| kernel | grid | calls | total ms | avg us | min us | max us | VGPR | AGPR | LDS B |\n")
        f.write("|---|---|---|---|---|---|---|---|---|---|\n")
        for r in rows:
            f.write(f"| `{short_name(r[0])}` | {r[1]} | {r[2]} | {r[3]:.3f} | {r[4]:.1f} | {r[5]:.1f} | "
                    f"{r[6]:.1f} | {r[7]} | {r[8]} | {r[9]} |\n")


def summarize_counters(csv_a, counts_json, out, cmd_a):
    """Matrix-core utilisation and instruction counts of the dominant kernels
    from one counter pass over --counter-run (the counts line that run prints
    gives the P2P pair and M2L V-pair numbers)."""
    import csv
    from collections import defaultdict
    counts = None
    for line in open(counts_json):
        line = line.strip()
        if line.startswith("{") and '"counts"' in line:
            counts = json.loads(line)
    if counts is None:
        raise SystemExit("no counts line in " + counts_json)
    c = counts["counts"]
    acc = defaultdict(lambda: defaultdict(list))
    dur = defaultdict(list)
    seen = set()
    for r in csv.DictReader(open(csv_a)):
        k = (short_name(r["Kernel_Name"]), int(r["Grid_Size"]))
        acc[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
        if r["Dispatch_Id"] not in seen:
            seen.add(r["Dispatch_Id"])
            dur[k].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
    mean = {k: {n: float(np.mean(v)) for n, v in d.items()} for k, d in acc.items()}
    simds = 256 * 4
    xcds = 8   # GRBM_GUI_ACTIVE of a dispatch is summed over the eight XCDs
    rows = []
    for k in sorted(mean, key=lambda k: -float(np.mean(dur[k]))):
        m = mean[k]
        t = float(np.mean(dur[k]))
        if "GRBM_GUI_ACTIVE" not in m or t < 20e-6:
            continue
        gui = m["GRBM_GUI_ACTIVE"]
        mfma = m.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) * xcds / (gui * simds) if gui else 0.0
        rows.append((k, t, mfma, m.get("SQ_INSTS_VALU", 0.0), m.get("SQ_INSTS_MFMA", 0.0)))
    n = c["surface_points"]
    nl = "\n"
    with open(out, "w") as f:
        f.write("# Matrix-core utilisation and instruction counts: clustered 1,048,576 charges, p = 6, "
                f"leaf 128, {counts['precision']} path, forward evaluation" + nl + nl)
        f.write("One counter pass over the program (repository root on an MI355X):" + nl + nl)
        f.write("```" + nl + cmd_a + nl + "```" + nl + nl)
        f.write("MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x GRBM_GUI_ACTIVE / 8), per dispatch "
                "and averaged over the dispatches of a kernel and grid: the busy cycles are summed over the "
                "SIMDs, and GRBM_GUI_ACTIVE is summed over the eight XCDs (it reads about 8 x the kernel's "
                "duration in cycles).  The instruction columns are wave-level instruction counts per "
                "dispatch.  Durations are those of the counter run." + nl + nl)
        f.write("| kernel | grid | avg us | MFMA busy | VALU instructions | MFMA instructions |" + nl)
        f.write("|---|---|---|---|---|---|" + nl)
        for (k, t, mf, iv, im) in rows[:16]:
            f.write(f"| `{k[0]}` | {k[1]} | {t * 1e6:.1f} | {mf:.3f} | {iv:.4g} | {im:.4g} |" + nl)
        m2l = [r for r in rows if r[0][0].startswith("void k_m2l")]
        p2p = [r for r in rows if r[0][0].split("<")[0].split()[-1] == "k_p2p"]
        f.write(nl + "Achieved rates in this run (algorithmic work over the dispatch's own duration):" + nl + nl)
        if m2l:
            t = m2l[0][1]
            kr, tile = c.get("m2l_rank", n), c.get("m2l_tile", ((n + 31) // 32) * 32)
            fl = 2.0 * kr * kr * c["v_pairs"]
            ex = m2l[0][4] * 2 * 16 * 16 * 32   # every M2L MFMA of the split path is a 16x16x32 bf16 product
            f.write(f"* `k_m2l`: {c['v_pairs']:,} V pairs x 2 x {kr}^2 = {fl / 1e9:.1f} GFLOP in {t * 1e3:.3f} ms "
                    f"= {fl / t / 1e12:.1f} TFLOP/s useful ({fl / t / 2.5e15 * 100:.1f} % of the bf16 dense "
                    f"peak); executed {m2l[0][4]:.4g} bf16 16x16x32 MFMAs = {ex / 1e12:.2f} TFLOP, "
                    f"{ex / t / 1e15:.2f} PFLOP/s ({ex / t / 2.5e15 * 100:.1f} % of 2.5 PFLOP/s: three products "
                    f"per split product, padding to {tile} rows, slots walked for a block's "
                    f"union of targets); MFMA busy {m2l[0][2] * 100:.1f} %.  (Rank {kr} of the operators in use: the "
                    f"truncated common basis of the {n}-point surface when it is smaller than {n}.)" + nl)
        if p2p:
            t = p2p[0][1]
            fl = 20.0 * c["p2p_pairs"]
            f.write(f"* `k_p2p`: {c['p2p_pairs']:,} pairs x 20 FLOP = {fl / 1e9:.1f} GFLOP in {t * 1e3:.3f} ms = "
                    f"{fl / t / 1e12:.1f} TFLOP/s FP32 ({fl / t / 157.3e12 * 100:.1f} % of 157.3 TFLOP/s); "
                    f"{p2p[0][3] * 64 / max(1, c['p2p_pairs']):.1f} VALU instructions per pair (each lane "
                    "takes one pair per pass of the inner loop)." + nl)


def summarize_traffic(fetch_csv, write_csv, out, cmd_fetch, cmd_write, precision):
    """FETCH_SIZE / WRITE_SIZE per dispatch, calibrated by the plain copy."""
    import csv
    from collections import defaultdict

    def per_kernel(path, counter):
        acc = defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                acc[(short_name(r["Kernel_Name"]), int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
        return {k: float(np.mean(v)) for k, v in acc.items()}

    fe = per_kernel(fetch_csv, "FETCH_SIZE")
    wr = per_kernel(write_csv, "WRITE_SIZE")
    copy = [k for k in fe if "neg" in k[0].lower()]
    if not copy:
        raise SystemExit("calibration copy kernel not found in the counter file")
    kib = CALIB_BYTES / 1024.0
    f_fac = kib / fe[copy[0]]
    w_fac = kib / wr[copy[0]]
    lines = []
    recs = []
    for k in sorted(fe, key=lambda k: -fe[k]):
        if k not in wr:
            continue
        fb = fe[k] * f_fac * 1024
        wb = wr[k] * w_fac * 1024
        lines.append(f"| `{k[0]}` | {k[1]} | {fe[k]:.0f} | {wr[k]:.0f} | {fb / 1e6:.1f} | {wb / 1e6:.1f} |")
        base = k[0].split("<")[0].split()[-1]
        for kern in KERNEL_SOURCE:
            if base == kern and not any(r["kernel"] == kern for r in recs):
                # the first (largest-fetch) entry of a kernel is its forward launch
                recs.append(dict(kernel=kern, precision=precision, workload=COUNTER_WORKLOAD[0],
                                 n=COUNTER_WORKLOAD[1], grid=k[1], bytes_per_launch=fb + wb,
                                 fetch_bytes=fb, write_bytes=wb, source_sha256_16=source_digest(kern)))
    with open(out, "w") as f:
        f.write("# HBM traffic per dispatch: clustered 1,048,576 charges, p = 6, leaf 128, "
                f"{precision} path, forward evaluation\n\n")
        f.write("Two counter passes over the same program (repository root on an MI355X):\n\n")
        f.write(f"```\n{cmd_fetch}\n{cmd_write}\n```\n\n")
        f.write(f"Calibration: a plain copy kernel (`{copy[0][0]}`) reads and writes {CALIB_BYTES >> 20} MiB; "
                f"its counters read FETCH_SIZE {fe[copy[0]]:.0f} KiB and WRITE_SIZE {wr[copy[0]]:.0f} KiB, "
                f"so the factors are {f_fac:.4f} (fetch) and {w_fac:.4f} (write).\n\n")
        f.write("| kernel | grid | FETCH_SIZE KiB | WRITE_SIZE KiB | fetch MB (calibrated) | write MB (calibrated) |\n")
        f.write("|---|---|---|---|---|---|\n")
        f.write("\n".join(lines[:30]) + "\n\n")
        f.write("The benchmark reads the lines below; it reports null once the kernel's source file has changed "
                "(the digest no longer matches).\n\n")
        for r in recs:
            f.write("traffic_json: " + json.dumps(r) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None, help="override the number of charges")
    ap.add_argument("--workload", type=int, default=2, choices=sorted(WORKLOADS),
                    help="workload generator (2 = the clustered 1M headline)")
    ap.add_argument("--move", type=float, default=0.0,
                    help="per-step random displacement (std per axis) of every particle before the re-tree")
    ap.add_argument("--paths", default="split_bf16,fp32")
    ap.add_argument("--m2l-rtol", type=float, default=M2L_RTOL,
                    help="M2L in the truncated common basis of the offset operators (0: exact operators)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle legs (CPU baseline and accuracy check)")
    ap.add_argument("--no-largest", action="store_true", help="skip the largest workload beside the headline")
    ap.add_argument("--f4", action="store_true",
                    help="time the dipole, field-gradient and Stokeslet sums on the clustered 1M workload "
                         "and check them against the oracle at sampled targets (prints its own JSON line)")
    ap.add_argument("--counter-run", metavar="PRECISION", help="short run for rocprofv3 counter passes")
    ap.add_argument("--summarize-trace", nargs="+", metavar="DB OUT CMD [TITLE]")
    ap.add_argument("--summarize-counters", nargs=4, metavar=("CSV", "COUNTS_LOG", "OUT", "CMD"))
    ap.add_argument("--summarize-traffic", nargs=6,
                    metavar=("FETCH_CSV", "WRITE_CSV", "OUT", "CMD_FETCH", "CMD_WRITE", "PRECISION"))
    args = ap.parse_args()
    if args.summarize_trace:
        if len(args.summarize_trace) not in (3, 4):
            raise SystemExit("--summarize-trace takes DB OUT CMD [TITLE]")
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic)
        return
    if args.counter_run:
        counter_run(args.counter_run)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on a single GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import workloads
    from paper_2512_09478_amd import Plan
    if args.f4:
        print(json.dumps({"f4": run_f4(Plan, args.steps, args.warmup, args.m2l_rtol, check=not args.no_cpu)}),
              flush=True)
        return
    w = workloads.make(args.workload, n=args.n)
    n = w.n
    pos = torch.tensor(w.positions, dtype=torch.float64, device="cuda")
    q = torch.tensor(w.charges, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(77)
    gu = torch.tensor(workloads.round_f32(rng.standard_normal(n)), dtype=torch.float32, device="cuda")
    gE = torch.tensor(workloads.round_f32(rng.standard_normal((n, 3))), dtype=torch.float32, device="cuda")
    paths = {}
    for prec in args.paths.split(","):
        log(f"[bench] {prec}: N={n} steps={args.steps} warmup={args.warmup}")
        paths[prec] = run_path(Plan, w, pos, q, gu, gE, prec, args.steps, args.warmup, args.move, args.m2l_rtol)
        r = paths[prec]
        log(f"[bench] {prec}: {r['ms_per_step']:.3f} ms/step  tree {r['t_tree_ms']:.2f} fwd {r['t_fwd_ms']:.2f} "
            f"adj {r['t_adj_ms']:.2f}  phases {json.dumps({k: round(v, 3) for k, v in r['phases_fwd_ms'].items()})}"
            f"  adjoint {json.dumps({k: round(v, 3) for k, v in r['phases_adj_ms'].items()})}")
    head = "split_bf16" if "split_bf16" in paths else next(iter(paths))
    H = paths[head]
    ops_n = H["counts"]["surface_points"]
    # stored counter traffic applies to the static workload it was taken on only
    wkey = w.name + ("+move" if args.move else "")
    agree = {}
    if "fp32" in paths and "split_bf16" in paths:
        names = ("F_c", "T_c") if w.clump_offsets is not None else ("u", "E")
        for name, i in ((names[0], 0), (names[1], 1), ("qbar", 2), ("xbar", 3)):
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
        "config": {"workload": WORKLOADS[args.workload] + "; step = re-tree + forward + adjoint"
                               + (f"; particles move by N(0, {args.move}^2) per axis each step" if args.move else ""),
                   "name": w.name, "n": n, "p": w.p, "leaf_size": w.leaf_size, "path": head,
                   "m2l_rtol": args.m2l_rtol},
        "roofline": roofline(H, ops_n, head, wkey, n),
        # the forward near field beside it (the other kernel of the step)
        "roofline_near": near_roofline(H, head, wkey, n),
        "paths": {k: {"particles_per_s": n / (v["ms_per_step"] * 1e-3), "ms_per_step": v["ms_per_step"],
                      "particles_per_s_without_tree": n / ((v["t_fwd_ms"] + v["t_adj_ms"]) * 1e-3),
                      "particles_per_s_forward": n / (v["t_fwd_ms"] * 1e-3),
                      "particles_per_s_adjoint": n / (v["t_adj_ms"] * 1e-3),
                      "t_tree_ms": v["t_tree_ms"], "t_fwd_ms": v["t_fwd_ms"], "t_adj_ms": v["t_adj_ms"],
                      "phases_fwd_ms": v["phases_fwd_ms"], "phases_adj_ms": v["phases_adj_ms"],
                      "tree_builds": v["builds"],
                      "roofline": roofline(v, ops_n, k, wkey, n),
                      "roofline_near": near_roofline(v, k, wkey, n)}
                  for k, v in paths.items()},
        "counts": H["counts"],
        "timed_launches_per_path": H["timed_launches"],
        "split_vs_fp32_rel_l2": agree,
    }
    if args.workload == 2 and args.n is None and not args.move and not args.no_largest:
        log("[bench] largest workload (Plummer, 8,388,608 points, p = 8), split-bf16 path")
        out["largest_config"] = run_largest(Plan, 5, 2, args.m2l_rtol)
        log(f"[bench] largest: {out['largest_config']['ms_per_step']:.2f} ms/step")
        # the other sums of eq. (1) on the same workload, timed only (their
        # oracle check is `--f4` and the full-size GPU test)
        log("[bench] dipole, field-gradient and Stokeslet sums (timing)")
        out["f4"] = run_f4(Plan, 5, 2, args.m2l_rtol, check=False)
    if not args.no_cpu:
        if w.clump_offsets is None and not args.move:
            log("[bench] oracle check of the timed outputs (256 sampled targets)")
            out["accuracy_vs_oracle"] = oracle_check(w, paths, gu, gE, args.m2l_rtol)
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.m2l_rtol)
    for v in paths.values():
        v.pop("outputs", None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
