"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times, on sampled outputs the oracle computes one by one.

The oracle builds the same tree and lists (compared bit for bit where that is
affordable), runs the full upward pass and the downward pass only for the
ancestors of the sampled targets, and evaluates the sampled targets.  Each
phase prints a line so that a long oracle phase is visibly alive.
"""
import sys
import time

import numpy as np
import pytest

import workloads
from oracle import clump as oclump
from oracle import kifmm
from _parity import check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NSAMPLE = 256
# the benchmark's configuration: M2L in the truncated common basis (cut-off 1e-6)
M2L_RTOL = 1e-6


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def say(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)
    sys.stdout.flush()


def gpu_plan(w, precision):
    from paper_2512_09478_amd import Plan
    pos = torch.tensor(w.positions, dtype=torch.float64, device="cuda")
    return Plan(pos, w.kernel, w.p, w.leaf_size, w.adaptive, w.max_depth, precision=precision, root=w.root,
                periodic=w.periodic, m2l_rtol=M2L_RTOL)


def oracle_plan(w):
    t = time.time()
    P = kifmm.plan(w.positions, w.kernel, w.p, w.leaf_size, w.adaptive, w.max_depth, w.root,
                   periodic=w.periodic, m2l_rtol=M2L_RTOL)
    say(f"  oracle tree + lists: {P.tree.nboxes} boxes, {time.time() - t:.1f} s")
    return P


def sample(n, seed):
    return np.sort(np.random.default_rng(seed).choice(n, NSAMPLE, replace=False))


def check_tree(G, P):
    t = G.tree()
    ot = P.tree
    np.testing.assert_array_equal(t["perm"], ot.perm)
    np.testing.assert_array_equal(t["keys"], ot.keys)
    for name in ("level", "begin", "end", "parent", "is_leaf"):
        np.testing.assert_array_equal(t[name], getattr(ot, name), err_msg=name)
    np.testing.assert_array_equal(t["anchor"], ot.anchor)
    for which in "UVWX":
        off, idx = G.list_csr(which)
        ooff, oidx = P.lists.csr(which)
        np.testing.assert_array_equal(off, ooff, err_msg=which)
        np.testing.assert_array_equal(idx, oidx, err_msg=which)


def test_clustered_1M_headline_step_forward_and_adjoint():
    """The benchmark's step at full size: evaluate, then backward(None, ...)
    reusing that forward pass, with the benchmark's adjoint sources; M2L in the
    truncated basis on both paths.  Sampled outputs against the oracle with the
    same operators, and the forward also against the oracle with the exact
    operators (the compression's own error at this size)."""
    import dataclasses

    from oracle.operators import Operators
    say("clustered 1,048,576 charges, p=6, leaf 128: tree + sampled forward and adjoint")
    w = workloads.make(2)
    P = oracle_plan(w)
    idx = sample(w.n, 21)
    rng = np.random.default_rng(77)          # the benchmark's adjoint sources
    ub = workloads.round_f32(rng.standard_normal(w.n))
    Eb = workloads.round_f32(rng.standard_normal((w.n, 3)))
    t = time.time()
    uo, Eo = kifmm.forward(P, w.charges, targets=idx)
    say(f"  oracle sampled forward {time.time() - t:.1f} s")
    t = time.time()
    qo, xo = kifmm.vjp(P, w.charges, ub, Eb, targets=idx)
    say(f"  oracle sampled adjoint {time.time() - t:.1f} s")
    t = time.time()
    PX = dataclasses.replace(P, ops=Operators(P.p, P.c, P.tree.s, P.tau, 0.0))
    uX, EX = kifmm.forward(PX, w.charges, targets=idx)
    say(f"  oracle sampled forward with the exact operators {time.time() - t:.1f} s "
        f"(compression moves u by {rel(uo, uX):.2e}, E by {rel(Eo, EX):.2e})")
    q = torch.tensor(w.charges, dtype=torch.float32, device="cuda")
    gu = torch.tensor(ub, dtype=torch.float32, device="cuda")
    gE = torch.tensor(Eb, dtype=torch.float32, device="cuda")
    for precision, tol in (("fp32", 1e-5), ("split_bf16", 1e-4)):
        G = gpu_plan(w, precision)
        if precision == "fp32":
            check_tree(G, P)
            say("  tree and lists bit-exact")
        u, E = G.evaluate(q)
        gq, gx = G.backward(None, gu, gE)
        torch.cuda.synchronize()
        say(f"  {precision}:")
        check("u", u.cpu().numpy()[idx], uo, tol)
        check("E", E.cpu().numpy()[idx], Eo, tol)
        check("qbar", gq.cpu().numpy()[idx], qo, tol)
        check("xbar", gx.cpu().numpy()[idx], xo, tol)
        say("  against the exact operators:")
        check("u", u.cpu().numpy()[idx], uX, tol)
        check("E", E.cpu().numpy()[idx], EX, tol)
        G.close()


def test_uniform_524k_adjoint_of_force_loss():
    """Loss sum |F - F_target|^2 with F = q E, F_target from charges + 0.1 N(0,1):
    gradients w.r.t. charges and positions at 64 sampled coordinates."""
    say("uniform 524,288 charges, p=6: adjoint of the force-matching loss")
    from paper_2512_09478_amd import kifmm as kop
    w = workloads.make(4)
    qt = workloads.adjoint_target_charges(w.charges, seed=4401)
    P = oracle_plan(w)
    t = time.time()
    _, Eo = kifmm.forward(P, w.charges)
    _, Eto = kifmm.forward(P, qt)
    say(f"  oracle two full forwards {time.time() - t:.1f} s")
    Fo = w.charges[:, None] * Eo
    Fto = qt[:, None] * Eto
    # dL/dE_k = 2 q_k (F_k - Ft_k); dL/dq_k has the direct term 2 (F_k - Ft_k).E_k
    Ebar = 2.0 * w.charges[:, None] * (Fo - Fto)
    coords = np.random.default_rng(64).choice(w.n, 64, replace=False)
    qb, xb = kifmm.vjp(P, w.charges, np.zeros(w.n), Ebar, targets=coords)
    qb = qb + 2.0 * np.sum((Fo - Fto)[coords] * Eo[coords], axis=1)
    say(f"  oracle sampled adjoint done")
    for precision, tol in (("fp32", 1e-5), ("split_bf16", 1e-4)):
        G = gpu_plan(w, precision)
        pos = G.positions.requires_grad_(True)
        q = torch.tensor(w.charges, dtype=torch.float32, device="cuda", requires_grad=True)
        with torch.no_grad():
            _, Et = G.evaluate(torch.tensor(qt, dtype=torch.float32, device="cuda"))
        Ft = torch.tensor(qt, dtype=torch.float32, device="cuda")[:, None] * Et
        u, E = kop(q, pos, G)
        F = q[:, None] * E
        loss = ((F - Ft) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        gq = q.grad.detach().cpu().numpy()[coords]
        gx = pos.grad.detach().cpu().numpy()[coords]
        say(f"  {precision}:")
        check("dL/dq", gq, qb, tol)
        check("dL/dx", gx, xb, tol)
        G.close()


def test_plummer_8M_gravity_forward():
    say("Plummer 8,388,608 unit masses, gravity, p=8, leaf 256, depth <= 12")
    w = workloads.make(5)
    P = oracle_plan(w)
    idx = sample(w.n, 51)
    t = time.time()
    uo, Eo = kifmm.forward(P, w.charges, targets=idx)
    say(f"  oracle sampled forward {time.time() - t:.1f} s")
    q = torch.tensor(w.charges, dtype=torch.float32, device="cuda")
    for precision in ("fp32", "split_bf16"):
        G = gpu_plan(w, precision)
        c = G.counts()
        assert c["depth"] <= 12 and c["boxes"] == P.tree.nboxes
        u, E = G.evaluate(q)
        torch.cuda.synchronize()
        say(f"  {precision}:")
        check("u", u.cpu().numpy()[idx], uo, 1e-4)
        check("E", E.cpu().numpy()[idx], Eo, 1e-4)
        G.close()


def test_clumps_1_6M_force_and_torque():
    """Per-clump force and torque (registered clumps, same-clump pairs left out
    of the near field, where they cancel) on 32 sampled clumps by the plain
    rel-L2 of each output; the pebble field of a plain evaluation beside it."""
    say("200,000 clumps x 8 pebbles, p=6: per-clump force and torque on 32 sampled clumps")
    t = time.time()
    w = workloads.make(3)
    say(f"  packing {time.time() - t:.1f} s")
    P = oracle_plan(w)
    cl = np.sort(np.random.default_rng(33).choice(len(w.clump_offsets) - 1, 32, replace=False))
    peb = np.concatenate([np.arange(w.clump_offsets[c], w.clump_offsets[c + 1]) for c in cl])
    t = time.time()
    _, Eo = kifmm.forward(P, w.charges, targets=peb)
    say(f"  oracle sampled forward {time.time() - t:.1f} s")
    sub_off = np.concatenate([[0], np.cumsum(np.diff(w.clump_offsets)[cl])])
    Fo, To = oclump.clump_reduce(w.positions[peb], w.charges[peb], Eo, sub_off, w.clump_centers[cl])
    q = torch.tensor(w.charges, dtype=torch.float32, device="cuda")
    off = torch.tensor(w.clump_offsets, device="cuda")
    cen = torch.tensor(w.clump_centers, device="cuda")
    for precision, tol in (("fp32", 1e-5), ("split_bf16", 1e-4)):
        G = gpu_plan(w, precision)
        u, E = G.evaluate(q)
        G.set_clumps(off)
        F, T = G.clump_forces(q, cen)
        G.synchronize()
        say(f"  {precision}:")
        check("pebble E", E.cpu().numpy()[peb], Eo, tol)
        check("F_c", F.cpu().numpy()[cl], Fo, tol)
        check("T_c", T.cpu().numpy()[cl], To, tol)
        # the same sums over the plain evaluation's field (every pair kept)
        F2, T2 = G.clump_reduce(q, E, off, cen)
        say(f"    over the plain field: rel-L2 F_c {rel(F2.cpu().numpy()[cl], Fo):.3e}, "
            f"T_c {rel(T2.cpu().numpy()[cl], To):.3e}")
        G.close()


def test_periodic_platelets_forward_and_adjoint():
    say("periodic cell of 50 platelets (54,700 charges), p=6, leaf 64: tree + sampled forward and adjoint")
    w = workloads.make(6)
    P = oracle_plan(w)
    idx = sample(w.n, 61)
    rng = np.random.default_rng(62)
    ub = workloads.round_f32(rng.standard_normal(w.n))
    Eb = workloads.round_f32(rng.standard_normal((w.n, 3)))
    t = time.time()
    uo, Eo = kifmm.forward(P, w.charges, targets=idx)
    qo, xo = kifmm.vjp(P, w.charges, ub, Eb, targets=idx)
    say(f"  oracle sampled forward and adjoint {time.time() - t:.1f} s")
    q = torch.tensor(w.charges, dtype=torch.float32, device="cuda")
    for precision, tol in (("fp32", 1e-5), ("split_bf16", 1e-4)):
        G = gpu_plan(w, precision)
        if precision == "fp32":
            check_tree(G, P)
            say("  tree and lists (with image shifts) bit-exact")
        u, E = G.evaluate(q)
        gq, gx = G.backward(None, torch.tensor(ub, dtype=torch.float32, device="cuda"),
                            torch.tensor(Eb, dtype=torch.float32, device="cuda"))
        torch.cuda.synchronize()
        say(f"  {precision}:")
        check("u", u.cpu().numpy()[idx], uo, tol)
        check("E", E.cpu().numpy()[idx], Eo, tol)
        check("qbar", gq.cpu().numpy()[idx], qo, tol)
        check("xbar", gx.cpu().numpy()[idx], xo, tol)
        G.close()


def test_uniform_65536_adjoint_against_finite_differences():
    """The GPU gradient of the force-matching loss (adjoint workload recipe at
    65,536 points) against the oracle's finite differences stored in
    golden/fd_adjoint_65536.txt: 64 position coordinates and 64 charges."""
    import os
    say("uniform 65,536 charges, p=6: adjoint against stored finite differences")
    from paper_2512_09478_amd import kifmm as kop
    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fd_adjoint_65536.txt")
    xs, qs = [], []
    for line in open(golden):
        if line.startswith("#") or not line.strip():
            continue
        kind, k, a, r = line.split()[:4]
        (xs if kind == "x" else qs).append((int(k), int(a), float(r)))
    w = workloads.make(4, n=65536)
    qt = workloads.adjoint_target_charges(w.charges, seed=4401)
    for precision, tol in (("fp32", 1e-5), ("split_bf16", 1e-4)):
        G = gpu_plan(w, precision)
        pos = G.positions.requires_grad_(True)
        q = torch.tensor(w.charges, dtype=torch.float32, device="cuda", requires_grad=True)
        with torch.no_grad():
            _, Et = G.evaluate(torch.tensor(qt, dtype=torch.float32, device="cuda"))
        Ft = torch.tensor(qt, dtype=torch.float32, device="cuda")[:, None] * Et
        u, E = kop(q, pos, G)
        loss = ((q[:, None] * E - Ft) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        gx = pos.grad.detach().cpu().numpy()
        gq = q.grad.detach().cpu().numpy()
        say(f"  {precision}:")
        check("dL/dx (64 coordinates)", np.array([gx[k, a] for k, a, _ in xs]), np.array([r for _, _, r in xs]), tol)
        check("dL/dq (64 charges)", np.array([gq[k] for k, _, _ in qs]), np.array([r for _, _, r in qs]), tol)
        G.close()


def test_clustered_1M_dipoles_gradient_and_stokes():
    """The other sums of eq. (1) at the headline size, with the inputs that
    `bench.py --f4` times: charges with point dipoles (u, E and dE/dx) and
    the Stokeslet velocity and pressure of point forces, sampled against the
    oracle on the same plan.  The library forms the Stokeslet's fourth harmonic charge
    about each box's own centre; the oracle's far and near parts show that
    the combination about the targets' leaf centres does not amplify errors
    of the far fields (about 0.9 here, against 12.5 about the root's centre),
    and the velocity is held to 2e-5 (FP32), the FP32 accuracy of far fields
    that make up most of it, and 1e-4 (split)."""
    from oracle import stokes
    say("clustered 1,048,576 points: dipoles, field gradient and Stokeslet")
    w = workloads.make(2)
    P = oracle_plan(w)
    idx = sample(w.n, 21)
    rng = np.random.default_rng(81)
    m = workloads.round_f32(rng.standard_normal((w.n, 3)) * 0.1 * w.n ** (-1.0 / 3.0))
    f = workloads.round_f32(rng.standard_normal((w.n, 3)))
    mu = 0.7
    t = time.time()
    uo, Eo, Go = kifmm.forward_dipoles(P, w.charges, m, targets=idx, grad=True)
    say(f"  oracle sampled dipole sweep {time.time() - t:.1f} s")
    t = time.time()
    vo, vmag, po = stokes.kifmm(P, f, mu, targets=idx, terms=True, frame="leaf", pressure=True)
    kappa = float(np.linalg.norm(vmag) / np.linalg.norm(vo))
    say(f"  oracle sampled Stokes sum {time.time() - t:.1f} s; amplification of the leaf-frame combination "
        f"{kappa:.2f}")
    assert kappa < 1.5
    q = torch.tensor(w.charges, dtype=torch.float32, device="cuda")
    md = torch.tensor(m, dtype=torch.float32, device="cuda")
    fd = torch.tensor(f, dtype=torch.float32, device="cuda")
    for precision, tol in (("fp32", 1e-5), ("split_bf16", 1e-4)):
        G = gpu_plan(w, precision)
        u, E = G.evaluate_dipoles(q, md)
        u2, E2, Gr = G.evaluate_gradient(q, md)
        v, pr = G.evaluate_stokes(fd, mu, pressure=True)
        torch.cuda.synchronize()
        say(f"  {precision}:")
        check("u (dipoles)", u.cpu().numpy()[idx], uo, tol)
        check("E (dipoles)", E.cpu().numpy()[idx], Eo, tol)
        check("u (gradient call)", u2.cpu().numpy()[idx], uo, tol)
        check("E (gradient call)", E2.cpu().numpy()[idx], Eo, tol)
        check("dE/dx", Gr.cpu().numpy()[idx], Go, tol)
        check("Stokes velocity", v.cpu().numpy()[idx], vo, 2e-5 if precision == "fp32" else tol)
        check("Stokes pressure", pr.cpu().numpy()[idx], po, tol)
        G.close()
