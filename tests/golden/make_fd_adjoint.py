"""Write ``fd_adjoint_65536.txt``: finite differences of the force-matching loss
of the adjoint workload, computed with the FP64 oracle only.

Workload: 65,536 charges uniform in the unit cube (the adjoint workload's
generator at the reduced size its specification allows when the oracle is too
slow at 524,288), q ~ N(0,1), p = 6, leaf 128, adaptive tree, M2L in the
truncated common basis (cut-off 1e-6).  Loss L = sum_i |q_i E_i - Ft_i|^2 with
Ft_i = qt_i E_i(qt) held fixed, qt = q + 0.1 N(0,1).

Stored: 64 (point, axis) position coordinates and 64 charges, each with the
central difference at steps h and h/2 combined by Richardson extrapolation
(tree frozen).  L is a polynomial of degree four in one charge, so that
combination is exact up to rounding there; in a position it removes the h^2
term.  The loss difference is summed from per-point force differences, which
keeps it free of the cancellation of L itself.

    python tests/golden/make_fd_adjoint.py [workers]
"""
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N = 65536
P_ORDER, LEAF, M2L_RTOL = 6, 128, 1e-6
HX = 2.0 ** -20          # position step (root side 1)
HQ = 2.0 ** -6           # charge step
SEED_COORDS = 6401
OUT = os.path.join(HERE, "fd_adjoint_65536.txt")

_state = {}


def _setup():
    import workloads
    from oracle import kifmm
    w = workloads.make(4, n=N)
    qt = workloads.adjoint_target_charges(w.charges, seed=4401)
    P = kifmm.plan(w.positions, w.kernel, P_ORDER, LEAF, True, 21, w.root, m2l_rtol=M2L_RTOL)
    _, Et = kifmm.forward(P, qt)
    Ft = qt[:, None] * Et
    _state.update(w=w, P=P, Ft=Ft)


def _forces(q, x=None):
    from oracle import kifmm
    P = _state["P"] if x is None else _state["P"].with_positions(x)
    _, E = kifmm.forward(P, q)
    return q[:, None] * E


def _dloss(Fp, Fm):
    # L(+) - L(-) = sum (Fp - Fm) . (Fp + Fm - 2 Ft)
    return float(np.sum((Fp - Fm) * (Fp + Fm - 2.0 * _state["Ft"])))


def _fd(task):
    kind, k, a = task
    w = _state["w"]
    vals = []
    for h in ((HQ, HQ / 2) if kind == "q" else (HX, HX / 2)):
        if kind == "q":
            qp = w.charges.copy(); qp[k] += h
            qm = w.charges.copy(); qm[k] -= h
            Fp, Fm = _forces(qp), _forces(qm)
        else:
            xp = w.positions.copy(); xp[k, a] += h
            xm = w.positions.copy(); xm[k, a] -= h
            Fp, Fm = _forces(w.charges, xp), _forces(w.charges, xm)
        vals.append(_dloss(Fp, Fm) / (2.0 * h))
    d1, d2 = vals
    return kind, k, a, (4.0 * d2 - d1) / 3.0, d1, d2


def tasks():
    rng = np.random.default_rng(SEED_COORDS)
    pts = rng.choice(N, 64, replace=False)
    axes = rng.integers(0, 3, 64)
    chg = rng.choice(N, 64, replace=False)
    return [("x", int(k), int(a)) for k, a in zip(pts, axes)] + [("q", int(k), -1) for k in chg]


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    T = tasks()
    t0 = time.time()
    with mp.get_context("fork").Pool(workers, initializer=_setup) as pool:
        rows = []
        for i, r in enumerate(pool.imap(_fd, T)):
            rows.append(r)
            print(f"[{time.time() - t0:7.1f} s] {i + 1}/{len(T)} {r[0]} {r[1]} {r[2]} {r[3]:.12e}", flush=True)
    with open(OUT, "w") as f:
        f.write("# Finite differences of L = sum_i |q_i E_i - Ft_i|^2 (FP64 oracle KIFMM, frozen tree),\n")
        f.write(f"# written by make_fd_adjoint.py: N = {N}, p = {P_ORDER}, leaf {LEAF}, m2l_rtol {M2L_RTOL},\n")
        f.write(f"# position step {HX!r}, charge step {HQ!r}; Richardson (4 D(h/2) - D(h)) / 3.\n")
        f.write("# columns: kind (x = position, q = charge) point axis richardson D(h) D(h/2)\n")
        for kind, k, a, r, d1, d2 in rows:
            f.write(f"{kind} {k} {a} {r:.17e} {d1:.17e} {d2:.17e}\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
