"""GPU edge cases of the Stokeslet entry points (velocity, and velocity with
pressure), whose fourth harmonic charge is carried about each box's own
centre: trees without a far field, shallow and deep adaptive trees, repeated
calls, rebuilds and the error paths; values against the FP64 direct sums
where the method is exact there, else against the oracle's KIFMM on the same
plan."""
import sys

import numpy as np
import pytest

import workloads
from oracle import kifmm, stokes
from _parity import check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_plan(x, p=4, leaf=8, precision="fp32", root=None, kernel="laplace", periodic=False, m2l_rtol=0.0):
    from paper_2512_09478_amd import Plan
    return Plan(torch.tensor(x, dtype=torch.float64, device="cuda"), kernel, p, leaf, True, 21,
                precision=precision, root=root, periodic=periodic, m2l_rtol=m2l_rtol)


def velocity(G, f, mu):
    v = G.evaluate_stokes(torch.tensor(f, dtype=torch.float32, device="cuda"), mu)
    torch.cuda.synchronize()
    return v.cpu().numpy()


def flow(G, f, mu):
    v, p = G.evaluate_stokes(torch.tensor(f, dtype=torch.float32, device="cuda"), mu, pressure=True)
    torch.cuda.synchronize()
    return v.cpu().numpy(), p.cpu().numpy()


def test_stokes_without_far_field():
    """One point has no velocity or pressure; two points and a single leaf of
    100 are summed point to point (the Stokeslet pair sum itself)."""
    say("Stokes: N = 1, N = 2, one leaf of 100")
    G = gpu_plan(np.array([[0.3, 0.4, 0.5]]))
    v, p = flow(G, np.array([[1.0, -2.0, 0.5]]), 0.9)
    assert np.all(v == 0.0) and np.all(p == 0.0)
    x = workloads.round_f32(np.array([[0.1, 0.2, 0.3], [0.7, 0.6, 0.2]]))
    f = np.array([[1.0, 0.5, -0.25], [-0.5, 2.0, 1.0]])
    v, p = flow(gpu_plan(x), f, 0.9)
    np.testing.assert_allclose(v, stokes.direct(x, f, 0.9), rtol=1e-6)
    np.testing.assert_allclose(p, stokes.pressure_direct(x, f), rtol=1e-6)
    rng = np.random.default_rng(11)
    x = workloads.round_f32(rng.random((100, 3)))
    f = workloads.round_f32(rng.standard_normal((100, 3)))
    v, p = flow(gpu_plan(x, leaf=128), f, 0.9)
    check("u (one leaf)", v, stokes.direct(x, f, 0.9), 1e-5)
    check("p (one leaf)", p, stokes.pressure_direct(x, f), 1e-5)


@pytest.mark.parametrize("n,leaf,p,precision", [(300, 64, 4, "fp32"), (1200, 64, 4, "fp32"),
                                                (4000, 8, 4, "fp32"), (4000, 8, 6, "split_bf16")])
def test_stokes_shallow_and_deep_trees(n, leaf, p, precision):
    """Trees of depth 1 (no far field), 2 (the first far-field level only)
    and 6 (eight points per leaf on the clustered shape, where the frames of
    the fourth charge are shifted through many levels) against the oracle's
    same method."""
    say(f"Stokes: clustered n={n} leaf={leaf} p={p} {precision}")
    w = workloads.make(2, n=n)
    f = workloads.round_f32(np.random.default_rng(12).standard_normal((w.n, 3)))
    G = gpu_plan(w.positions, p, leaf, precision, root=w.root)
    depth = G.counts()["depth"]
    say(f"  depth {depth}")
    O = kifmm.plan(w.positions, "laplace", p, leaf, True, 21, w.root)
    uo, po = stokes.kifmm(O, f, 0.7, pressure=True)
    u, pr = flow(G, f, 0.7)
    tol = 1e-5 if precision == "fp32" else 1e-4
    check("u", u, uo, tol)
    check("p", pr, po, tol)


def test_stokes_repeat_rebuild_and_errors():
    """The same bits on a repeated call and after a rebuild equal to a fresh
    plan's; periodic and gravity plans and a non-positive viscosity are
    refused with the documented codes, with and without the pressure."""
    say("Stokes: repeat, rebuild, errors")
    from paper_2512_09478_amd import KifmmError
    w = workloads.make(4, n=6000)
    rng = np.random.default_rng(13)
    f = workloads.round_f32(rng.standard_normal((w.n, 3)))
    G = gpu_plan(w.positions, 6, 32, root=w.root, m2l_rtol=1e-6)
    v1 = velocity(G, f, 0.7)
    assert np.array_equal(v1, velocity(G, f, 0.7))
    # asking for the pressure leaves the velocity's bits alone; its own repeat
    v2, p2 = flow(G, f, 0.7)
    assert np.array_equal(v2, v1)
    assert np.array_equal(flow(G, f, 0.7)[1], p2)
    x2 = np.clip(workloads.round_f32(w.positions + 0.01 * rng.standard_normal(w.positions.shape)), 0, 0.999)
    G.rebuild(torch.tensor(x2, dtype=torch.float64, device="cuda"))
    H = gpu_plan(x2, 6, 32, root=w.root, m2l_rtol=1e-6)
    assert np.array_equal(velocity(G, f, 0.7), velocity(H, f, 0.7))
    assert np.array_equal(flow(G, f, 0.7)[1], flow(H, f, 0.7)[1])
    fd = torch.tensor(f, dtype=torch.float32, device="cuda")
    with pytest.raises(KifmmError) as ei:
        G.evaluate_stokes(fd, 0.0)
    assert ei.value.code == -1
    with pytest.raises(KifmmError) as ei:
        G.evaluate_stokes(fd, -1.0, pressure=True)
    assert ei.value.code == -1
    P = gpu_plan(w.positions, 4, 32, root=w.root, periodic=True)
    Q = gpu_plan(w.positions, 4, 32, root=w.root, kernel="gravity")
    for plan in (P, Q):
        for pressure in (False, True):
            with pytest.raises(KifmmError) as ei:
                plan.evaluate_stokes(fd, 1.0, pressure=pressure)
            assert ei.value.code == -5
    # the refused calls leave the plan usable
    assert np.array_equal(velocity(H, f, 0.7), velocity(G, f, 0.7))
