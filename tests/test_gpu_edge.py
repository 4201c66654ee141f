"""GPU edge cases and error paths, each against the FP64 oracle where there
is a value to compare."""
import sys

import numpy as np
import pytest

import workloads
from oracle import direct, kifmm
from _parity import check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def run(x, q, kernel="laplace", p=4, leaf=8, adaptive=True, max_depth=21, root=None, precision="fp32"):
    from paper_2512_09478_amd import Plan
    pos = torch.tensor(x, dtype=torch.float64, device="cuda")
    G = Plan(pos, kernel, p, leaf, adaptive, max_depth, precision=precision, root=root)
    u, E = G.evaluate(torch.tensor(q, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    return G, u.cpu().numpy(), E.cpu().numpy()


def test_single_point_and_pair():
    say("N = 1 and N = 2")
    G, u, E = run(np.array([[0.3, 0.4, 0.5]]), np.array([2.0]))
    assert u[0] == 0.0 and np.all(E == 0.0)
    x = workloads.round_f32(np.array([[0.1, 0.2, 0.3], [0.7, 0.6, 0.2]]))
    q = np.array([1.5, -0.5])
    G, u, E = run(x, q)
    ud, Ed, _ = direct.potential_field(x, q)
    np.testing.assert_allclose(u, ud, rtol=1e-6)
    np.testing.assert_allclose(E, Ed, rtol=1e-6)


@pytest.mark.parametrize("max_depth", [6, 12, 21])
def test_coincident_points_reach_max_depth(max_depth):
    """300 coincident charges on a box corner force a chain of single-child
    boxes down to max_depth.  Their field then comes from the leaf's local
    expansion alone (the coincident pairs are skipped, no near field): a
    relative representation error delta of that expansion becomes a field
    error of about delta |u| / w over a leaf of width w = 2^-depth.  The FP64
    method's own field there drifts with depth for that reason (truncation),
    and the FP32 path adds delta ~ eps32 times the conditioning of the
    downward densities.  The bound on the coincident field is that product with
    a conditioning factor of 64 (measured: 15 at depth 12, 27 at depth 21,
    p = 4); every other output keeps the 1e-5 bound."""
    say(f"coincident points, max_depth {max_depth}")
    nc = 300
    x = np.tile(workloads.round_f32(np.array([[0.25, 0.5, 0.75]])), (nc, 1))
    x = np.concatenate([x, workloads.uniform_cube(np.random.default_rng(0), 200)])
    q = workloads.round_f32(np.random.default_rng(1).standard_normal(nc + 200))
    G, u, E = run(x, q, leaf=16, max_depth=max_depth, root=((0, 0, 0), 1.0))
    c = G.counts()
    assert c["depth"] == max_depth
    P = kifmm.plan(x, "laplace", 4, 16, True, max_depth, ((0, 0, 0), 1.0))
    uo, Eo = kifmm.forward(P, q)
    check("u", u, uo, 1e-5)
    check("E (other points)", E[nc:], Eo[nc:], 1e-5)
    eps32 = float(np.finfo(np.float32).eps) / 2
    bound = 64 * eps32 * np.abs(uo[:nc]).max() / 2.0 ** -max_depth
    err = np.abs(E[:nc] - Eo[:nc]).max()
    say(f"  coincident field |dE| {err:.3e}, bound {bound:.3e}")
    assert np.all(np.isfinite(E)) and err <= bound


def test_upper_face_and_explicit_root():
    say("points on the upper faces of an explicit root")
    rng = np.random.default_rng(2)
    x = workloads.uniform_cube(rng, 2000)
    x[:10, 0] = 1.0
    x[10:20, 1] = 1.0
    x[20:30] = 1.0
    q = workloads.round_f32(rng.standard_normal(2000))
    G, u, E = run(x, q, p=5, leaf=24, root=((0, 0, 0), 1.0))
    t = G.tree()
    P = kifmm.plan(x, "laplace", 5, 24, True, 21, ((0, 0, 0), 1.0))
    np.testing.assert_array_equal(t["keys"], P.tree.keys)
    uo, Eo = kifmm.forward(P, q)
    check("u", u, uo, 1e-5)
    check("E", E, Eo, 1e-5)


@pytest.mark.parametrize("leaf,max_depth,adaptive", [(1, 21, True), (8, 2, True), (50, 21, False), (4, 3, False)])
def test_leaf_and_depth_limits(leaf, max_depth, adaptive):
    say(f"leaf {leaf} max_depth {max_depth} adaptive {adaptive}")
    w = workloads.make(2, n=1500)
    G, u, E = run(w.positions, w.charges, p=3, leaf=leaf, adaptive=adaptive, max_depth=max_depth, root=w.root)
    P = kifmm.plan(w.positions, "laplace", 3, leaf, adaptive, max_depth, w.root)
    t = G.tree()
    np.testing.assert_array_equal(t["begin"], P.tree.begin)
    np.testing.assert_array_equal(t["is_leaf"], P.tree.is_leaf)
    uo, Eo = kifmm.forward(P, w.charges)
    check("u", u, uo, 1e-5)
    check("E", E, Eo, 1e-5)


@pytest.mark.parametrize("p", [2, 3, 5, 7])
def test_other_orders(p):
    say(f"order p = {p}")
    w = workloads.make(5, n=3000)
    G, u, E = run(w.positions, w.charges, kernel="gravity", p=p, leaf=32, max_depth=12, root=w.root)
    P = kifmm.plan(w.positions, "gravity", p, 32, True, 12, w.root)
    uo, Eo = kifmm.forward(P, w.charges)
    tol = 1e-4 if p >= 7 else 1e-5
    check("u", u, uo, tol)
    check("E", E, Eo, tol)


def test_automatic_root_and_negative_coordinates():
    say("automatic root around negative coordinates")
    rng = np.random.default_rng(4)
    x = workloads.round_f32(rng.standard_normal((3000, 3)) * 3.0 - 10.0)
    q = workloads.round_f32(rng.uniform(-1, 1, 3000))
    G, u, E = run(x, q, p=4, leaf=32)
    P = kifmm.plan(x, "laplace", 4, 32, True, 21, None)
    t = G.tree()
    assert t["side"] == P.tree.s and np.array_equal(t["lo"], P.tree.lo)
    uo, Eo = kifmm.forward(P, q)
    check("u", u, uo, 1e-5)
    check("E", E, Eo, 1e-5)


def test_rebuild_matches_fresh_setup_and_precision_switch():
    say("rebuild with moved points; precision switch")
    from paper_2512_09478_amd import Plan
    w = workloads.make(4, n=5000)
    rng = np.random.default_rng(5)
    x2 = np.clip(workloads.round_f32(w.positions + 0.01 * rng.standard_normal(w.positions.shape)), 0, 0.999)
    pos = torch.tensor(w.positions, dtype=torch.float64, device="cuda")
    q = torch.tensor(w.charges, dtype=torch.float32, device="cuda")
    G = Plan(pos, "laplace", 5, 32, True, 21, root=w.root)
    G.evaluate(q)
    G.rebuild(torch.tensor(x2, dtype=torch.float64, device="cuda"))
    u1, E1 = G.evaluate(q)
    H = Plan(torch.tensor(x2, dtype=torch.float64, device="cuda"), "laplace", 5, 32, True, 21, root=w.root)
    u2, E2 = H.evaluate(q)
    assert torch.equal(u1, u2) and torch.equal(E1, E2)
    G.set_precision("split_bf16")
    u3, E3 = G.evaluate(q)
    P = kifmm.plan(x2, "laplace", 5, 32, True, 21, w.root)
    uo, Eo = kifmm.forward(P, w.charges)
    check("u", u3, uo, 1e-4)
    check("E", E3, Eo, 1e-4)


def test_side_stream_and_phase_times():
    say("non-default stream, phase times")
    from paper_2512_09478_amd import Plan
    w = workloads.make(2, n=20000)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        pos = torch.tensor(w.positions, dtype=torch.float64, device="cuda")
        q = torch.tensor(w.charges, dtype=torch.float32, device="cuda")
        G = Plan(pos, "laplace", 4, 48, True, 21, root=w.root, profile=True)
        u, E = G.evaluate(q)
        ph = G.phase_times()
    s.synchronize()
    assert set(ph) >= {"m2l", "p2p", "total"} and ph["total"] > 0
    P = kifmm.plan(w.positions, "laplace", 4, 48, True, 21, w.root)
    uo, Eo = kifmm.forward(P, w.charges)
    check("u", u, uo, 1e-5)
    check("E", E, Eo, 1e-5)


def test_input_errors_leave_destroyable_handles():
    say("input errors")
    from paper_2512_09478_amd import KifmmError, Plan
    x = np.random.default_rng(6).random((100, 3))
    bad = x.copy()
    bad[17, 1] = np.nan
    with pytest.raises(KifmmError) as ei:
        Plan(torch.tensor(bad, device="cuda"), "laplace", 4, 8)
    assert ei.value.code == -2
    with pytest.raises(KifmmError) as ei:
        Plan(torch.tensor(x + 1.5, device="cuda"), "laplace", 4, 8, root=((0, 0, 0), 1.0))
    assert ei.value.code == -2
    G = Plan(torch.tensor(x, device="cuda"), "laplace", 4, 8)
    q = torch.ones(100, dtype=torch.float32, device="cuda")
    u, E = G.evaluate(q)
    off = torch.tensor([0, 50, 40, 100], dtype=torch.int64, device="cuda")   # not monotone
    cen = torch.zeros((3, 3), dtype=torch.float64, device="cuda")
    # the clump calls check their offsets on the device: NaN for the bad
    # clumps, the error at the next synchronisation
    F, T = G.clump_reduce(q, E, off, cen)
    with pytest.raises(KifmmError) as ei:
        G.synchronize()
    assert ei.value.code == -2
    assert torch.isnan(F[1]).all() and torch.isfinite(F[0]).all()
    G.synchronize()   # cleared
    off = torch.tensor([0, 50, 120], dtype=torch.int64, device="cuda")      # beyond N
    G.clump_reduce(q, E, off, cen[:2])
    with pytest.raises(KifmmError) as ei:
        G.synchronize()
    assert ei.value.code == -2
    G.clump_backward(q, E, torch.tensor([0, 50, 40, 100], dtype=torch.int64, device="cuda"), cen,
                     torch.ones((3, 3), dtype=torch.float64, device="cuda"))
    with pytest.raises(KifmmError) as ei:
        G.synchronize()
    assert ei.value.code == -2
    # registration checks them at once
    with pytest.raises(KifmmError) as ei:
        G.set_clumps(off)
    assert ei.value.code == -2
    with pytest.raises(KifmmError) as ei:
        G.clump_forces(q, cen[:0])     # nothing registered
    assert ei.value.code == -5
    # the handle still works and is destroyable
    u2, E2 = G.evaluate(q)
    assert torch.equal(u, u2)
    # an adjoint that reuses the forward pass needs one since the last rebuild
    G.rebuild(torch.tensor(x, device="cuda"))
    with pytest.raises(KifmmError) as ei:
        G.backward(None, q, None)
    assert ei.value.code == -5
    G.evaluate(q)
    G.backward(None, q, None)
    G.close()
    with pytest.raises(KifmmError):
        G.evaluate(q)



def test_pair_counts_follow_rebuild():
    """The V-pair and near-field pair counts are taken on request after each
    build: after a rebuild on other positions they are those of the new tree,
    checked against the oracle's lists of the same positions."""
    from paper_2512_09478_amd import Plan
    say("pair counts after a rebuild")
    rng = np.random.default_rng(31)
    xa = workloads.uniform_cube(rng, 3000)
    xb = workloads.round_f32(np.clip(workloads.clustered(rng, 3000), 0.0, np.nextafter(1.0, 0.0)))
    root = ((0.0, 0.0, 0.0), 1.0)
    G = Plan(torch.tensor(xa, dtype=torch.float64, device="cuda"), "laplace", 4, 16, root=root)
    ca = G.counts()
    G.rebuild(torch.tensor(xb, dtype=torch.float64, device="cuda"))
    cb = G.counts()
    O = kifmm.plan(xb, "laplace", 4, 16, True, 21, root)
    voff, _ = O.lists.csr("V")
    near = kifmm.near_lists(O)
    npts = O.tree.end - O.tree.begin
    pairs = sum(int(npts[b]) * int(npts[e]) for b, row in enumerate(near) for e in row)   # free space: no shifts
    assert cb["v_pairs"] == int(voff[-1])
    assert cb["p2p_pairs"] == pairs
    assert cb["boxes"] == O.tree.nboxes and ca["n"] == cb["n"] == 3000
    G.close()


def test_box_storage_grows_mid_build():
    """100 pairs of points 2^-19 apart with leaf size 1: each pair is a chain of
    single-child boxes down to the level that separates it, about 1,700 boxes
    in all, more than the 1,024 the build first allocates.  The level that
    overflows is redone after the storage grows; tree, lists and fields match
    the oracle."""
    from paper_2512_09478_amd import Plan
    say("box storage growth during the build")
    rng = np.random.default_rng(77)
    a = workloads.round_f32(0.1 + 0.8 * rng.random((100, 3)))
    b = workloads.round_f32(a + np.array([2.0 ** -19, 0.0, 0.0]))
    x = np.concatenate([a, b])
    q = workloads.round_f32(rng.standard_normal(200))
    root = ((0.0, 0.0, 0.0), 1.0)
    G = Plan(torch.tensor(x, dtype=torch.float64, device="cuda"), "laplace", 4, 1, root=root)
    t = G.tree()
    O = kifmm.plan(x, "laplace", 4, 1, True, 21, root)
    assert O.tree.nboxes > 1024
    np.testing.assert_array_equal(t["level"], O.tree.level)
    np.testing.assert_array_equal(t["anchor"], O.tree.anchor)
    np.testing.assert_array_equal(t["begin"], O.tree.begin)
    np.testing.assert_array_equal(t["parent"], O.tree.parent)
    for which in "UVWX":
        off, idx = G.list_csr(which)
        ooff, oidx = O.lists.csr(which)
        np.testing.assert_array_equal(off, ooff, err_msg=which)
        np.testing.assert_array_equal(idx, oidx, err_msg=which)
    u, E = G.evaluate(torch.tensor(q, dtype=torch.float32, device="cuda"))
    uo, Eo = kifmm.forward(O, q)
    say(f"  boxes {O.tree.nboxes}, depth {G.counts()['depth']}")
    check("u", u, uo, 1e-5)
    check("E", E, Eo, 1e-5)
    G.close()


@pytest.mark.parametrize("n", [3000, 20000])
def test_rebuild_resorts_from_previous_order(n):
    """Particles that move a little between builds: the rebuild starts from the
    previous order (points out of order with a neighbour sorted on their own
    and merged back), and keys, permutation and boxes equal the oracle's for
    the new positions, bit for bit; coincident pairs moved together keep
    equal keys, whose order is by caller index.  A large move falls back to
    the full sort with the same result."""
    from paper_2512_09478_amd import Plan
    say(f"rebuild from the previous order, n={n}")
    rng = np.random.default_rng(71)
    base = workloads.clustered(rng, n - 100)
    x = np.concatenate([base, base[:50], base[:50]])           # 50 coincident pairs
    x = workloads.round_f32(np.clip(x, 0.0, np.nextafter(1.0, 0.0)))
    root = ((0.0, 0.0, 0.0), 1.0)
    G = Plan(torch.tensor(x, dtype=torch.float64, device="cuda"), "laplace", 4, 32, root=root)
    for step, sigma in enumerate((1e-4, 1e-4, 3e-2)):
        dx = rng.standard_normal(x.shape) * sigma
        dx[n - 50:] = dx[n - 100:n - 50]                        # the pairs move together
        x = workloads.round_f32(np.clip(x + dx, 0.0, np.nextafter(1.0, 0.0)))
        G.rebuild(torch.tensor(x, dtype=torch.float64, device="cuda"))
        t = G.tree()
        O = kifmm.plan(x, "laplace", 4, 32, True, 21, root)
        np.testing.assert_array_equal(t["keys"], O.tree.keys)
        np.testing.assert_array_equal(t["perm"], O.tree.perm)
        np.testing.assert_array_equal(t["begin"], O.tree.begin)
        np.testing.assert_array_equal(t["level"], O.tree.level)
        st = G.build_stats()
        say(f"  step {step} (sigma {sigma}): {st}")
    st = G.build_stats()
    assert st["builds"] == 4 and st["resort_tried"] == 3 and st["resort_done"] >= 2
    u, E = G.evaluate(torch.tensor(workloads.round_f32(rng.standard_normal(n)), dtype=torch.float32, device="cuda"))
    assert torch.isfinite(u).all()
    G.close()
