"""GPU parity of the periodic path (Section 2.4: periodic boundaries, neutral
cells) against the FP64 oracle through the C ABI.

Tree and lists (with image shifts) are compared bit for bit; potentials,
fields and the adjoint by relative L2 norms: <= 1e-5 for the FP32 path and
<= 1e-4 for the split-bf16 M2L path, the same discrete method on both sides
(tree, lists, surfaces, pseudoinverse cut-off and root lattice term).
"""
import sys

import numpy as np
import pytest

import workloads
from _parity import check
from oracle import kifmm
from oracle import periodic as per

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_bf16": 1e-4}
CELL = ((0.0, 0.0, 0.0), 1.0)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def built():
    import paper_2512_09478_amd as k
    k.lib()
    return k


def neutral_cell(n, seed):
    rng = np.random.default_rng(seed)
    m = n // 3
    x = np.concatenate([rng.random((n - 2 * m, 3)),
                        (np.array([0.1, 0.95, 0.5]) + 0.04 * rng.standard_normal((m, 3))) % 1.0,
                        (np.array([0.97, 0.2, 0.03]) + 0.04 * rng.standard_normal((m, 3))) % 1.0])
    x = workloads.round_f32(x)
    x = np.where(x >= 1.0, 0.0, x)
    q = rng.standard_normal(n)
    q[n - 2 * m:n - m] += 0.3
    q[n - m:] -= 0.3
    return x, workloads.round_f32(q - q.mean())


def cases():
    w = workloads.make(6, n=6 * 1094)
    xs, qs = neutral_cell(9000, 21)
    return {"platelets": (w.positions, w.charges, 64), "clusters": (xs, qs, 32)}


CASES = cases()


def plans(name, precision="fp32", p=6):
    from paper_2512_09478_amd import Plan
    x, q, leaf = CASES[name]
    G = Plan(torch.tensor(x, dtype=torch.float64, device="cuda"), "laplace", p, leaf, True, 21,
             precision=precision, root=CELL, periodic=True)
    O = kifmm.plan(x, "laplace", p, leaf, True, 21, CELL, periodic=True)
    return x, q, G, O


@pytest.mark.parametrize("name", sorted(CASES))
def test_periodic_tree_and_lists_bit_exact(built, name):
    say(f"periodic lists {name}")
    x, q, G, O = plans(name)
    t = G.tree()
    np.testing.assert_array_equal(t["perm"], O.tree.perm)
    np.testing.assert_array_equal(t["anchor"], O.tree.anchor)
    np.testing.assert_array_equal(t["is_leaf"], O.tree.is_leaf)
    shifted = 0
    for which in "UVWX":
        off, idx = G.list_csr(which)
        ooff, oidx = O.lists.csr(which)
        np.testing.assert_array_equal(off, ooff, err_msg=which)
        np.testing.assert_array_equal(idx, oidx, err_msg=which)
        shifted += int(np.sum(np.asarray(idx) >= (1 << 26)))
    assert shifted > 0   # the cell's faces are crossed
    # near lists: U plus the W/X pairs summed point to point
    near = kifmm.near_lists(O)
    off, idx = G.list_csr("N")
    np.testing.assert_array_equal(off[1:] - off[:-1], [len(r) for r in near])
    np.testing.assert_array_equal(idx, [e for r in near for e in r])


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_periodic_forward_parity(built, name, precision):
    say(f"periodic forward {name} {precision}")
    x, q, G, O = plans(name, precision)
    u, E = G.evaluate(torch.tensor(q, dtype=torch.float32, device="cuda"))
    uo, Eo = kifmm.forward(O, q)
    check("u", u.cpu().numpy(), uo, TOL[precision])
    check("E", E.cpu().numpy(), Eo, TOL[precision])


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_periodic_compressed_m2l_parity(built, precision):
    say(f"periodic compressed M2L {precision}")
    from paper_2512_09478_amd import Plan
    x, q, leaf = CASES["platelets"]
    G = Plan(torch.tensor(x, dtype=torch.float64, device="cuda"), "laplace", 6, leaf, True, 21,
             precision=precision, root=CELL, periodic=True, m2l_rtol=1e-6)
    O = kifmm.plan(x, "laplace", 6, leaf, True, 21, CELL, periodic=True, m2l_rtol=1e-6)
    u, E = G.evaluate(torch.tensor(q, dtype=torch.float32, device="cuda"))
    uo, Eo = kifmm.forward(O, q)
    check("u", u.cpu().numpy(), uo, TOL[precision])
    check("E", E.cpu().numpy(), Eo, TOL[precision])


def test_periodic_matches_ewald_sum(built):
    # the same run against the definition itself, at the method's accuracy
    say("periodic vs Ewald")
    x, q, G, O = plans("platelets")
    u, E = G.evaluate(torch.tensor(q, dtype=torch.float32, device="cuda"))
    t = np.arange(0, x.shape[0], 11)
    ue, Ee = per.ewald(x, q, 1.0, targets=t)
    # the method's own accuracy (not parity): rel-L2 only
    eu, eE = rel(u.cpu().numpy()[t], ue), rel(E.cpu().numpy()[t], Ee)
    say(f"  rel-L2 u {eu:.3e}  E {eE:.3e}")
    assert eu <= 5e-5 and eE <= 5e-5


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_periodic_backward_parity(built, precision):
    say(f"periodic backward {precision}")
    x, q, G, O = plans("clusters", precision)
    rng = np.random.default_rng(5)
    ub = workloads.round_f32(rng.standard_normal(x.shape[0]))
    Eb = workloads.round_f32(rng.standard_normal((x.shape[0], 3)))
    qt = torch.tensor(q, dtype=torch.float32, device="cuda")
    gq, gx = G.backward(qt, torch.tensor(ub, dtype=torch.float32, device="cuda"),
                        torch.tensor(Eb, dtype=torch.float32, device="cuda"))
    qo, xo = kifmm.vjp(O, q, ub, Eb)
    check("qbar", gq, qo, TOL[precision])
    check("xbar", gx, xo, TOL[precision])
    # reusing the forward pass gives the same product
    G.evaluate(qt)
    gq2, gx2 = G.backward(None, torch.tensor(ub, dtype=torch.float32, device="cuda"),
                          torch.tensor(Eb, dtype=torch.float32, device="cuda"))
    assert rel(gq2.cpu().numpy(), gq.cpu().numpy().astype(np.float64)) <= 1e-6
    assert rel(gx2.cpu().numpy(), gx.cpu().numpy().astype(np.float64)) <= 1e-6


def test_periodic_dipoles_parity(built):
    say("periodic dipoles")
    x, q, G, O = plans("platelets")
    rng = np.random.default_rng(6)
    m = workloads.round_f32(rng.standard_normal((x.shape[0], 3)) * 3e-3)
    u, E = G.evaluate_dipoles(None, torch.tensor(m, dtype=torch.float32, device="cuda"))
    uo, Eo = kifmm.forward_dipoles(O, None, m)
    check("u", u.cpu().numpy(), uo, TOL["fp32"])
    check("E", E.cpu().numpy(), Eo, TOL["fp32"])


def test_periodic_field_gradient_parity(built):
    say("periodic field gradient")
    x, q, G, O = plans("clusters")
    rng = np.random.default_rng(7)
    m = workloads.round_f32(rng.standard_normal((x.shape[0], 3)) * 3e-3)
    u, E, Gr = G.evaluate_gradient(torch.tensor(q, dtype=torch.float32, device="cuda"),
                                   torch.tensor(m, dtype=torch.float32, device="cuda"))
    uo, Eo, Go = kifmm.forward_dipoles(O, q, m, grad=True)
    check("u", u, uo, TOL["fp32"])
    check("E", E, Eo, TOL["fp32"])
    check("dE/dx", Gr, Go, TOL["fp32"])


@pytest.mark.parametrize("n,leaf", [(20, 64), (300, 64)])
def test_periodic_shallow_trees(built, n, leaf):
    # a root leaf (its own 27 images in U) and a depth-1 tree (V lists at level 1 only)
    say(f"periodic shallow n={n} leaf={leaf}")
    from paper_2512_09478_amd import Plan
    x, q = neutral_cell(n, 22)
    G = Plan(torch.tensor(x, dtype=torch.float64, device="cuda"), "laplace", 6, leaf, True, 21, root=CELL,
             periodic=True)
    O = kifmm.plan(x, "laplace", 6, leaf, True, 21, CELL, periodic=True)
    u, E = G.evaluate(torch.tensor(q, dtype=torch.float32, device="cuda"))
    uo, Eo = kifmm.forward(O, q)
    say(f"  depth {G.counts()['depth']}")
    check("u", u.cpu().numpy(), uo, 1e-5)
    check("E", E.cpu().numpy(), Eo, 1e-5)


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_periodic_uniform_tree(built, precision):
    # every leaf at depth 2 (4 x 4 x 4 leaves): neighbours wrap at every face
    say(f"periodic uniform tree {precision}")
    from paper_2512_09478_amd import Plan
    w = workloads.make(1, n=4096)
    q = workloads.round_f32(w.charges - w.charges.mean())
    G = Plan(torch.tensor(w.positions, dtype=torch.float64, device="cuda"), "laplace", 4, 64, False, 21,
             precision=precision, root=CELL, periodic=True)
    O = kifmm.plan(w.positions, "laplace", 4, 64, False, 21, CELL, periodic=True)
    for which in "UVWX":
        off, idx = G.list_csr(which)
        ooff, oidx = O.lists.csr(which)
        np.testing.assert_array_equal(idx, oidx, err_msg=which)
    u, E = G.evaluate(torch.tensor(q, dtype=torch.float32, device="cuda"))
    uo, Eo = kifmm.forward(O, q)
    check("u", u.cpu().numpy(), uo, TOL[precision])
    check("E", E.cpu().numpy(), Eo, TOL[precision])


def test_periodic_argument_errors(built):
    from paper_2512_09478_amd import KifmmError, Plan
    x = torch.rand((50, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(KifmmError):
        Plan(x, "gravity", 4, 16, root=CELL, periodic=True)
    with pytest.raises(KifmmError):
        Plan(x, "laplace", 4, 16, periodic=True)
