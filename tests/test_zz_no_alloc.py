"""The allocation-free clump reduction (kifmm_clump_reduce_noalloc, fixed
device scratch) against kifmm_clump_reduce through the C ABI: two calls in a
row, the second with fewer clumps over fewer pebbles; both against the
oracle's caller-order FP64 sums on the same field."""
import sys

import numpy as np
import pytest

import workloads
from oracle import clump

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def offsets(n, seed, cover):
    """Clumps of 0 to 700 pebbles over the first `cover` pebbles (several span
    blocks of 256)."""
    rng = np.random.default_rng(seed)
    sizes = []
    while True:
        s = int(rng.choice([0, 1, 5, 8, 100, 255, 256, 257, 700]))
        if sum(sizes) + s > cover:
            break
        sizes.append(s)
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def test_noalloc_clump_reduce_matches_allocating_call():
    from paper_2512_09478_amd import Plan
    print("allocation-free clump reduction", flush=True)
    sys.stdout.flush()
    w = workloads.make(4, n=9000)
    G = Plan(torch.tensor(w.positions, device="cuda"), "laplace", 4, 32, root=w.root)
    q = torch.tensor(w.charges, dtype=torch.float32, device="cuda")
    _, E = G.evaluate(q)
    qh = np.asarray(w.charges, np.float32).astype(np.float64)
    Eh = E.cpu().numpy().astype(np.float64)
    for seed, cover in ((1, 9000), (2, 3000)):   # the second call is smaller
        off = offsets(w.n, seed, cover)
        C = len(off) - 1
        cen = np.random.default_rng(seed + 10).random((C, 3))
        offd = torch.tensor(off, device="cuda")
        cend = torch.tensor(cen, device="cuda")
        F0, T0 = G.clump_reduce(q, E, offd, cend)
        F1 = torch.full((C, 3), np.nan, dtype=torch.float64, device="cuda")
        T1 = torch.full((C, 3), np.nan, dtype=torch.float64, device="cuda")
        G.clump_reduce_noalloc(q, E, offd, cend, F1, T1)
        G.synchronize()
        print(f"  C = {C} clumps over {off[-1]} pebbles", flush=True)
        assert torch.equal(F0, F1) and torch.equal(T0, T1)   # same kernels, same order
        Fo, To = clump.clump_reduce(w.positions, qh, Eh, off, cen)
        np.testing.assert_allclose(F1.cpu().numpy(), Fo, rtol=1e-12, atol=1e-12 * np.abs(Fo).max())
        np.testing.assert_allclose(T1.cpu().numpy(), To, rtol=1e-12, atol=1e-12 * np.abs(To).max())
    G.close()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    from paper_2512_09478_amd import KifmmError, Plan
    n = 11_184_641
    x = torch.rand((n, 3), dtype=torch.float64, device="cuda")
    G = Plan(x, "laplace", 2, 4096, root=((0, 0, 0), 1.0))
    q = torch.zeros(n, dtype=torch.float32, device="cuda")
    E = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    off = torch.tensor([0, n], dtype=torch.int64, device="cuda")
    cen = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    F = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(KifmmError) as ei:
        G.clump_reduce_noalloc(q, E, off, cen, F, F.clone())
    assert ei.value.code == -1
    G.close()
