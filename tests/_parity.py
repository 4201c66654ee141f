"""Parity measures shared by the GPU tests.

Every floating-point output is compared with the oracle's by two numbers:
the relative L2 error over all entries, ||y - y_ref||_2 / ||y_ref||_2, which
must stay within the path's tolerance, and the worst element,
max_i |y_i - y_ref,i| / max_i |y_ref,i|, which must stay within ten times it
(so that an error confined to a few targets, e.g. one leaf, cannot hide in the
norm over all of them).
"""
import sys

import numpy as np

WORST_FACTOR = 10.0


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def worst(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def check(name, got, ref, tol, log=True):
    """Assert rel-L2 <= tol and worst element <= 10 tol; returns (rel-L2, worst)."""
    if hasattr(got, "detach"):
        got = got.detach().cpu().numpy()
    e2, ei = rel(got, ref), worst(got, ref)
    if log:
        print(f"    {name}: rel-L2 {e2:.3e} (bound {tol:.0e}), worst element {ei:.3e} "
              f"(bound {WORST_FACTOR * tol:.0e})", flush=True)
        sys.stdout.flush()
    assert e2 <= tol, f"{name}: rel-L2 {e2:.3e} > {tol:.1e}"
    assert ei <= WORST_FACTOR * tol, f"{name}: worst element {ei:.3e} > {WORST_FACTOR * tol:.1e}"
    return e2, ei
