"""ctypes loader for the oracle's plain-C pair sums (``csrc/pairsum.c``).

TEST INFRASTRUCTURE ONLY.  The shared object is built next to this file by
``build()``; if it is missing it is compiled here on first use (gcc, -O2,
OpenMP, no fast-math, no FP contraction).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "pairsum.c")
_SO = os.path.join(_HERE, "_pairsum.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the helper; returns the path of the shared object."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            P = ctypes.c_void_p
            I = ctypes.c_int64
            D = ctypes.c_double
            lib.oracle_direct.argtypes = [I, P, I, P, P, P, D, P, P, P]
            lib.oracle_direct.restype = None
            lib.oracle_p2p.argtypes = [I, P, P, P, P, P, P, P, P, P, P, D, P, P, P]
            lib.oracle_p2p.restype = None
            _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def direct(xt, ys, s, m=None, c=1.0, hess=False):
    """Exact sums over all sources.  Returns (u [nt], E [nt,3], H [nt,6] or None)."""
    lib = _load()
    xt = _c64(xt, (-1, 3))
    ys = _c64(ys, (-1, 3))
    s = _c64(s, (-1,))
    m = _c64(m, (-1, 3))
    nt, ns = xt.shape[0], ys.shape[0]
    u = np.zeros(nt)
    e = np.zeros((nt, 3))
    h = np.zeros((nt, 6)) if hess else None
    lib.oracle_direct(nt, _p(xt), ns, _p(ys), _p(s), _p(m), float(c), _p(u), _p(e), _p(h))
    return u, e, h


def p2p(tidx, tleaf, begin, end, uoff, uidx, x, s, m=None, c=1.0, hess=False, ushift=None):
    """Near-field sums over U lists for the sorted targets ``tidx`` (``ushift``:
    optional [len(uidx), 3] displacement of each list entry's points)."""
    lib = _load()
    i64 = lambda a: np.ascontiguousarray(a, dtype=np.int64)
    tidx, tleaf, begin, end, uoff, uidx = map(i64, (tidx, tleaf, begin, end, uoff, uidx))
    x = _c64(x, (-1, 3))
    s = _c64(s, (-1,))
    m = _c64(m, (-1, 3))
    ushift = _c64(ushift, (-1, 3))
    nt = tidx.shape[0]
    u = np.zeros(nt)
    e = np.zeros((nt, 3))
    h = np.zeros((nt, 6)) if hess else None
    lib.oracle_p2p(nt, _p(tidx), _p(tleaf), _p(begin), _p(end), _p(uoff), _p(uidx), _p(ushift),
                   _p(x), _p(s), _p(m), float(c), _p(u), _p(e), _p(h))
    return u, e, h
