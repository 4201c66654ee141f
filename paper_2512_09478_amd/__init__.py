"""KIFMM (kernel-independent fast multipole method) for MI355X.

Long-range Laplace/Coulomb and gravity potentials and fields of point and
clump charges (arXiv 2512.09478, Sections 2.2-2.4), evaluated by hand-written
HIP kernels behind the C ABI in include/kifmm.h; this package is the thin
Python binding (torch supplies device memory and streams).
"""
from ._lib import KifmmError, lib  # noqa: F401
from .plan import (ClumpForcesFunction, ClumpFunction, KifmmFunction, Plan, clump_forces,  # noqa: F401
                   clump_reduce, kifmm)
