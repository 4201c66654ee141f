"""CPU oracle for the KIFMM hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 implementation of what the GPU library computes, written
from the paper's description of the kernel-independent fast multipole method
(Section 2.2: octree with at most M points per leaf, upward pass, downward
pass, leaf evaluation; equivalent densities on surfaces and automatically
computed translation matrices) and its problem statement (eq. (1) with the
Laplace/Coulomb potential of eq. (3) and the gravitational one of eq. (4);
clump aggregation of Section 2.4).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2512_09478_amd``) and never imports it; the library never imports it
either.

Modules
  pairsum    plain C double loops for pair sums (direct sum, near field)
  direct     exact O(N^2) sums: potential, field, Hessian, gradients
  tree       root cube, Morton keys, sort, octree, interaction lists
  operators  surfaces, kernel matrices, truncated-SVD pseudoinverses
  kifmm      FMM forward sweep and its discrete adjoint
  clump      per-clump force and torque
  stokes     Stokeslet sums of point forces (direct, and through the Laplace KIFMM)
  closed_forms  analytic reference values used to pin the above
"""
