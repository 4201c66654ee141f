"""Python front end: a plan handle and the autograd wrapper.

Torch provides device memory and the stream; every step of the evaluation runs
in libkifmm.so.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import KifmmError, Options, check

KERNELS = {"laplace": _lib.KIFMM_LAPLACE, "coulomb": _lib.KIFMM_LAPLACE, "gravity": _lib.KIFMM_GRAVITY}
PRECISIONS = {"fp32": _lib.KIFMM_FP32, "split_bf16": _lib.KIFMM_SPLIT_BF16}
PHASES = ["p2m", "up", "p2l", "m2l", "down", "far", "p2p", "total"]


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _need(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.contiguous()


class Plan:
    """KIFMM plan for N points: tree, lists and operators on the device."""

    def __init__(self, positions: torch.Tensor, kernel: str = "laplace", p: int = 6, leaf_size: int = 128,
                 adaptive: bool = True, max_depth: int = 21, precision: str = "fp32",
                 pinv_rtol: float = 1e-7, root=None, profile: bool = False, stream=None,
                 periodic: bool = False, m2l_rtol: float = 0.0):
        L = _lib.lib()
        self.n = int(positions.shape[0])
        self.positions = _need(positions, torch.float64, (self.n, 3), "positions")
        self.kernel = kernel
        self.p = p
        self.leaf_size = leaf_size
        opt = Options()
        L.kifmm_default_options(ctypes.byref(opt))
        opt.adaptive = int(bool(adaptive))
        opt.max_depth = int(max_depth)
        opt.precision = PRECISIONS[precision]
        opt.pinv_rtol = float(pinv_rtol)
        opt.profile = int(bool(profile))
        opt.periodic = int(bool(periodic))
        opt.m2l_rtol = float(m2l_rtol)
        self.periodic = bool(periodic)
        if root is not None:
            opt.explicit_root = 1
            for d in range(3):
                opt.root_lo[d] = float(root[0][d])
            opt.root_side = float(root[1])
        h = ctypes.c_void_p()
        check(L.kifmm_setup_ex(_ptr(self.positions), self.n, KERNELS[kernel], int(p), int(leaf_size),
                               ctypes.byref(opt), _stream(stream), ctypes.byref(h)))
        self._h = h
        # changes whenever the forward state held by the library changes; None
        # while there is no reusable forward pass
        self._fwd_token = None
        self._calls = 0

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.lib().kifmm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if not self._h or not self._h.value:
            raise KifmmError(-5, "plan is closed")
        return self._h

    # -- calls
    def rebuild(self, positions: torch.Tensor, stream=None):
        self.positions = _need(positions, torch.float64, (self.n, 3), "positions")
        self._fwd_token = None
        check(_lib.lib().kifmm_rebuild(self.handle, _ptr(self.positions), _stream(stream)))

    def set_precision(self, precision: str):
        self._fwd_token = None
        check(_lib.lib().kifmm_set_precision(self.handle, PRECISIONS[precision]))

    def _new_forward_state(self):
        self._calls += 1
        self._fwd_token = self._calls
        return self._fwd_token

    def evaluate(self, charges: torch.Tensor, potential=True, field=True, stream=None):
        q = _need(charges, torch.float32, (self.n,), "charges")
        u = torch.empty(self.n, dtype=torch.float32, device=q.device) if potential else None
        E = torch.empty((self.n, 3), dtype=torch.float32, device=q.device) if field else None
        self._fwd_token = None
        check(_lib.lib().kifmm_evaluate(self.handle, _ptr(q), _ptr(u), _ptr(E), _stream(stream)))
        self._new_forward_state()
        return u, E

    def evaluate_dipoles(self, charges, dipoles, potential=True, field=True, stream=None):
        """u, E of charges (or None) and point dipoles m at the plan's points."""
        q = None if charges is None else _need(charges, torch.float32, (self.n,), "charges")
        m = _need(dipoles, torch.float32, (self.n, 3), "dipoles")
        u = torch.empty(self.n, dtype=torch.float32, device=m.device) if potential else None
        E = torch.empty((self.n, 3), dtype=torch.float32, device=m.device) if field else None
        self._fwd_token = None
        check(_lib.lib().kifmm_evaluate_dipoles(self.handle, _ptr(q), _ptr(m), _ptr(u), _ptr(E), _stream(stream)))
        return u, E

    def evaluate_gradient(self, charges=None, dipoles=None, potential=True, field=True, stream=None):
        """u, E and dE/dx ([N,6]: xx, yy, zz, xy, xz, yz) of charges and/or point dipoles."""
        q = None if charges is None else _need(charges, torch.float32, (self.n,), "charges")
        m = None if dipoles is None else _need(dipoles, torch.float32, (self.n, 3), "dipoles")
        dev = self.positions.device
        u = torch.empty(self.n, dtype=torch.float32, device=dev) if potential else None
        E = torch.empty((self.n, 3), dtype=torch.float32, device=dev) if field else None
        G = torch.empty((self.n, 6), dtype=torch.float32, device=dev)
        self._fwd_token = None
        check(_lib.lib().kifmm_evaluate_gradient(self.handle, _ptr(q), _ptr(m), _ptr(u), _ptr(E), _ptr(G),
                                                 _stream(stream)))
        return u, E, G

    def evaluate_stokes(self, forces, viscosity=1.0, stream=None, pressure=False):
        """Velocity [N, 3] of point forces [N, 3] (Stokeslet sum) at the plan's
        points; with ``pressure`` also the pressure [N] of the flow."""
        f = _need(forces, torch.float32, (self.n, 3), "forces")
        u = torch.empty((self.n, 3), dtype=torch.float32, device=f.device)
        self._fwd_token = None
        if not pressure:
            check(_lib.lib().kifmm_evaluate_stokes(self.handle, _ptr(f), float(viscosity), _ptr(u),
                                                   _stream(stream)))
            return u
        p = torch.empty((self.n,), dtype=torch.float32, device=f.device)
        check(_lib.lib().kifmm_evaluate_stokes_ex(self.handle, _ptr(f), float(viscosity), _ptr(u), _ptr(p),
                                                  _stream(stream)))
        return u, p

    def backward(self, charges, grad_potential=None, grad_field=None, stream=None):
        """dL/dq, dL/dx.  ``charges=None`` reuses the charges and forward
        densities of the last evaluate on this plan (no forward sweep)."""
        q = None if charges is None else _need(charges, torch.float32, (self.n,), "charges")
        gu = None if grad_potential is None else _need(grad_potential, torch.float32, (self.n,), "grad_potential")
        gE = None if grad_field is None else _need(grad_field, torch.float32, (self.n, 3), "grad_field")
        dev = self.positions.device
        gq = torch.empty(self.n, dtype=torch.float32, device=dev)
        gx = torch.empty((self.n, 3), dtype=torch.float32, device=dev)
        if q is not None:
            self._fwd_token = None
        check(_lib.lib().kifmm_backward(self.handle, _ptr(q), _ptr(gu), _ptr(gE), _ptr(gq), _ptr(gx),
                                        _stream(stream)))
        if q is not None:
            self._new_forward_state()
        return gq, gx

    def clump_reduce(self, charges, field, offsets, centers, stream=None):
        C = int(offsets.shape[0]) - 1
        q = _need(charges, torch.float32, (self.n,), "charges")
        E = _need(field, torch.float32, (self.n, 3), "field")
        off = _need(offsets, torch.int64, (C + 1,), "offsets")
        cen = _need(centers, torch.float64, (C, 3), "centers")
        F = torch.empty((C, 3), dtype=torch.float64, device=q.device)
        T = torch.empty((C, 3), dtype=torch.float64, device=q.device)
        check(_lib.lib().kifmm_clump_reduce(self.handle, _ptr(q), _ptr(E), _ptr(off), C, _ptr(cen), _ptr(F),
                                            _ptr(T), _stream(stream)))
        return F, T

    def clump_reduce_noalloc(self, charges, field, offsets, centers, force, torque, stream=None):
        """clump_reduce into caller-given force and torque [C, 3] float64,
        through the entry point that allocates nothing (fixed device scratch)."""
        C = int(offsets.shape[0]) - 1
        q = _need(charges, torch.float32, (self.n,), "charges")
        E = _need(field, torch.float32, (self.n, 3), "field")
        off = _need(offsets, torch.int64, (C + 1,), "offsets")
        cen = _need(centers, torch.float64, (C, 3), "centers")
        F = _need(force, torch.float64, (C, 3), "force")
        T = _need(torque, torch.float64, (C, 3), "torque")
        if F.data_ptr() != force.data_ptr() or T.data_ptr() != torque.data_ptr():
            raise ValueError("force and torque must be contiguous")
        check(_lib.lib().kifmm_clump_reduce_noalloc(self.handle, _ptr(q), _ptr(E), _ptr(off), C, _ptr(cen),
                                                    _ptr(F), _ptr(T), _stream(stream)))
        return F, T

    def clump_backward(self, charges, field, offsets, centers, grad_force=None, grad_torque=None, stream=None):
        """Direct parts of the clump VJP: (dL/dq, dL/dE, dL/dx, dL/dX_c)."""
        C = int(offsets.shape[0]) - 1
        q = _need(charges, torch.float32, (self.n,), "charges")
        E = _need(field, torch.float32, (self.n, 3), "field")
        off = _need(offsets, torch.int64, (C + 1,), "offsets")
        cen = _need(centers, torch.float64, (C, 3), "centers")
        Fb = None if grad_force is None else _need(grad_force, torch.float64, (C, 3), "grad_force")
        Tb = None if grad_torque is None else _need(grad_torque, torch.float64, (C, 3), "grad_torque")
        dev = q.device
        qb = torch.empty(self.n, dtype=torch.float32, device=dev)
        Eb = torch.empty((self.n, 3), dtype=torch.float32, device=dev)
        xb = torch.empty((self.n, 3), dtype=torch.float32, device=dev)
        Xb = torch.empty((C, 3), dtype=torch.float64, device=dev)
        check(_lib.lib().kifmm_clump_backward(self.handle, _ptr(q), _ptr(E), _ptr(off), C, _ptr(cen), _ptr(Fb),
                                              _ptr(Tb), _ptr(qb), _ptr(Eb), _ptr(xb), _ptr(Xb), _stream(stream)))
        return qb, Eb, xb, Xb

    def set_clumps(self, offsets, stream=None):
        """Register clumps (CSR offsets [C+1] int64 over caller order, checked
        here) for clump_forces; they stay through rebuild."""
        C = int(offsets.shape[0]) - 1
        off = _need(offsets, torch.int64, (C + 1,), "offsets")
        check(_lib.lib().kifmm_set_clumps(self.handle, _ptr(off), C, _stream(stream)))
        self.clumps = C
        self._fwd_token = None

    def clump_forces(self, charges, centers, field=False, stream=None):
        """Per-clump force and torque of the registered clumps, from an
        evaluation without the point-to-point pairs inside a clump (they add
        nothing to either); with field=True also the pebble fields used."""
        C = getattr(self, "clumps", 0)
        q = _need(charges, torch.float32, (self.n,), "charges")
        cen = _need(centers, torch.float64, (C, 3), "centers")
        F = torch.empty((C, 3), dtype=torch.float64, device=q.device)
        T = torch.empty((C, 3), dtype=torch.float64, device=q.device)
        E = torch.empty((self.n, 3), dtype=torch.float32, device=q.device) if field else None
        self._fwd_token = None
        check(_lib.lib().kifmm_clump_forces(self.handle, _ptr(q), _ptr(cen), _ptr(F), _ptr(T), _ptr(E),
                                            _stream(stream)))
        self._new_forward_state()
        return (F, T, E) if field else (F, T)

    def clump_forces_backward(self, charges, centers, grad_force=None, grad_torque=None, stream=None):
        """dL/dq, dL/dx, dL/dX_c of the last clump_forces (whole gradient)."""
        C = getattr(self, "clumps", 0)
        q = _need(charges, torch.float32, (self.n,), "charges")
        cen = _need(centers, torch.float64, (C, 3), "centers")
        Fb = None if grad_force is None else _need(grad_force, torch.float64, (C, 3), "grad_force")
        Tb = None if grad_torque is None else _need(grad_torque, torch.float64, (C, 3), "grad_torque")
        dev = q.device
        gq = torch.empty(self.n, dtype=torch.float32, device=dev)
        gx = torch.empty((self.n, 3), dtype=torch.float32, device=dev)
        gX = torch.empty((C, 3), dtype=torch.float64, device=dev)
        check(_lib.lib().kifmm_clump_forces_backward(self.handle, _ptr(q), _ptr(cen), _ptr(Fb), _ptr(Tb), _ptr(gq),
                                                     _ptr(gx), _ptr(gX), _stream(stream)))
        return gq, gx, gX

    def synchronize(self, stream=None):
        """Wait for the plan's work and raise input errors found on the device."""
        check(_lib.lib().kifmm_synchronize(self.handle, _stream(stream)))

    # -- introspection
    def counts(self) -> dict:
        """Sizes of the tree and lists.  The V-pair and near-field pair counts
        are taken on the first call after a build (two small kernels on the
        plan's last stream, which is then synchronised)."""
        out = (ctypes.c_int64 * 10)()
        check(_lib.lib().kifmm_get_counts(self.handle, out))
        keys = ["boxes", "leaves", "depth", "v_pairs", "p2p_pairs", "w_pairs", "x_pairs", "u_pairs", "n",
                "surface_points"]
        return dict(zip(keys, [int(v) for v in out]))

    def m2l_rank(self) -> tuple:
        """(rank of the M2L operators in use, tile the M2L kernel runs at)."""
        out = (ctypes.c_int64 * 2)()
        check(_lib.lib().kifmm_get_m2l_rank(self.handle, out))
        return int(out[0]), int(out[1])

    def build_stats(self) -> dict:
        """Tree builds of the plan, and how many re-sorted from the previous order."""
        out = (ctypes.c_int64 * 3)()
        check(_lib.lib().kifmm_get_build_stats(self.handle, out))
        return dict(builds=int(out[0]), resort_tried=int(out[1]), resort_done=int(out[2]))

    def operator(self, which: int):
        """(values, rank) of the plan's FP64 operators: 0 singular values of
        K(uc, ue), 1 singular values of the stacked M2L operators, 2 UC2E [n, n]."""
        L = _lib.lib()
        out = (ctypes.c_int64 * 2)()
        check(L.kifmm_get_operator(self.handle, int(which), None, 0, out))
        v = np.empty(int(out[0]), dtype=np.float64)
        check(L.kifmm_get_operator(self.handle, int(which), v.ctypes.data_as(ctypes.c_void_p), v.size, out))
        if which == 2:
            n = int(round(np.sqrt(v.size)))
            v = v.reshape(n, n)
        return v, int(out[1])

    def tree(self) -> dict:
        c = self.counts()
        N, B = c["n"], c["boxes"]
        keys = np.empty(N, dtype=np.uint64)
        perm = np.empty(N, dtype=np.int64)
        level = np.empty(B, dtype=np.int32)
        anchor = np.empty((B, 3), dtype=np.int32)
        begin = np.empty(B, dtype=np.int64)
        end = np.empty(B, dtype=np.int64)
        parent = np.empty(B, dtype=np.int64)
        leaf = np.empty(B, dtype=np.int8)
        root = np.empty(4, dtype=np.float64)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        check(_lib.lib().kifmm_copy_tree(self.handle, p(keys), p(perm), p(level), p(anchor), p(begin), p(end),
                                         p(parent), p(leaf), p(root)))
        return dict(keys=keys, perm=perm, level=level, anchor=anchor, begin=begin, end=end, parent=parent,
                    is_leaf=leaf.astype(bool), lo=root[:3].copy(), side=float(root[3]))

    def list_csr(self, which: str):
        B = self.counts()["boxes"]
        off = np.empty(B + 1, dtype=np.int64)
        L = _lib.lib()
        check(L.kifmm_copy_list(self.handle, which.encode(), off.ctypes.data_as(ctypes.c_void_p), None))
        idx = np.empty(int(off[-1]), dtype=np.int64)
        check(L.kifmm_copy_list(self.handle, which.encode(), off.ctypes.data_as(ctypes.c_void_p),
                                idx.ctypes.data_as(ctypes.c_void_p) if idx.size else None))
        return off, idx

    def phase_times(self, back: int = 0) -> dict:
        """Phase times (ms) of the profiled call ``back`` calls before the last."""
        out = (ctypes.c_float * 8)()
        n = check(_lib.lib().kifmm_get_phase_times_at(self.handle, int(back), out, 8))
        return {PHASES[k]: float(out[k]) for k in range(n)}


class KifmmFunction(torch.autograd.Function):
    """(charges, positions) -> (potential, field) with the library's adjoint as backward.

    ``positions`` must be the tensor the plan was built from (the tree is
    frozen at those positions); its gradient is returned in float64.
    """

    @staticmethod
    def forward(ctx, charges, positions, plan: Plan):
        if positions.data_ptr() != plan.positions.data_ptr():
            raise ValueError("positions must be the tensor the plan was built from")
        u, E = plan.evaluate(charges)
        ctx.plan = plan
        ctx.token = plan._fwd_token
        ctx.save_for_backward(charges)
        return u, E

    @staticmethod
    def backward(ctx, gu, gE):
        (charges,) = ctx.saved_tensors
        gu = None if gu is None else gu.contiguous().float()
        gE = None if gE is None else gE.contiguous().float()
        # the library still holds this forward pass unless the plan has been
        # used since; autograd forbids in-place changes of the saved charges
        same = ctx.token is not None and ctx.plan._fwd_token == ctx.token
        gq, gx = ctx.plan.backward(None if same else charges, gu, gE)
        return gq, gx.to(torch.float64), None


def kifmm(charges, positions, plan: Plan):
    return KifmmFunction.apply(charges, positions, plan)


class ClumpFunction(torch.autograd.Function):
    """(charges, field, positions, centers) -> per-clump (force, torque) with
    the library's backward; compose with ``kifmm`` for the field, so that the
    gradient of a clump loss reaches the charges and positions through both
    the aggregation and the FMM adjoint."""

    @staticmethod
    def forward(ctx, charges, field, positions, centers, plan: Plan, offsets):
        if positions.data_ptr() != plan.positions.data_ptr():
            raise ValueError("positions must be the tensor the plan was built from")
        F, T = plan.clump_reduce(charges, field, offsets, centers)
        ctx.plan = plan
        ctx.offsets = offsets
        ctx.save_for_backward(charges, field, centers)
        return F, T

    @staticmethod
    def backward(ctx, gF, gT):
        charges, field, centers = ctx.saved_tensors
        gF = None if gF is None else gF.contiguous().double()
        gT = None if gT is None else gT.contiguous().double()
        qb, Eb, xb, Xb = ctx.plan.clump_backward(charges, field.detach(), ctx.offsets, centers, gF, gT)
        return qb, Eb, xb.to(torch.float64), Xb, None, None


def clump_reduce(charges, field, positions, centers, plan: Plan, offsets):
    return ClumpFunction.apply(charges, field, positions, centers, plan, offsets)


class ClumpForcesFunction(torch.autograd.Function):
    """(charges, positions, centers) -> per-clump (force, torque) of the
    plan's registered clumps, with the library's whole gradient as backward."""

    @staticmethod
    def forward(ctx, charges, positions, centers, plan: Plan):
        if positions.data_ptr() != plan.positions.data_ptr():
            raise ValueError("positions must be the tensor the plan was built from")
        F, T = plan.clump_forces(charges, centers)
        ctx.plan = plan
        ctx.token = plan._fwd_token
        ctx.save_for_backward(charges, centers)
        return F, T

    @staticmethod
    def backward(ctx, gF, gT):
        charges, centers = ctx.saved_tensors
        if ctx.token is None or ctx.plan._fwd_token != ctx.token:
            # the plan has been used since: redo the forward pass
            ctx.plan.clump_forces(charges, centers)
        gF = None if gF is None else gF.contiguous().double()
        gT = None if gT is None else gT.contiguous().double()
        gq, gx, gX = ctx.plan.clump_forces_backward(charges, centers, gF, gT)
        return gq, gx.to(torch.float64), gX, None


def clump_forces(charges, positions, centers, plan: Plan):
    return ClumpForcesFunction.apply(charges, positions, centers, plan)
