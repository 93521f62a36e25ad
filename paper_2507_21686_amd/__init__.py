"""Analytic SPH boundary integrals on MI355X -- Python binding.

Thin ctypes wrapper over the C-ABI of ``libsphbi.so`` (see ``include/sphbi.h``).
It only marshals torch tensors (device memory) and the current HIP stream to
the library; every step of the computation runs in the library's kernels.
There is no fallback: if the library is missing the call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

from . import workloads  # noqa: F401  (seeded input generators)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsphbi.so")

WENDLAND_C2, WENDLAND_C4, WENDLAND_C6, CUBIC_BSPLINE = 0, 1, 2, 3
FP64, MIXED = 0, 1
REFINE_AUTO, REFINE_OFF, REFINE_ALL = 0, 1, 2
STATUS = {0: "OK", -1: "EINVAL", -2: "EUNSUPPORTED", -3: "EDEVICE", -4: "ENOWORKSPACE", -5: "ECAPACITY", -6: "EGRID"}
EGRID = -6

EXPORTS = ["sphbi_kernel_preset", "sphbi_default_opts", "sphbi_last_error", "sphbi_pairlist_plan",
           "sphbi_pairlist_count", "sphbi_pairlist_recount", "sphbi_pairlist_fill", "sphbi_integrate_workspace", "sphbi_integrate",
           "sphbi_field_prepare", "sphbi_integrate_prepared", "sphbi_integrate_backward_workspace",
           "sphbi_integrate_backward", "sphbi_surrogate_features", "sphbi_surrogate_targets", "sphbi_mlp_workspace", "sphbi_mlp_forward",
           "sphbi_mlp_loss_grad", "sphbi_adam_step", "sphbi_surrogate_model_bytes", "sphbi_surrogate_pack",
           "sphbi_surrogate_workspace", "sphbi_surrogate_integrate", "sphbi_operator_workspace", "sphbi_operator",
           "sphbi_pressure_contact", "sphbi_integrate_quadrature", "sphbi_integrate_noalloc", "sphbi_probe_fp64_fma"]
MLP_PARAMS = 34692
NOALLOC_MAX_TRIANGLES = 131072


class SphbiKernel(C.Structure):
    _fields_ = [("n_pieces", C.c_int32), ("degree", C.c_int32 * 2), ("reserved", C.c_int32),
                ("radius", C.c_double * 2), ("b", (C.c_double * 12) * 2), ("c_d", C.c_double)]


class SphbiOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("refine", C.c_int32), ("tau_edge", C.c_double),
                ("refine_gate", C.c_double), ("pair_status", C.c_void_p)]


class SphbiGrid(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("cell", C.c_double), ("nx", C.c_int32),
                ("ny", C.c_int32), ("n_refs", C.c_int64)]


class SphbiError(RuntimeError):
    pass


_lib = None


def lib():
    """Load ``libsphbi.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SphbiError(f"{LIB_PATH} missing: build it with paper_2507_21686_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.sphbi_kernel_preset.argtypes = [i32, C.POINTER(SphbiKernel)]
        L.sphbi_default_opts.argtypes = [C.POINTER(SphbiOpts)]
        L.sphbi_default_opts.restype = None
        L.sphbi_last_error.restype = C.c_char_p
        L.sphbi_pairlist_plan.argtypes = [i64, vp, vp, i64, vp, d, C.POINTER(SphbiGrid), C.POINTER(C.c_size_t), vp]
        L.sphbi_pairlist_count.argtypes = [i64, vp, vp, i64, vp, d, C.POINTER(SphbiGrid), vp, C.c_size_t, vp,
                                           C.POINTER(C.c_int64), vp]
        L.sphbi_pairlist_recount.argtypes = L.sphbi_pairlist_count.argtypes
        L.sphbi_pairlist_fill.argtypes = [i64, vp, vp, i64, vp, d, C.POINTER(SphbiGrid), vp, C.c_size_t, vp, vp,
                                          i64, vp]
        L.sphbi_integrate_workspace.argtypes = [i64]
        L.sphbi_integrate_workspace.restype = C.c_size_t
        L.sphbi_integrate.argtypes = [C.POINTER(SphbiKernel), C.POINTER(SphbiOpts), d, i32, i64, vp, vp, i64, vp,
                                      vp, vp, vp, i64, vp, vp, vp, vp, vp, C.c_size_t, vp]
        L.sphbi_integrate_noalloc.argtypes = [C.POINTER(SphbiKernel), C.POINTER(SphbiOpts), d, i32, i64, vp, vp,
                                              i64, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp]
        L.sphbi_field_prepare.argtypes = [d, i32, i64, vp, vp, vp, C.c_size_t, vp]
        L.sphbi_integrate_prepared.argtypes = [C.POINTER(SphbiKernel), C.POINTER(SphbiOpts), d, i32, i64, vp, vp,
                                               i64, vp, vp, vp, i64, vp, vp, vp, vp, vp]
        L.sphbi_integrate_backward_workspace.argtypes = [i64, i64, i32]
        L.sphbi_integrate_backward_workspace.restype = C.c_size_t
        L.sphbi_integrate_backward.argtypes = [C.POINTER(SphbiKernel), C.POINTER(SphbiOpts), d, i32, i64, vp, vp,
                                               i64, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp,
                                               C.c_size_t, vp]
        L.sphbi_operator_workspace.argtypes = [i64, i64]
        L.sphbi_operator_workspace.restype = C.c_size_t
        L.sphbi_operator.argtypes = [C.POINTER(SphbiKernel), C.POINTER(SphbiOpts), i32, d, i32, i64, vp, vp, vp,
                                     vp, i64, vp, vp, vp, vp, vp, i64, vp, vp, vp, C.c_size_t, vp]
        L.sphbi_pressure_contact.argtypes = [C.POINTER(SphbiKernel), C.POINTER(SphbiOpts), d, d, i64, vp, vp, vp, vp,
                                             i64, vp, vp, vp, i64, vp, vp, vp, vp, C.c_size_t, vp]
        f = C.c_float
        L.sphbi_integrate_quadrature.argtypes = [C.POINTER(SphbiKernel), d, i32, i32, i64, vp, vp, i64, vp, vp,
                                                 vp, vp, i64, vp, vp, vp, vp]
        L.sphbi_surrogate_features.argtypes = [d, i64, vp, vp, i64, vp, vp, vp, i64, vp, vp, vp]
        L.sphbi_surrogate_targets.argtypes = [i64, d, vp, vp, C.POINTER(C.c_float), C.POINTER(C.c_float), vp, vp]
        L.sphbi_mlp_workspace.argtypes = [i64]
        L.sphbi_mlp_workspace.restype = C.c_size_t
        L.sphbi_mlp_forward.argtypes = [vp, i64, vp, vp, vp, C.c_size_t, vp]
        L.sphbi_mlp_loss_grad.argtypes = [vp, i64, vp, vp, C.POINTER(C.c_float), f, vp, vp, vp, C.c_size_t, vp]
        L.sphbi_adam_step.argtypes = [vp, vp, vp, vp, i64, d, d, d, d, i64, vp]
        L.sphbi_surrogate_model_bytes.argtypes = []
        L.sphbi_surrogate_model_bytes.restype = C.c_size_t
        L.sphbi_surrogate_pack.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_float), f, vp, vp]
        L.sphbi_surrogate_workspace.argtypes = [i64, i64]
        L.sphbi_surrogate_workspace.restype = C.c_size_t
        L.sphbi_surrogate_integrate.argtypes = [C.POINTER(SphbiKernel), d, i64, vp, vp, i64, vp, vp, vp, vp, i64,
                                                vp, f, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]
        L.sphbi_probe_fp64_fma.argtypes = [i64, vp, C.POINTER(C.c_double), vp]
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        msg = lib().sphbi_last_error().decode()
        raise SphbiError(f"{what} failed: {STATUS.get(rc, rc)}: {msg}")


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(None)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype=torch.float64):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise SphbiError(f"expected a contiguous {dtype} tensor on the GPU")
    return t


def kernel_preset(kernel_id: int) -> SphbiKernel:
    k = SphbiKernel()
    _check(lib().sphbi_kernel_preset(int(kernel_id), C.byref(k)), "sphbi_kernel_preset")
    return k


def opts(precision: int = FP64, tau_edge: float = 1e-4, refine: int = REFINE_AUTO,
         refine_gate: float = 0.0) -> SphbiOpts:
    o = SphbiOpts()
    lib().sphbi_default_opts(C.byref(o))
    o.precision = precision
    o.tau_edge = tau_edge
    o.refine = refine
    o.refine_gate = refine_gate
    return o


def pairlist(px, py, tri, h: float):
    """Pairs with dist(x_i, T_j) < h as CSR: (offsets int64 [N+1], tri_idx int32 [P])."""
    px, py, tri = _dev(px), _dev(py), _dev(tri)
    N, T = px.numel(), tri.shape[1]
    L, s = lib(), _stream()
    grid = SphbiGrid()
    ws_bytes = C.c_size_t(0)
    _check(L.sphbi_pairlist_plan(N, _ptr(px), _ptr(py), T, _ptr(tri), float(h), C.byref(grid), C.byref(ws_bytes), s),
           "sphbi_pairlist_plan")
    ws = torch.empty(max(int(ws_bytes.value), 1), dtype=torch.uint8, device=px.device)
    offsets = torch.empty(N + 1, dtype=torch.int64, device=px.device)
    n = C.c_int64(0)
    _check(L.sphbi_pairlist_count(N, _ptr(px), _ptr(py), T, _ptr(tri), float(h), C.byref(grid), _ptr(ws),
                                  ws.numel(), _ptr(offsets), C.byref(n), s), "sphbi_pairlist_count")
    tri_idx = torch.empty(max(int(n.value), 1), dtype=torch.int32, device=px.device)
    _check(L.sphbi_pairlist_fill(N, _ptr(px), _ptr(py), T, _ptr(tri), float(h), C.byref(grid), _ptr(ws), ws.numel(),
                                 _ptr(offsets), _ptr(tri_idx), int(n.value), s), "sphbi_pairlist_fill")
    return offsets, tri_idx[: int(n.value)]


class PairList:
    """Pair lists of a mesh that does not move, for particles that do.

    Keeps the cell grid and its triangle lists between calls and only counts
    and fills the pairs again (``sphbi_pairlist_recount``); the grid is
    planned again, over the particles' bounding box grown by ``pad`` on every
    side, when a particle has left it or N has grown.  ``tri`` must not change
    while the object is in use.  The lists are identical to ``pairlist``'s
    (the pair tests do not depend on the grid).
    """

    def __init__(self, tri, h: float, pad: float | None = None):
        self.tri = _dev(tri)
        self.h = float(h)
        self.pad = 2.0 * self.h if pad is None else float(pad)
        self.grid = None
        self.ws = None
        self.n_plan = 0       # particles the workspace was sized for
        self.plans = self.reuses = 0

    def _plan_on(self, px, py):
        grid, ws_bytes = SphbiGrid(), C.c_size_t(0)
        _check(lib().sphbi_pairlist_plan(px.numel(), _ptr(px), _ptr(py), self.tri.shape[1], _ptr(self.tri), self.h,
                                         C.byref(grid), C.byref(ws_bytes), _stream()), "sphbi_pairlist_plan")
        return grid, ws_bytes

    def _plan(self, px, py):
        grid, ws_bytes = self._plan_on(px, py)
        if self.pad > 0.0 and px.numel() > 0:
            # plan again with two corner points that grow the particles' box
            # (x0, y0 is its low corner, the cells reach past its high one)
            g = grid
            cx = torch.tensor([g.x0 - self.pad, g.x0 + g.nx * g.cell + self.pad], dtype=torch.float64)
            cy = torch.tensor([g.y0 - self.pad, g.y0 + g.ny * g.cell + self.pad], dtype=torch.float64)
            qx = torch.cat([px, cx.to(px.device)])
            qy = torch.cat([py, cy.to(py.device)])
            grid, ws_bytes = self._plan_on(qx, qy)
        self.grid = grid
        self.ws = torch.empty(max(int(ws_bytes.value), 1), dtype=torch.uint8, device=px.device)
        self.n_plan = px.numel()
        self.plans += 1

    def __call__(self, px, py):
        """(offsets int64 [N+1], tri_idx int32 [P]) for the current positions."""
        px, py = _dev(px), _dev(py)
        N, T = px.numel(), self.tri.shape[1]
        L, s = lib(), _stream()
        offsets = torch.empty(N + 1, dtype=torch.int64, device=px.device)
        n = C.c_int64(0)
        rc = EGRID
        if self.grid is not None and N <= self.n_plan:
            rc = L.sphbi_pairlist_recount(N, _ptr(px), _ptr(py), T, _ptr(self.tri), self.h, C.byref(self.grid),
                                          _ptr(self.ws), self.ws.numel(), _ptr(offsets), C.byref(n), s)
            if rc == 0:
                self.reuses += 1
            elif rc != EGRID:
                _check(rc, "sphbi_pairlist_recount")
        if rc == EGRID:
            self._plan(px, py)
            _check(L.sphbi_pairlist_count(N, _ptr(px), _ptr(py), T, _ptr(self.tri), self.h, C.byref(self.grid),
                                          _ptr(self.ws), self.ws.numel(), _ptr(offsets), C.byref(n), s),
                   "sphbi_pairlist_count")
        tri_idx = torch.empty(max(int(n.value), 1), dtype=torch.int32, device=px.device)
        _check(L.sphbi_pairlist_fill(N, _ptr(px), _ptr(py), T, _ptr(self.tri), self.h, C.byref(self.grid),
                                     _ptr(self.ws), self.ws.numel(), _ptr(offsets), _ptr(tri_idx), int(n.value), s),
               "sphbi_pairlist_fill")
        return offsets, tri_idx[: int(n.value)]


class Integrator:
    """Holds the kernel description and a reusable workspace for repeated calls."""

    def __init__(self, kernel, h: float, n_nodes: int, precision: int = FP64, tau_edge: float = 1e-4,
                 refine: int = REFINE_AUTO, refine_gate: float = 0.0):
        self.kernel = kernel_preset(kernel) if isinstance(kernel, int) else kernel
        self.h = float(h)
        self.n_nodes = int(n_nodes)
        self.opts = opts(precision, tau_edge, refine, refine_gate)
        self.ws = None

    def workspace(self, T, device):
        need = int(lib().sphbi_integrate_workspace(T))
        if self.ws is None or self.ws.numel() < need or self.ws.device != device:
            self.ws = torch.empty(need, dtype=torch.uint8, device=device)
        return self.ws

    def prepare(self, tri, nodal):
        """Per-triangle field records (the first stage); returns the record buffer."""
        tri, nodal = _dev(tri), _dev(nodal)
        T = tri.shape[1]
        if nodal.shape[0] != self.n_nodes or nodal.shape[1] != T:
            raise SphbiError("nodal must be [n_nodes, T]")
        ws = self.workspace(T, tri.device)
        _check(lib().sphbi_field_prepare(self.h, self.n_nodes, T, _ptr(tri), _ptr(nodal), _ptr(ws), ws.numel(),
                                         _stream()), "sphbi_field_prepare")
        return ws

    def integrate_prepared(self, px, py, T, rec, offsets, tri_idx, per_pair: bool = False, out=None):
        """Pair kernel on records from :meth:`prepare` (the second stage)."""
        px, py = _dev(px), _dev(py)
        offsets, tri_idx = _dev(offsets, torch.int64), _dev(tri_idx, torch.int32)
        N, P = px.numel(), tri_idx.numel()
        if out is None:
            I = torch.empty(N, dtype=torch.float64, device=px.device)
            Gx = torch.empty_like(I)
            Gy = torch.empty_like(I)
        else:
            I, Gx, Gy = out
        pp = torch.empty((3, P), dtype=torch.float64, device=px.device) if per_pair else None
        _check(lib().sphbi_integrate_prepared(C.byref(self.kernel), C.byref(self.opts), self.h, self.n_nodes, N,
                                              _ptr(px), _ptr(py), int(T), _ptr(rec), _ptr(offsets), _ptr(tri_idx), P,
                                              _ptr(I), _ptr(Gx), _ptr(Gy), _ptr(pp), _stream()),
               "sphbi_integrate_prepared")
        return (I, Gx, Gy, pp) if per_pair else (I, Gx, Gy)

    def __call__(self, px, py, tri, nodal, offsets, tri_idx, per_pair: bool = False, out=None, status=None):
        """sphbi_integrate; status: optional uint8 device tensor [P] receiving
        the per-pair non-finite flags."""
        px, py, tri, nodal = _dev(px), _dev(py), _dev(tri), _dev(nodal)
        offsets, tri_idx = _dev(offsets, torch.int64), _dev(tri_idx, torch.int32)
        N, T, P = px.numel(), tri.shape[1], tri_idx.numel()
        if nodal.shape[0] != self.n_nodes or nodal.shape[1] != T:
            raise SphbiError("nodal must be [n_nodes, T]")
        if out is None:
            I = torch.empty(N, dtype=torch.float64, device=px.device)
            Gx = torch.empty_like(I)
            Gy = torch.empty_like(I)
        else:
            I, Gx, Gy = out
        pp = torch.empty((3, P), dtype=torch.float64, device=px.device) if per_pair else None
        ws = self.workspace(T, px.device)
        o = SphbiOpts.from_buffer_copy(self.opts)
        if status is not None:
            status = _dev(status, torch.uint8)
            if status.numel() < P:
                raise SphbiError("status must have one entry per pair")
            o.pair_status = _ptr(status)
        _check(lib().sphbi_integrate(C.byref(self.kernel), C.byref(o), self.h, self.n_nodes, N, _ptr(px),
                                     _ptr(py), T, _ptr(tri), _ptr(nodal), _ptr(offsets), _ptr(tri_idx), P, _ptr(I),
                                     _ptr(Gx), _ptr(Gy), _ptr(pp), _ptr(ws), ws.numel(), _stream()),
               "sphbi_integrate")
        return (I, Gx, Gy, pp) if per_pair else (I, Gx, Gy)


def integrate_noalloc(kernel, h, px, py, tri, nodal, offsets, tri_idx, out, per_pair=None, precision=FP64,
                      tau_edge=1e-4, refine=REFINE_AUTO, refine_gate=0.0):
    """``sphbi_integrate_noalloc``: :func:`integrate` into caller-provided outputs.

    ``out`` = (I, Gx, Gy) float64 [N] device tensors; ``per_pair`` an optional
    [3, P] tensor.  The library allocates nothing (its records live in a fixed
    per-GPU array of NOALLOC_MAX_TRIANGLES triangles); this wrapper allocates
    nothing either.
    """
    k = kernel_preset(kernel) if isinstance(kernel, int) else kernel
    px, py, tri, nodal = _dev(px), _dev(py), _dev(tri), _dev(nodal)
    offsets, tri_idx = _dev(offsets, torch.int64), _dev(tri_idx, torch.int32)
    I, Gx, Gy = (_dev(t) for t in out)
    N, T, P, nn = px.numel(), tri.shape[1], tri_idx.numel(), nodal.shape[0]
    if nodal.shape[1] != T:
        raise SphbiError("nodal must be [n_nodes, T]")
    if I.numel() != N or Gx.numel() != N or Gy.numel() != N:
        raise SphbiError("outputs must be [N]")
    if per_pair is not None and (_dev(per_pair).shape != (3, P)):
        raise SphbiError("per_pair must be [3, P]")
    o = opts(precision, tau_edge, refine, refine_gate)
    _check(lib().sphbi_integrate_noalloc(C.byref(k), C.byref(o), float(h), nn, N, _ptr(px), _ptr(py), T, _ptr(tri),
                                         _ptr(nodal), _ptr(offsets), _ptr(tri_idx), P, _ptr(I), _ptr(Gx), _ptr(Gy),
                                         _ptr(per_pair), _stream()), "sphbi_integrate_noalloc")
    return I, Gx, Gy


def integrate_backward(kernel, h, px, py, tri, nodal, offsets, tri_idx, gI, gGx, gGy, precision=FP64,
                       tau_edge=1e-4):
    """Vector-Jacobian product of :func:`integrate`: (dpx, dpy, dtri [6,T], dnodal [n_nodes,T]).

    precision: FP64, or MIXED (square roots, reciprocals and, for constant and
    linear fields, the sector angles on the FP32 units; FP64 within tau_edge*h
    of an edge line)."""
    k = kernel_preset(kernel) if isinstance(kernel, int) else kernel
    px, py, tri, nodal = _dev(px), _dev(py), _dev(tri), _dev(nodal)
    gI, gGx, gGy = _dev(gI), _dev(gGx), _dev(gGy)
    offsets, tri_idx = _dev(offsets, torch.int64), _dev(tri_idx, torch.int32)
    N, T, P, nn = px.numel(), tri.shape[1], tri_idx.numel(), nodal.shape[0]
    dpx = torch.empty_like(px)
    dpy = torch.empty_like(py)
    dtri = torch.empty_like(tri)
    dnod = torch.empty_like(nodal)
    need = int(lib().sphbi_integrate_backward_workspace(T, P, nn))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=px.device)
    o = opts(precision, tau_edge)
    _check(lib().sphbi_integrate_backward(C.byref(k), C.byref(o), float(h), nn, N, _ptr(px), _ptr(py), T, _ptr(tri),
                                          _ptr(nodal), _ptr(offsets), _ptr(tri_idx), P, _ptr(gI), _ptr(gGx),
                                          _ptr(gGy), _ptr(dpx), _ptr(dpy), _ptr(dtri), _ptr(dnod), _ptr(ws),
                                          ws.numel(), _stream()), "sphbi_integrate_backward")
    return dpx, dpy, dtri, dnod


class BoundaryIntegral(torch.autograd.Function):
    """(I, Gx, Gy) = boundary integrals with gradients for px, py, tri and nodal.

    forward(px, py, tri, nodal, offsets, tri_idx, kernel, h, precision=FP64); the
    pair list is treated as constant (it changes only where the kernel
    vanishes).  The backward pass runs in the forward pass's precision mode.
    """

    @staticmethod
    def forward(ctx, px, py, tri, nodal, offsets, tri_idx, kernel, h, precision=FP64):
        ctx.save_for_backward(px, py, tri, nodal, offsets, tri_idx)
        ctx.kernel, ctx.h, ctx.precision = kernel, h, precision
        return integrate(kernel, h, px, py, tri, nodal, offsets, tri_idx, precision=precision)

    @staticmethod
    def backward(ctx, gI, gGx, gGy):
        px, py, tri, nodal, offsets, tri_idx = ctx.saved_tensors
        z = torch.zeros_like(px)
        gI = z if gI is None else gI.contiguous()
        gGx = z if gGx is None else gGx.contiguous()
        gGy = z if gGy is None else gGy.contiguous()
        dpx, dpy, dtri, dnod = integrate_backward(ctx.kernel, ctx.h, px, py, tri, nodal, offsets, tri_idx,
                                                  gI, gGx, gGy, precision=ctx.precision)
        return dpx, dpy, dtri, dnod, None, None, None, None, None


def integrate(kernel, h, px, py, tri, nodal, offsets, tri_idx, per_pair=False, precision=FP64, tau_edge=1e-4,
              refine=REFINE_AUTO, refine_gate=0.0, status=None):
    """Per-particle (I, Gx, Gy) [N] (and optionally per-pair [3, P]) on the GPU;
    status: optional uint8 tensor [P] for the per-pair non-finite flags."""
    return Integrator(kernel, h, nodal.shape[0], precision, tau_edge, refine, refine_gate)(
        px, py, tri, nodal, offsets, tri_idx, per_pair=per_pair, status=status)


# ----------------------------------------------------------------------------
# SPH operators on the boundary (Sec. 2) and the boundary normal (App. A)
# ----------------------------------------------------------------------------
OP_GRAD_DIFFERENCE, OP_GRAD_SYMMETRIC, OP_DIV_CURL, OP_NORMAL = 0, 1, 2, 3


def operator(op, kernel, h, px, py, tri, offsets, tri_idx, fa=None, fb=None, qa=None, qb=None, ws=None):
    """``sphbi_operator``: two per-particle outputs [N] of operator ``op``.

    OP_GRAD_DIFFERENCE / OP_GRAD_SYMMETRIC: fa = A, fb = rho nodal [n_nodes, T],
    qa = A(x), qb = rho(x) [N] -> (d/dx, d/dy); OP_DIV_CURL: fa = A_x, fb = A_y
    -> (div, curl); OP_NORMAL: -> int grad W.  ``ws``: optional uint8 device
    workspace of at least ``sphbi_operator_workspace(N, T)`` bytes.
    """
    k = kernel_preset(kernel) if isinstance(kernel, int) else kernel
    px, py, tri = _dev(px), _dev(py), _dev(tri)
    offsets, tri_idx = _dev(offsets, torch.int64), _dev(tri_idx, torch.int32)
    N, T, P = px.numel(), tri.shape[1], tri_idx.numel()
    nn = 1
    if op != OP_NORMAL:
        fa, fb = _dev(fa), _dev(fb)
        nn = fa.shape[0]
        if fa.shape != (nn, T) or fb.shape != (nn, T):
            raise SphbiError("fa, fb must both be [n_nodes, T]")
    if op in (OP_GRAD_DIFFERENCE, OP_GRAD_SYMMETRIC):
        qa, qb = _dev(qa), _dev(qb)
        if qa.numel() != N or qb.numel() != N:
            raise SphbiError("qa, qb must be [N]")
    out_a = torch.empty(N, dtype=torch.float64, device=px.device)
    out_b = torch.empty_like(out_a)
    if ws is None or ws.numel() < int(lib().sphbi_operator_workspace(N, T)):
        ws = torch.empty(int(lib().sphbi_operator_workspace(N, T)), dtype=torch.uint8, device=px.device)
    o = opts(FP64)
    _check(lib().sphbi_operator(C.byref(k), C.byref(o), int(op), float(h), nn, N, _ptr(px), _ptr(py), _ptr(qa),
                                _ptr(qb), T, _ptr(tri), _ptr(fa), _ptr(fb), _ptr(offsets), _ptr(tri_idx), P,
                                _ptr(out_a), _ptr(out_b), _ptr(ws), ws.numel(), _stream()), "sphbi_operator")
    return out_a, out_b


def gradient_difference(kernel, h, px, py, A_p, rho_p, tri, A, rho, offsets, tri_idx):
    """(1/rho(x)) int rho (A - A(x)) grad W with per-node pre-weights (Sec. 2)."""
    return operator(OP_GRAD_DIFFERENCE, kernel, h, px, py, tri, offsets, tri_idx, A, rho, A_p, rho_p)


def gradient_symmetric(kernel, h, px, py, A_p, rho_p, tri, A, rho, offsets, tri_idx):
    """rho(x) int rho (A/rho^2 + A(x)/rho(x)^2) grad W with per-node pre-weights (Sec. 2)."""
    return operator(OP_GRAD_SYMMETRIC, kernel, h, px, py, tri, offsets, tri_idx, A, rho, A_p, rho_p)


def divergence_curl(kernel, h, px, py, tri, Ax, Ay, offsets, tri_idx):
    """(div, curl) of the boundary vector field (Ax, Ay) (Sec. 2)."""
    return operator(OP_DIV_CURL, kernel, h, px, py, tri, offsets, tri_idx, Ax, Ay)


def boundary_normal(kernel, h, px, py, tri, offsets, tri_idx):
    """int grad W over the boundary, per particle (App. A)."""
    return operator(OP_NORMAL, kernel, h, px, py, tri, offsets, tri_idx)


def pressure_contact(kernel, h, rho0, px, py, p_particle, rho_particle, tri, offsets, tri_idx, p_pair, ws=None):
    """Boundary pressure acceleration (ax, ay) [N] with one pressure per contact (App. A):
    -sum_q rho0 (p_q/rho0^2 + p_i/rho_i^2) int_T grad W; p_pair [n_pairs] in tri_idx order."""
    k = kernel_preset(kernel) if isinstance(kernel, int) else kernel
    px, py, tri = _dev(px), _dev(py), _dev(tri)
    p_particle, rho_particle, p_pair = _dev(p_particle), _dev(rho_particle), _dev(p_pair)
    offsets, tri_idx = _dev(offsets, torch.int64), _dev(tri_idx, torch.int32)
    N, T, P = px.numel(), tri.shape[1], tri_idx.numel()
    if p_pair.numel() != P or p_particle.numel() != N or rho_particle.numel() != N:
        raise SphbiError("p_pair must be [n_pairs], p_particle and rho_particle [N]")
    ax = torch.empty(N, dtype=torch.float64, device=px.device)
    ay = torch.empty_like(ax)
    need = int(lib().sphbi_operator_workspace(N, T))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=px.device)
    o = opts(FP64)
    _check(lib().sphbi_pressure_contact(C.byref(k), C.byref(o), float(h), float(rho0), N, _ptr(px), _ptr(py),
                                        _ptr(p_particle), _ptr(rho_particle), T, _ptr(tri), _ptr(offsets),
                                        _ptr(tri_idx), P, _ptr(p_pair), _ptr(ax), _ptr(ay), _ptr(ws), ws.numel(),
                                        _stream()), "sphbi_pressure_contact")
    return ax, ay


# ----------------------------------------------------------------------------
# quadrature of the same sums (the comparison of Sec. 6.1-6.2)
# ----------------------------------------------------------------------------
MAX_GAUSS = 64


def probe_fp64_fma(iters: int, sink):
    """``sphbi_probe_fp64_fma``: launches the FP64 FMA probe on the current
    stream and returns the FP64 operations it executes (time it to get the
    device's FP64 vector rate).  sink: a one-element float64 device tensor."""
    sink = _dev(sink)
    flops = C.c_double(0.0)
    _check(lib().sphbi_probe_fp64_fma(int(iters), _ptr(sink), C.byref(flops), _stream()), "sphbi_probe_fp64_fma")
    return flops.value


def integrate_quadrature(kernel, h, px, py, tri, nodal, offsets, tri_idx, n_gauss):
    """``sphbi_integrate_quadrature``: per-particle (I, Gx, Gy) [N] with an
    n_gauss x n_gauss collapsed Gauss-Legendre rule per pair."""
    k = kernel_preset(kernel) if isinstance(kernel, int) else kernel
    px, py, tri, nodal = _dev(px), _dev(py), _dev(tri), _dev(nodal)
    offsets, tri_idx = _dev(offsets, torch.int64), _dev(tri_idx, torch.int32)
    N, T, P = px.numel(), tri.shape[1], tri_idx.numel()
    if nodal.shape[-1] != T or offsets.numel() != N + 1:
        raise SphbiError("nodal must be [n_nodes, T] and offsets [N + 1]")
    I = torch.empty(N, dtype=torch.float64, device=px.device)
    Gx, Gy = torch.empty_like(I), torch.empty_like(I)
    _check(lib().sphbi_integrate_quadrature(C.byref(k), float(h), int(nodal.shape[0]), int(n_gauss), N, _ptr(px),
                                            _ptr(py), T, _ptr(tri), _ptr(nodal), _ptr(offsets), _ptr(tri_idx), P,
                                            _ptr(I), _ptr(Gx), _ptr(Gy), _stream()), "sphbi_integrate_quadrature")
    return I, Gx, Gy


# ----------------------------------------------------------------------------
# learned surrogate (C-ABI wrappers; the training loop is in surrogate.py)
# ----------------------------------------------------------------------------
def _f32(t):
    return _dev(t, torch.float32)


def surrogate_features(px, py, tri, h, offsets, tri_idx):
    """Canonical pair features (float32 [P, 8]) and frame rotations (float32 [P, 2])."""
    px, py, tri = _dev(px), _dev(py), _dev(tri)
    offsets, tri_idx = _dev(offsets, torch.int64), _dev(tri_idx, torch.int32)
    N, T, P = px.numel(), tri.shape[1], tri_idx.numel()
    feats = torch.empty((P, 8), dtype=torch.float32, device=px.device)
    rot = torch.empty((P, 2), dtype=torch.float32, device=px.device)
    _check(lib().sphbi_surrogate_features(float(h), N, _ptr(px), _ptr(py), T, _ptr(tri), _ptr(offsets),
                                          _ptr(tri_idx), P, _ptr(feats), _ptr(rot), _stream()),
           "sphbi_surrogate_features")
    return feats, rot


def surrogate_targets(per_pair, rot, h, mean=(0.0, 0.0, 0.0), stdev=(1.0, 1.0, 1.0)):
    """Standardised targets float32 [P, 3] in the rotated frame from per-pair values [3, P]."""
    per_pair, rot = _dev(per_pair), _f32(rot)
    P = per_pair.shape[1]
    out = torch.empty((P, 3), dtype=torch.float32, device=per_pair.device)
    m = (C.c_float * 3)(*[float(x) for x in mean])
    sd = (C.c_float * 3)(*[float(x) for x in stdev])
    _check(lib().sphbi_surrogate_targets(P, float(h), _ptr(per_pair), _ptr(rot), m, sd, _ptr(out), _stream()),
           "sphbi_surrogate_targets")
    return out


class MLPWorkspace:
    """Device workspace of the training calls for batches of up to B rows."""

    def __init__(self, B, device="cuda:0"):
        self.B = int(B)
        self.buf = torch.empty(max(int(lib().sphbi_mlp_workspace(self.B)), 1), dtype=torch.uint8, device=device)

    def fits(self, B):
        return B <= self.B


def mlp_forward(params, feats, ws=None):
    """Network outputs float32 [B, 4] for features float32 [B, 8]."""
    params, feats = _f32(params), _f32(feats)
    B = feats.shape[0]
    ws = ws if ws is not None and ws.fits(B) else MLPWorkspace(B, feats.device)
    out = torch.empty((B, 4), dtype=torch.float32, device=feats.device)
    _check(lib().sphbi_mlp_forward(_ptr(params), B, _ptr(feats), _ptr(out), _ptr(ws.buf), ws.buf.numel(), _stream()),
           "sphbi_mlp_forward")
    return out


def mlp_loss_grad(params, feats, targets, scale, lam, ws=None, grad=None, loss=None):
    """(loss float32 [1], grad float32 [MLP_PARAMS]) of one batch (see include/sphbi.h)."""
    params, feats, targets = _f32(params), _f32(feats), _f32(targets)
    B = feats.shape[0]
    ws = ws if ws is not None and ws.fits(B) else MLPWorkspace(B, feats.device)
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=feats.device) if grad is None else grad
    loss = torch.empty(1, dtype=torch.float32, device=feats.device) if loss is None else loss
    sc = (C.c_float * 3)(*[float(x) for x in scale])
    _check(lib().sphbi_mlp_loss_grad(_ptr(params), B, _ptr(feats), _ptr(targets), sc, float(lam), _ptr(loss),
                                     _ptr(grad), _ptr(ws.buf), ws.buf.numel(), _stream()), "sphbi_mlp_loss_grad")
    return loss, grad


def adam_step(params, m, v, grad, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One in-place Adam update of params (and the moments m, v)."""
    for t in (params, m, v, grad):
        _f32(t)
    _check(lib().sphbi_adam_step(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), params.numel(), float(lr), float(beta1),
                                 float(beta2), float(eps), int(step), _stream()), "sphbi_adam_step")


def surrogate_pack(params, mean, stdev, fmax):
    """Serving model (device uint8 buffer) from FP32 parameters and output statistics."""
    params = _f32(params)
    model = torch.empty(int(lib().sphbi_surrogate_model_bytes()), dtype=torch.uint8, device=params.device)
    m = (C.c_float * 3)(*[float(x) for x in mean])
    sd = (C.c_float * 3)(*[float(x) for x in stdev])
    _check(lib().sphbi_surrogate_pack(_ptr(params), m, sd, float(fmax), _ptr(model), _stream()),
           "sphbi_surrogate_pack")
    return model


def surrogate_integrate(kernel, h, px, py, tri, nodal, offsets, tri_idx, model, threshold, per_pair=False, ws=None):
    """Per-particle integrals of a P0 field with the surrogate and the analytic fallback.

    Returns (I, Gx, Gy, per_pair or None, flags uint8 [P], n_flagged int64 [1] on the device).
    """
    px, py, tri, nodal = _dev(px), _dev(py), _dev(tri), _dev(nodal)
    offsets, tri_idx = _dev(offsets, torch.int64), _dev(tri_idx, torch.int32)
    N, T, P = px.numel(), tri.shape[1], tri_idx.numel()
    k = kernel if isinstance(kernel, SphbiKernel) else kernel_preset(kernel)
    need = int(lib().sphbi_surrogate_workspace(T, P))
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=px.device)
    dev = px.device
    I = torch.empty(N, dtype=torch.float64, device=dev)
    Gx = torch.empty(N, dtype=torch.float64, device=dev)
    Gy = torch.empty(N, dtype=torch.float64, device=dev)
    pp = torch.empty((3, P), dtype=torch.float64, device=dev) if per_pair else None
    flags = torch.empty(max(P, 1), dtype=torch.uint8, device=dev)
    nf = torch.zeros(1, dtype=torch.int64, device=dev)
    _check(lib().sphbi_surrogate_integrate(C.byref(k), float(h), N, _ptr(px), _ptr(py), T, _ptr(tri), _ptr(nodal),
                                           _ptr(offsets), _ptr(tri_idx), P, _ptr(model), float(threshold), _ptr(I),
                                           _ptr(Gx), _ptr(Gy), _ptr(pp), _ptr(flags), _ptr(nf), _ptr(ws), ws.numel(),
                                           _stream()), "sphbi_surrogate_integrate")
    return I, Gx, Gy, pp, flags[:P], nf
