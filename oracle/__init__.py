"""CPU oracle for the SPH boundary integrals -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The device library never links or
calls it, and it shares no source with the device library.

``definition.c``  plain FP64 evaluation of the integrals from their
                  definition (Sec. 2 eq. boundaryint / nablaIntegral) by
                  polar quadrature with an exact radial rule.
``closed_form.c`` the paper's decomposition (Sec. 4, Alg. 1-5, T2/T3) and
                  closed forms (Sec. 5) in plain FP64.

Both are compiled with gcc into ``oracle/liboracle.so`` by :func:`build`.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["definition.c", "closed_form.c"]
OPCOUNT_LIB = os.path.join(HERE, "liboracle_opcount.so")

_lib = None


class OracleCapped(ValueError):
    """The definition oracle's adaptive rule stopped at its depth or call cap."""


def build(force: bool = True) -> str:
    """Compile the oracle sources with gcc (OpenMP) into ``oracle/liboracle.so``."""
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    # the operation-counting build of the closed-form oracle (C++), with the
    # definition oracle's kernel tables
    obj = OPCOUNT_LIB + ".def.o"
    subprocess.run(["gcc", "-O2", "-fPIC", "-std=c11", "-c", os.path.join(HERE, "definition.c"), "-o", obj],
                   check=True)
    tmp = OPCOUNT_LIB + ".tmp"
    subprocess.run(["g++", "-O2", "-fPIC", "-shared", "-std=c++17", "-o", tmp, os.path.join(HERE, "opcount.cpp"), obj,
                    "-lm"], check=True)
    os.remove(obj)
    os.replace(tmp, OPCOUNT_LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        d, i64, i32, vp = C.c_double, C.c_int64, C.c_int32, C.c_void_p
        L.oracle_pair.argtypes = [C.c_int, d, C.c_int, d, d, vp, vp, vp]
        L.oracle_pair.restype = C.c_int
        L.oracle_integrate.argtypes = [C.c_int, d, C.c_int, i64, vp, vp, i64, vp, vp, vp, vp,
                                       vp, vp, vp, vp, C.c_int]
        L.oracle_integrate.restype = C.c_int
        L.oracle_pairlist.argtypes = [i64, vp, vp, i64, vp, d, vp, vp, C.c_int]
        L.oracle_pairlist.restype = i64
        L.oracle_kernel_monomials.argtypes = [C.c_int, vp, vp, vp, vp, vp]
        L.oracle_kernel_monomials.restype = C.c_int
        L.oracle_point_triangle_dist2.argtypes = [d, d, vp]
        L.oracle_point_triangle_dist2.restype = d
        if hasattr(L, "oracle_cf_pair"):
            L.oracle_cf_pair.argtypes = [C.c_int, d, C.c_int, d, d, vp, vp, vp]
            L.oracle_cf_pair.restype = C.c_int
            L.oracle_cf_integrate.argtypes = L.oracle_integrate.argtypes
            L.oracle_cf_integrate.restype = C.c_int
            L.oracle_cf_radial.argtypes = [C.c_int, C.c_int, d, d, d]
            L.oracle_cf_radial.restype = d
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def kernel_monomials(kernel_id: int):
    """(n_pieces, radii[2], degrees[2], b[2,12], C_d) of a preset kernel."""
    n = np.zeros(1, np.int32)
    R = np.zeros(2)
    deg = np.zeros(2, np.int32)
    b = np.zeros((2, 12))
    cd = np.zeros(1)
    rc = lib().oracle_kernel_monomials(kernel_id, _p(n), _p(R), _p(deg), _p(b), _p(cd))
    if rc:
        raise ValueError("unknown kernel")
    return int(n[0]), R, deg, b, float(cd[0])


def pair(kernel_id, h, px, py, tri6, A, method="definition"):
    """(I, Gx, Gy) of one particle/triangle pair in world coordinates."""
    tri6 = _f64(tri6).reshape(6)
    A = _f64(np.atleast_1d(A))
    out = np.zeros(3)
    fn = lib().oracle_pair if method == "definition" else lib().oracle_cf_pair
    rc = fn(int(kernel_id), float(h), int(A.shape[0]), float(px), float(py), _p(tri6), _p(A), _p(out))
    if rc > 0 and method == "definition":
        raise OracleCapped("the adaptive rule reached its depth or call cap: the pair is unverified")
    if rc < 0:
        raise ValueError(f"oracle pair failed ({rc})")
    return out


def pairs_normalised(kernel_id, tri, A, method="definition"):
    """Vectorised :func:`pair` for triangles [6, n] already in the unit-support frame."""
    tri = _f64(tri)
    A = _f64(A)
    n = tri.shape[1]
    out = np.zeros((3, n))
    for k in range(n):
        out[:, k] = pair(kernel_id, 1.0, 0.0, 0.0, tri[:, k], A[:, k], method)
    return out


def integrate(kernel_id, h, px, py, tri, nodal, offsets, tri_idx, per_pair=False,
              nthreads=0, method="definition"):
    """Per-particle (I, Gx, Gy) over a CSR pair list; optionally per-pair [3, P]."""
    px, py, tri, nodal = _f64(px), _f64(py), _f64(tri), _f64(nodal)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    tri_idx = np.ascontiguousarray(tri_idx, dtype=np.int32)
    N = px.shape[0]
    T = tri.shape[1]
    P = int(offsets[-1]) if N else 0
    I = np.zeros(N); Gx = np.zeros(N); Gy = np.zeros(N)
    pp = np.zeros((3, P)) if per_pair else None
    fn = lib().oracle_integrate if method == "definition" else lib().oracle_cf_integrate
    rc = fn(int(kernel_id), float(h), int(nodal.shape[0]), N, _p(px), _p(py), T, _p(tri), _p(nodal),
            _p(offsets), _p(tri_idx), _p(I), _p(Gx), _p(Gy), _p(pp) if pp is not None else None,
            int(nthreads))
    if rc > 0 and method == "definition":
        raise OracleCapped(f"the adaptive rule reached its depth or call cap on {rc} pairs: unverified")
    if rc < 0:
        raise ValueError(f"oracle integrate failed ({rc})")
    return (I, Gx, Gy, pp) if per_pair else (I, Gx, Gy)


_opc = None
OPCOUNT_KINDS = ("add", "mul", "div", "sqrt", "transcendental")


def opcount_pairs(kernel_id, tri, A):
    """Operation counts of the paper's closed form (closed_form.c) per pair.

    tri [6, n] in the support-normalised frame, A [n_nodes, n].  Returns
    (counts int64 [n, 5] in the order of OPCOUNT_KINDS, case int [n] = number
    of vertices inside the support, out [3, n] = the counted evaluation)."""
    global _opc
    if _opc is None:
        if not os.path.exists(OPCOUNT_LIB):
            build()
        _opc = C.CDLL(OPCOUNT_LIB)
        _opc.oracle_opcount_pair.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                             C.c_void_p]
    tri, A = _f64(tri), _f64(A)
    n = tri.shape[1]
    counts = np.zeros((n, 5), np.int64)
    cls = np.zeros(n, np.int32)
    out = np.zeros((3, n))
    t6 = np.zeros(6)
    a = np.zeros(10)
    o = np.zeros(3)
    c = np.zeros(5, np.int64)
    k = np.zeros(1, np.int32)
    for j in range(n):
        t6[:] = tri[:, j]
        a[:A.shape[0]] = A[:, j]
        _opc.oracle_opcount_pair(int(kernel_id), int(A.shape[0]), _p(t6), _p(a), _p(o), _p(c), _p(k))
        counts[j] = c
        cls[j] = k[0]
        out[:, j] = o
    return counts, cls, out


def pairlist(px, py, tri, h, nthreads=0):
    """Brute-force CSR (offsets [N+1] int64, tri_idx [P] int32) of dist(x_i, T_j) < h."""
    px, py, tri = _f64(px), _f64(py), _f64(tri)
    N = px.shape[0]
    T = tri.shape[1]
    off = np.zeros(N + 1, np.int64)
    P = lib().oracle_pairlist(N, _p(px), _p(py), T, _p(tri), float(h), _p(off), None, int(nthreads))
    idx = np.zeros(max(P, 1), np.int32)
    lib().oracle_pairlist(N, _p(px), _p(py), T, _p(tri), float(h), _p(off), _p(idx), int(nthreads))
    return off, idx[:P]


def point_triangle_dist2(px, py, tri6):
    t = _f64(tri6).reshape(6)
    return lib().oracle_point_triangle_dist2(float(px), float(py), _p(t))
