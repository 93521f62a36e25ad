"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every function declared in include/sphbi.h,
reproduce the kernel presets independently of the oracle, and reject bad
arguments before touching the device.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_2507_21686_amd as sb
from tests import exact

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "sphbi.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(sphbi_\w+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert len(names) >= 8
    L = sb.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(sb.EXPORTS) <= set(names)


@pytest.mark.parametrize("kid", [0, 1, 2, 3])
def test_kernel_presets(kid):
    k = sb.kernel_preset(kid)
    mono = exact.monomials(kid)
    assert k.n_pieces == len(mono)
    for p, (coef, rad) in enumerate(mono):
        assert k.radius[p] == rad
        assert k.degree[p] == len(coef) - 1
        np.testing.assert_allclose([k.b[p][i] for i in range(len(coef))], coef, rtol=1e-13, atol=1e-12)
    assert k.c_d == pytest.approx(float(exact.c_d(kid)), rel=1e-14)
    n, R, deg, b, cd = oracle.kernel_monomials(kid)
    assert k.c_d == pytest.approx(cd, rel=1e-14)


def test_bad_arguments_rejected_without_device():
    L = sb.lib()
    k = sb.kernel_preset(0)
    o = sb.opts()
    z = C.c_void_p(None)
    # h <= 0
    rc = L.sphbi_integrate(C.byref(k), C.byref(o), 0.0, 1, 0, z, z, 0, z, z, z, z, 0, z, z, z, z, z, 0, z)
    assert rc == -1 and b"h must be" in L.sphbi_last_error()
    # n_nodes
    rc = L.sphbi_integrate(C.byref(k), C.byref(o), 1.0, 4, 0, z, z, 0, z, z, z, z, 0, z, z, z, z, z, 0, z)
    assert rc == -1
    # NULL kernel
    rc = L.sphbi_integrate(None, C.byref(o), 1.0, 1, 0, z, z, 0, z, z, z, z, 0, z, z, z, z, z, 0, z)
    assert rc == -1
    # degree out of range
    k2 = sb.kernel_preset(0)
    k2.degree[0] = 12
    rc = L.sphbi_integrate(C.byref(k2), C.byref(o), 1.0, 1, 0, z, z, 0, z, z, z, z, 0, z, z, z, z, z, 0, z)
    assert rc == -1
    # NULL particle arrays with N > 0
    rc = L.sphbi_integrate(C.byref(k), C.byref(o), 1.0, 1, 5, z, z, 0, z, z, z, z, 0, z, z, z, z, z, 0, z)
    assert rc == -1
    # unknown preset / precision
    assert L.sphbi_kernel_preset(9, C.byref(sb.SphbiKernel())) == -1
    o2 = sb.opts()
    o2.precision = 7
    rc = L.sphbi_integrate(C.byref(k), C.byref(o2), 1.0, 1, 0, z, z, 0, z, z, z, z, 0, z, z, z, z, z, 0, z)
    assert rc == -1
    # N = 0 is a no-op
    rc = L.sphbi_integrate(C.byref(k), C.byref(o), 1.0, 1, 0, z, z, 0, z, z, z, z, 0, z, z, z, z, z, 0, z)
    assert rc == 0


def test_workspace_size():
    # 128 B records per triangle (rounded up to 256 B), then 256 B for the refinement counter
    # records (128 B per triangle, in 256-B steps), the counter, double-double records
    assert sb.lib().sphbi_integrate_workspace(1000) == 3 * 1000 * 16 * 8 + 256
    assert sb.lib().sphbi_integrate_workspace(1001) == 3 * 1002 * 16 * 8 + 256
    assert sb.lib().sphbi_integrate_workspace(0) >= 8


def test_operator_arguments_rejected_without_device():
    """sphbi_operator validates before any launch: unknown operator, mixed
    precision, missing particle values or fields, and a short workspace."""
    import numpy as np
    L = sb.lib()
    k = sb.kernel_preset(0)
    o = sb.opts()
    z = C.c_void_p(None)
    N, T = 4, 2
    host = np.zeros(64, dtype=np.float64)            # stand-in pointers: never dereferenced on these paths
    p = C.c_void_p(host.ctypes.data)
    need = int(L.sphbi_operator_workspace(N, T))
    assert need >= 2 * T * 128 + 2 * N * 8

    def call(op, opts, qa=p, fa=p, ws_bytes=need):
        return L.sphbi_operator(C.byref(k), C.byref(opts), op, 1.0, 3, N, p, p, qa, p, T, p, fa, p, p, p, 8, p, p,
                                p, ws_bytes, z)

    assert call(7, o) == -1 and b"unknown operator" in L.sphbi_last_error()
    om = sb.opts(sb.MIXED)
    assert call(sb.OP_GRAD_DIFFERENCE, om) == -2
    assert call(sb.OP_GRAD_DIFFERENCE, o, qa=z) == -1
    assert call(sb.OP_DIV_CURL, o, fa=z) == -1
    assert call(sb.OP_GRAD_SYMMETRIC, o, ws_bytes=need - 8) == -4
    # N = 0 is a no-op
    assert L.sphbi_operator(C.byref(k), C.byref(o), 0, 1.0, 3, 0, z, z, z, z, 0, z, z, z, z, z, 0, z, z, z, 0,
                            z) == 0


def test_pressure_contact_arguments_rejected_without_device():
    """sphbi_pressure_contact validates before any launch."""
    import numpy as np
    L = sb.lib()
    k = sb.kernel_preset(0)
    o = sb.opts()
    z = C.c_void_p(None)
    N, T = 4, 2
    host = np.zeros(64, dtype=np.float64)            # stand-in pointers: never dereferenced on these paths
    p = C.c_void_p(host.ctypes.data)
    need = int(L.sphbi_operator_workspace(N, T))

    def call(rho0=1000.0, opts=o, p_pair=p, ws_bytes=need):
        return L.sphbi_pressure_contact(C.byref(k), C.byref(opts), 1.0, rho0, N, p, p, p, p, T, p, p, p, 8, p_pair,
                                        p, p, p, ws_bytes, z)

    assert call(rho0=0.0) == -1 and b"rho0" in L.sphbi_last_error()
    assert call(opts=sb.opts(sb.MIXED)) == -2
    assert call(p_pair=z) == -1
    assert call(ws_bytes=need - 8) == -4


def test_quadrature_arguments_rejected_without_device():
    """sphbi_integrate_quadrature validates before any launch."""
    L = sb.lib()
    k = sb.kernel_preset(1)
    z = C.c_void_p(None)
    host = np.zeros(64, dtype=np.float64)            # stand-in pointers: never dereferenced on these paths
    p = C.c_void_p(host.ctypes.data)

    def call(n_gauss=8, h=1.0, n_nodes=3, N=4, px=p, tri=p):
        return L.sphbi_integrate_quadrature(C.byref(k), h, n_nodes, n_gauss, N, px, p, 2, tri, p, p, p, 8, p, p, p,
                                            z)

    assert call(n_gauss=0) == -1 and b"n_gauss" in L.sphbi_last_error()
    assert call(n_gauss=sb.MAX_GAUSS + 1) == -1
    assert call(h=0.0) == -1
    assert call(n_nodes=4) == -1
    assert call(px=z) == -1
    assert call(tri=z) == -1
    assert call(N=0) == 0                              # nothing to do, nothing launched


def test_binding_fails_loudly_without_library_or_device(monkeypatch):
    """No CPU fallback: a missing library raises, and so do host tensors."""
    import torch
    monkeypatch.setattr(sb, "_lib", None)
    monkeypatch.setattr(sb, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libsphbi.so"))
    with pytest.raises(sb.SphbiError, match="missing"):
        sb.lib()
    monkeypatch.undo()
    x = torch.zeros(4, dtype=torch.float64)
    tri = torch.zeros(6, 2, dtype=torch.float64)
    with pytest.raises(sb.SphbiError, match="GPU"):
        sb.integrate_quadrature(0, 1.0, x, x, tri, torch.zeros(1, 2, dtype=torch.float64),
                                torch.zeros(5, dtype=torch.int64), torch.zeros(0, dtype=torch.int32), 4)
    with pytest.raises(sb.SphbiError, match="GPU"):
        sb.integrate(0, 1.0, x, x, tri, torch.zeros(1, 2, dtype=torch.float64), torch.zeros(5, dtype=torch.int64),
                     torch.zeros(0, dtype=torch.int32))


def test_oversized_launches_rejected_without_device():
    """Sizes whose grids would not fit a 32-bit thread count are refused with
    EUNSUPPORTED before any launch (stand-in pointers, never dereferenced)."""
    L = sb.lib()
    k = sb.kernel_preset(0)
    o = sb.opts()
    z = C.c_void_p(None)
    host = np.zeros(64, dtype=np.float64)
    p = C.c_void_p(host.ctypes.data)
    big = 1 << 28
    rc = L.sphbi_integrate(C.byref(k), C.byref(o), 1.0, 1, big, p, p, 4, p, p, p, p, 8, p, p, p, z, p, 1 << 20, z)
    assert rc == -2 and b"particles" in L.sphbi_last_error()
    rc = L.sphbi_integrate(C.byref(k), C.byref(o), 1.0, 1, 4, p, p, big, p, p, p, p, 8, p, p, p, z, p, 1 << 20, z)
    assert rc == -2
    grid, wsb = sb.SphbiGrid(), C.c_size_t(0)
    rc = L.sphbi_pairlist_plan(big, p, p, 4, p, 1.0, C.byref(grid), C.byref(wsb), z)
    assert rc == -2
    rc = L.sphbi_integrate_noalloc(C.byref(k), C.byref(o), 1.0, 1, 4, p, p, sb.NOALLOC_MAX_TRIANGLES + 1, p, p, p,
                                   p, 8, p, p, p, z, z)
    assert rc == -2 and b"fixed record array" in L.sphbi_last_error()
    # the quadrature grid holds 256 // n_gauss particles per block
    rc = L.sphbi_integrate_quadrature(C.byref(k), 1.0, 1, 64, (1 << 27), p, p, 2, p, p, p, p, 8, p, p, p, z)
    assert rc == -2 and b"at most" in L.sphbi_last_error()
