"""Mixed FP32/FP64 forward path against the FP64 oracle.

The mixed path takes its square roots and reciprocals (and, for P0/P1
fields, the sector arctangents) from the FP32 units and keeps the logarithm
of the radial term, the radial recurrences, the kernel contraction and the
per-particle sums in FP64; edges whose line passes within tau*h of the
particle run fully in FP64.  Target: 1e-6 in the scale-normalised error of
tests/metrics.py.  The remaining FP32 roundings sit where neither the
kernel's monomial cancellation nor the P3 extrapolation factor multiplies
them.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2507_21686_amd as sb
from paper_2507_21686_amd import workloads as W
from tests import metrics

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NTH = 16
TOL = 1e-6


def say(msg):
    print(msg, flush=True)


def to_dev(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a), device=DEV) for a in arrs]


def gpu_pairs(wl):
    tpx, tpy, ttri = to_dev(wl.px, wl.py, wl.tri)
    off, idx = sb.pairlist(tpx, tpy, ttri, wl.h)
    torch.cuda.synchronize()
    return off.cpu().numpy(), idx.cpu().numpy()


def run(kid, h, px, py, tri, nodal, off, idx, precision, tau=1e-4, per_pair=False):
    tpx, tpy, ttri, tnod = to_dev(px, py, tri, nodal)
    toff = torch.as_tensor(off, device=DEV, dtype=torch.int64)
    tidx = torch.as_tensor(idx, device=DEV, dtype=torch.int32)
    out = sb.integrate(kid, h, tpx, tpy, ttri, tnod, toff, tidx, per_pair=per_pair, precision=precision,
                       tau_edge=tau)
    torch.cuda.synchronize()
    return [o.cpu().numpy() if o is not None else None for o in out]


def sub_csr(off, idx, sel):
    soff = np.concatenate([[0], np.cumsum(off[sel + 1] - off[sel])])
    sidx = np.concatenate([idx[off[i]:off[i + 1]] for i in sel]) if len(sel) else np.zeros(0, np.int32)
    return soff, sidx


def amax_of(wl):
    return float(np.abs(wl.nodal).max()) * (3.0 if wl.n_nodes == 10 else 1.0)


def check_mixed(wl, tol=TOL, sample=None, tau=1e-4):
    say(f"mixed {wl.name}: kernel={wl.kernel} n_nodes={wl.n_nodes} tau={tau}")
    off, idx = gpu_pairs(wl)
    got = run(wl.kernel, wl.h, wl.px, wl.py, wl.tri, wl.nodal, off, idx, sb.MIXED, tau)
    sel = np.arange(wl.n_particles) if sample is None else sample
    soff, sidx = sub_csr(off, idx, sel)
    ref = oracle.integrate(wl.kernel, wl.h, wl.px[sel], wl.py[sel], wl.tri, wl.nodal, soff, sidx, nthreads=NTH)
    eI, eG = metrics.report(wl.kernel, wl.h, amax_of(wl), [g[sel] for g in got], ref)
    say(f"  pairs={off[-1]} checked={len(sel)} errI={eI:.2e} errG={eG:.2e}")
    assert eI <= tol and eG <= tol
    return eI, eG


@pytest.mark.parametrize("kid", [0, 1, 2, 3])
@pytest.mark.parametrize("order", [0, 1, 3])
def test_mixed_covering_small(kid, order):
    wl = W.covering_workload(n_side=64, nx=8, ny=16, seed=2, kernel=kid, field_order=order)
    check_mixed(wl)


def test_mixed_band_wall():
    check_mixed(W.band_wall(seed=1))


@pytest.mark.parametrize("kid", [0, 1, 2, 3])
@pytest.mark.parametrize("order", [0, 1, 3])
def test_mixed_slivers(kid, order):
    """Particles within 1e-8..1e-2 h of edges and vertices of 0.5-degree slivers."""
    wl = W.sliver_stress(seed=3, grid=16, kernel=kid, field_order=order)
    check_mixed(wl)


@pytest.mark.parametrize("kid", [0, 2])
def test_mixed_slivers_without_fp64_islands(kid):
    """tau = 0: every edge on the FP32 units, also for particles 1e-8 h from an edge."""
    wl = W.sliver_stress(seed=3, grid=16, kernel=kid, field_order=0)
    check_mixed(wl, tau=0.0)


@pytest.mark.parametrize("kid", [0, 1, 2, 3])
@pytest.mark.parametrize("order", [0, 3])
def test_mixed_random_pairs_per_pair(kid, order):
    """Every clipping case, one pair per particle, per-pair output.

    Bound: 1e-6 times the P3 extrapolation factor (d_max/width)^order, capped
    below by the FP64 bound 8 eps K kappa of the exact path.
    """
    from tests.test_gpu_forward import KFAC, conditioning
    n = 3000
    tri = W.random_pairs(n, 100 + kid, spread=1.3, scale_range=(0.2, 2.5))
    nn = {0: 1, 1: 3, 3: 10}[order]
    A = np.random.default_rng(kid * 7 + order).standard_normal((nn, n))
    say(f"mixed random pairs kid={kid} order={order}")
    px = np.zeros(n)
    py = np.zeros(n)
    off = np.arange(n + 1, dtype=np.int64)
    idx = np.arange(n, dtype=np.int32)
    got = run(kid, 1.0, px, py, tri, A, off, idx, sb.MIXED, per_pair=True)
    ref = oracle.integrate(kid, 1.0, px, py, tri, A, off, idx, per_pair=True, nthreads=NTH)
    np.testing.assert_array_equal(got[3][0], got[0])
    amax = np.maximum(np.abs(A).max(0) * (3.0 if nn == 10 else 1.0), 1.0)
    sG = metrics.grad_scale(kid, 1.0) * amax
    eI = np.abs(got[0] - ref[0]) / np.maximum(np.abs(ref[0]), amax)
    eG = np.maximum(np.abs(got[1] - ref[1]), np.abs(got[2] - ref[2])) / np.maximum(
        np.maximum(np.abs(ref[1]), np.abs(ref[2])), sG)
    kappa = conditioning(tri, order)
    bound = TOL * kappa + 8 * 1.1e-16 * KFAC[kid] * kappa
    say(f"  errI={eI.max():.2e} errG={eG.max():.2e} median errI={np.median(eI):.1e} "
        f"worst err/bound={max((eI / bound).max(), (eG / bound).max()):.2f}")
    assert np.all(eI <= bound) and np.all(eG <= bound)


def test_mixed_edge_cases():
    say("mixed edge cases")
    cases = [
        [0.0, 0.0, 0.5, 0.1, 0.2, 0.6],          # particle at a vertex
        [-0.5, 0.0, 0.5, 0.0, 0.0, 0.7],         # particle on an edge
        [-0.5, 0.3, 0.5, 0.3, 0.0, 0.3],         # zero area
        [-50, -50, 50, -50, 0, 60],              # huge triangle covering the disc
        [1.0, 0.0, 1.5, 0.0, 1.2, 0.5],          # vertex exactly on the support circle
        [0.3, 0.3, 0.3 + 1e-9, 0.3, 0.3, 0.3 + 1e-9],   # tiny triangle
        [1e-9, -0.4, 1e-9, 0.4, 0.8, 0.0],       # particle 1e-9 from an edge line
        [1e-30, -0.4, 1e-30, 0.4, 0.8, 0.0],     # 1e-30 from an edge line (below FP32 range)
        [0.999999, -0.4, 0.999999, 0.4, 2.0, 0.0],   # edge line 1e-6 inside the support circle
    ]
    tri = np.array(cases, dtype=np.float64).T.copy()
    n = tri.shape[1]
    A = np.ones((1, n))
    px = np.zeros(n)
    py = np.zeros(n)
    off = np.arange(n + 1, dtype=np.int64)
    idx = np.arange(n, dtype=np.int32)
    ref = oracle.integrate(0, 1.0, px, py, tri, A, off, idx)
    sG = metrics.grad_scale(0, 1.0)
    for tau in (1e-4, 0.0):
        got = run(0, 1.0, px, py, tri, A, off, idx, sb.MIXED, tau)
        for k in range(3):
            assert np.all(np.isfinite(got[k]))
        assert np.abs(got[0] - ref[0]).max() <= TOL
        assert max(np.abs(got[1] - ref[1]).max(), np.abs(got[2] - ref[2]).max()) <= TOL * sG
        assert got[0][2] == 0.0 and got[1][2] == 0.0
    # a threshold above every edge distance sends every edge to FP64
    got = run(0, 1.0, px, py, tri, A, off, idx, sb.MIXED, 1e30)
    for k in range(3):
        np.testing.assert_allclose(got[k], ref[k], atol=1e-12)


def test_mixed_rejects_bad_tau():
    say("mixed bad tau")
    tri = np.array([[0.0, 0.0, 0.5, 0.1, 0.2, 0.6]]).T.copy()
    with pytest.raises(RuntimeError, match="tau_edge"):
        run(0, 1.0, np.zeros(1), np.zeros(1), tri, np.ones((1, 1)), np.array([0, 1]), np.array([0], np.int32),
            sb.MIXED, -1.0)


def test_mixed_full_size_against_fp64_path():
    """All 1,048,576 particles of the 65,536-triangle P3 workload, mixed vs the
    FP64 path (itself within 2e-12 of the oracle), plus 1024 sampled particles
    against the oracle directly."""
    wl = W.covering_workload()
    say("mixed full size")
    off, idx = gpu_pairs(wl)
    a = run(wl.kernel, wl.h, wl.px, wl.py, wl.tri, wl.nodal, off, idx, sb.MIXED)
    b = run(wl.kernel, wl.h, wl.px, wl.py, wl.tri, wl.nodal, off, idx, sb.FP64)
    eI, eG = metrics.report(wl.kernel, wl.h, amax_of(wl), a, b)
    say(f"  vs FP64 path: pairs={off[-1]} errI={eI:.2e} errG={eG:.2e}")
    assert eI <= TOL and eG <= TOL
    sel = np.sort(np.random.default_rng(5).choice(wl.n_particles, 1024, replace=False))
    soff, sidx = sub_csr(off, idx, sel)
    ref = oracle.integrate(wl.kernel, wl.h, wl.px[sel], wl.py[sel], wl.tri, wl.nodal, soff, sidx, nthreads=NTH)
    eI, eG = metrics.report(wl.kernel, wl.h, amax_of(wl), [g[sel] for g in a], ref)
    say(f"  vs oracle (1024 particles): errI={eI:.2e} errG={eG:.2e}")
    assert eI <= TOL and eG <= TOL


@pytest.mark.parametrize("kid", [0, 1, 2, 3])
@pytest.mark.parametrize("order", [0, 3])
def test_mixed_precision_stress_full_size(kid, order):
    """262,144 particles near 16,384 slivers, per kernel, constant and cubic
    fields: mixed vs the FP64 path on every particle, 1024 sampled particles
    vs the oracle."""
    wl = W.sliver_stress(seed=3, kernel=kid, field_order=order)
    say(f"mixed stress kid={kid}: N={wl.n_particles} T={wl.n_triangles}")
    off, idx = gpu_pairs(wl)
    a = run(wl.kernel, wl.h, wl.px, wl.py, wl.tri, wl.nodal, off, idx, sb.MIXED)
    b = run(wl.kernel, wl.h, wl.px, wl.py, wl.tri, wl.nodal, off, idx, sb.FP64)
    eI, eG = metrics.report(kid, wl.h, amax_of(wl), a, b)
    say(f"  vs FP64 path: pairs={off[-1]} errI={eI:.2e} errG={eG:.2e}")
    assert eI <= TOL and eG <= TOL
    sel = np.sort(np.random.default_rng(6).choice(wl.n_particles, 1024, replace=False))
    soff, sidx = sub_csr(off, idx, sel)
    ref = oracle.integrate(kid, wl.h, wl.px[sel], wl.py[sel], wl.tri, wl.nodal, soff, sidx, nthreads=NTH)
    eI, eG = metrics.report(kid, wl.h, amax_of(wl), [g[sel] for g in a], ref)
    say(f"  vs oracle: errI={eI:.2e} errG={eG:.2e}")
    assert eI <= TOL and eG <= TOL
