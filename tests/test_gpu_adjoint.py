"""GPU adjoint (vector-Jacobian product) against the oracle.

* Leibniz: with cotangent gI = 1 the particle gradient is G itself
  (eq. nablaIntegral is the x-derivative of eq. sphintegral).
* Nodal gradients: the integrals are linear in the nodal values, so the
  oracle gives them exactly from unit-field evaluations.
* Vertex and particle gradients: 4th-order central differences of the
  oracle (step 1e-3 h; truncation and oracle noise both near 1e-11).
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


def say(msg):
    print(msg, flush=True)


def setup(wl, seed=0):
    t = [torch.as_tensor(np.ascontiguousarray(a), device=DEV) for a in (wl.px, wl.py, wl.tri, wl.nodal)]
    off, idx = sb.pairlist(t[0], t[1], t[2], wl.h)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((3, wl.n_particles))
    tg = [torch.as_tensor(x, device=DEV) for x in g]
    return t, off, idx, g, tg


def owners(off):
    return np.repeat(np.arange(len(off) - 1), np.diff(off))


def loss_pairs(kid, h, wl, pairs, g, px=None, py=None, tri=None):
    """sum over the given (particle, triangle) pairs of g . (I, Gx, Gy), by the oracle"""
    px = wl.px if px is None else px
    py = wl.py if py is None else py
    tri = wl.tri if tri is None else tri
    s = 0.0
    for i, t in pairs:
        o = oracle.pair(kid, h, px[i], py[i], tri[:, t], wl.nodal[:, t])
        s += g[0][i] * o[0] + g[1][i] * o[1] + g[2][i] * o[2]
    return s


def fd4(f, e):
    return (8 * (f(1) - f(-1)) - (f(2) - f(-2))) / (12 * e)


def test_leibniz_particle_gradient_is_G():
    wl = W.covering_workload(n_side=64, nx=8, ny=16, seed=4, kernel=1, field_order=3)
    say("adjoint leibniz")
    (px, py, tri, nod), off, idx, _, _ = setup(wl)
    I, Gx, Gy = sb.integrate(wl.kernel, wl.h, px, py, tri, nod, off, idx)
    one = torch.ones_like(px)
    zero = torch.zeros_like(px)
    dpx, dpy, _, _ = sb.integrate_backward(wl.kernel, wl.h, px, py, tri, nod, off, idx, one, zero, zero)
    torch.cuda.synchronize()
    # Two code paths: G from the forward call (refined to 1e-12 of the scale
    # where the conditioning gate fires) and dI/dx from the FP64 transport-rule
    # adjoint.  The adjoint carries the FP64 closed form's error model, per pair
    # 16 eps Kf kappa^3 of the pair's gradient scale (Kf = 1109 for Wendland
    # C4, kappa = d_max l_max / |2 area| of the pair), summed over the
    # particle's pairs, plus the forward call's 1e-12.
    off_h, idx_h = off.cpu().numpy(), idx.cpu().numpy()
    own = owners(off_h)
    v = wl.tri[:, idx_h].copy()
    v[0::2] -= wl.px[own]
    v[1::2] -= wl.py[own]
    v = v.reshape(3, 2, -1) / wl.h
    d2 = (v ** 2).sum(1).max(0)
    l2 = np.max([((v[(k + 1) % 3] - v[k]) ** 2).sum(0) for k in range(3)], 0)
    a2 = np.abs((v[1, 0] - v[0, 0]) * (v[2, 1] - v[0, 1]) - (v[2, 0] - v[0, 0]) * (v[1, 1] - v[0, 1]))
    kappa = np.sqrt(d2 * l2) / a2
    sG = metrics.grad_scale(wl.kernel, wl.h) * 3.0 * np.abs(wl.nodal[:, idx_h]).max(0)
    bound = np.bincount(own, weights=16 * 1.1e-16 * 1109.0 * kappa ** 3 * sG, minlength=wl.n_particles)
    bound += 1e-12 * metrics.grad_scale(wl.kernel, wl.h) * 3.0 * np.abs(wl.nodal).max()
    worst = 0.0
    for d, g in ((dpx, Gx), (dpy, Gy)):
        err = np.abs(d.cpu().numpy() - g.cpu().numpy())
        worst = max(worst, float((err / bound).max()))
        assert np.all(err <= bound)
    say(f"  worst |dI/dx - G| / error model: {worst:.2e}")


@pytest.mark.parametrize("kid", [0, 1, 2, 3])
@pytest.mark.parametrize("order", [0, 1, 3])
def test_every_instantiation_nodal_and_leibniz(kid, order):
    """Every compiled adjoint variant (kernel degree x field order): nodal
    gradients against the oracle's unit-field integrals (exact by linearity),
    and the particle gradient of sum I against the forward pass's G."""
    wl = W.covering_workload(n_side=16, nx=2, ny=4, seed=5, kernel=kid, field_order=order)
    say(f"adjoint instantiation kid={kid} order={order}")
    (px, py, tri, nod), off_t, idx_t, g, tg = setup(wl, seed=10 + kid)
    _, _, _, dnod = sb.integrate_backward(wl.kernel, wl.h, px, py, tri, nod, off_t, idx_t, *tg)
    I, Gx, Gy = sb.integrate(wl.kernel, wl.h, px, py, tri, nod, off_t, idx_t)
    one, zero = torch.ones_like(px), torch.zeros_like(px)
    dpx, dpy, _, _ = sb.integrate_backward(wl.kernel, wl.h, px, py, tri, nod, off_t, idx_t, one, zero, zero)
    torch.cuda.synchronize()
    dnod = dnod.cpu().numpy()
    off, idx = off_t.cpu().numpy(), idx_t.cpu().numpy()
    own = owners(off)
    ref = np.zeros_like(wl.nodal)
    for n in range(wl.n_nodes):
        unit = np.zeros_like(wl.nodal)
        unit[n] = 1.0
        _, _, _, pp = oracle.integrate(kid, wl.h, wl.px, wl.py, wl.tri, unit, off, idx, per_pair=True, nthreads=NTH)
        contrib = g[0][own] * pp[0] + g[1][own] * pp[1] + g[2][own] * pp[2]
        ref[n] = np.bincount(idx, weights=contrib, minlength=wl.n_triangles)
    kfac = {0: 141.0, 1: 1109.0, 2: 8704.0, 3: 30.0}[kid]
    err = np.abs(dnod - ref).max() / np.abs(ref).max()
    say(f"  nodal scaled error {err:.2e}")
    assert err <= 1e-13 * kfac
    # both sides are FP64 evaluations of the same integrals (the adjoint's
    # moments against the forward pass), so they differ by rounding that
    # scales with the kernel's cancellation factor K_f, and for cubic fields
    # with the extrapolation of the field about the particle: 5 eps' K_f with
    # eps' = 1e-15, four times that for cubic fields (measured on this
    # workload: 2e-15 ... 4.8e-12, between 4x and 44x below the bound)
    scale = float(torch.maximum(torch.abs(Gx), torch.abs(Gy)).max())
    bound = 5e-15 * kfac * (4.0 if order == 3 else 1.0)
    for d, gg in ((dpx, Gx), (dpy, Gy)):
        e = float(torch.abs(d - gg).max()) / scale
        say(f"  leibniz scaled error {e:.2e} (bound {bound:.1e})")
        assert e < bound


@pytest.mark.parametrize("kid,order", [(0, 0), (1, 3), (3, 1), (2, 3)])
def test_vjp_against_oracle(kid, order):
    wl = W.covering_workload(n_side=32, nx=4, ny=8, seed=4, kernel=kid, field_order=order)
    say(f"adjoint vjp kid={kid} order={order}")
    (px, py, tri, nod), off_t, idx_t, g, tg = setup(wl, seed=kid)
    dpx, dpy, dtri, dnod = sb.integrate_backward(wl.kernel, wl.h, px, py, tri, nod, off_t, idx_t, *tg)
    torch.cuda.synchronize()
    dpx, dpy, dtri, dnod = [x.cpu().numpy() for x in (dpx, dpy, dtri, dnod)]
    off, idx = off_t.cpu().numpy(), idx_t.cpu().numpy()
    own = owners(off)
    nn = wl.n_nodes
    # nodal gradients: exact by linearity
    ref_nod = np.zeros_like(wl.nodal)
    for n in range(nn):
        unit = np.zeros_like(wl.nodal)
        unit[n] = 1.0
        _, _, _, pp = oracle.integrate(kid, wl.h, wl.px, wl.py, wl.tri, unit, off, idx, per_pair=True, nthreads=NTH)
        contrib = g[0][own] * pp[0] + g[1][own] * pp[1] + g[2][own] * pp[2]
        ref_nod[n] = np.bincount(idx, weights=contrib, minlength=wl.n_triangles)
    sc = np.abs(ref_nod).max()
    kfac = {0: 141.0, 1: 1109.0, 2: 8704.0, 3: 30.0}[kid]      # monomial kernel cancellation
    assert np.abs(dnod - ref_nod).max() <= 1e-13 * kfac * sc
    # vertex gradients of sampled triangles: finite differences of the oracle
    rng = np.random.default_rng(1)
    e = 1e-3 * wl.h
    tsel = rng.choice(wl.n_triangles, 12, replace=False)
    worst = 0.0
    for t in tsel:
        pairs = [(own[q], t) for q in np.nonzero(idx == t)[0]]
        for k in range(6):
            def f(s):
                tr = wl.tri.copy()
                tr[k, t] += s * e
                return loss_pairs(kid, wl.h, wl, pairs, g, tri=tr)
            ref = fd4(f, e)
            worst = max(worst, abs(dtri[k, t] - ref) / max(1.0, abs(ref)))
    say(f"  vertex grad worst rel err {worst:.2e}")
    assert worst < 3e-7          # finite-difference noise and truncation
    # particle gradients of sampled particles
    psel = rng.choice(np.nonzero(np.diff(off) > 0)[0], 12, replace=False)
    worst = 0.0
    for i in psel:
        pairs = [(i, idx[q]) for q in range(off[i], off[i + 1])]
        for comp, dref in ((0, dpx), (1, dpy)):
            def f(s):
                p2 = (wl.px if comp else wl.px.copy())
                q2 = (wl.py.copy() if comp else wl.py)
                if comp == 0:
                    p2[i] += s * e
                else:
                    q2[i] += s * e
                return loss_pairs(kid, wl.h, wl, pairs, g, px=p2, py=q2)
            ref = fd4(f, e)
            worst = max(worst, abs(dref[i] - ref) / max(1.0, abs(ref)))
    say(f"  particle grad worst rel err {worst:.2e}")
    assert worst < 3e-7


@pytest.mark.parametrize("kid,order", [(0, 3), (3, 1)])
def test_vjp_nodal_degenerate_geometry(kid, order):
    """Nodal gradients (exact by linearity) where a fan triangle is skipped:
    particle at a vertex, on an edge and on an edge's extension."""
    say(f"adjoint degenerate geometry kid={kid} order={order}")
    cases = [
        [0.0, 0.0, 0.5, 0.1, 0.2, 0.6],
        [-1.5, 0.0, 1.5, 0.0, 0.0, 1.7],
        [-0.5, 0.0, 1.5, 0.0, 0.0, 0.7],
        [0.3, 0.0, 1.8, 0.0, 0.9, 0.9],
        [-1.2, -0.4, 1.4, -0.4, 0.1, 1.3],
    ]
    tri = np.array(cases, dtype=np.float64).T.copy()
    n = tri.shape[1]
    nn = {0: 1, 1: 3, 3: 10}[order]
    rng = np.random.default_rng(3)
    A = rng.standard_normal((nn, n))
    px, py = np.zeros(n), np.zeros(n)
    off = np.arange(n + 1, dtype=np.int64)
    idx = np.arange(n, dtype=np.int32)
    g = [rng.standard_normal(n) for _ in range(3)]
    dev = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), device="cuda:0", dtype=dt)
    dpx, dpy, dtri, dnod = sb.integrate_backward(kid, 1.0, dev(px), dev(py), dev(tri), dev(A), dev(off, torch.int64),
                                                 dev(idx, torch.int32), dev(g[0]), dev(g[1]), dev(g[2]))
    torch.cuda.synchronize()
    dnod = dnod.cpu().numpy()
    ref = np.zeros_like(A)
    for k in range(nn):
        unit = np.zeros_like(A)
        unit[k] = 1.0
        I, X, Y = oracle.integrate(kid, 1.0, px, py, tri, unit, off, idx)
        ref[k] = g[0] * I + g[1] * X + g[2] * Y
    err = np.abs(dnod - ref).max() / max(1.0, np.abs(ref).max())
    say(f"  nodal gradient scaled error {err:.2e}")
    assert err < 1e-11


def test_autograd_function_and_determinism():
    wl = W.covering_workload(n_side=32, nx=4, ny=8, seed=4, kernel=1, field_order=3)
    say("autograd")
    (px, py, tri, nod), off, idx, g, tg = setup(wl)
    leaves = [x.clone().requires_grad_(True) for x in (px, py, tri, nod)]
    I, Gx, Gy = sb.BoundaryIntegral.apply(*leaves, off, idx, wl.kernel, wl.h)
    loss = (I * tg[0] + Gx * tg[1] + Gy * tg[2]).sum()
    loss.backward()
    ref = sb.integrate_backward(wl.kernel, wl.h, px, py, tri, nod, off, idx, *tg)
    ref2 = sb.integrate_backward(wl.kernel, wl.h, px, py, tri, nod, off, idx, *tg)
    for leaf, r, r2 in zip(leaves, ref, ref2):
        assert torch.equal(leaf.grad, r)
        assert torch.equal(r, r2)


def test_adjoint_full_size_sampled():
    """512^2 particles, 16,384-triangle mesh, Wendland C4, P3; sampled FD checks."""
    wl = W.covering_workload(n_side=512, nx=64, ny=128, seed=4, kernel=1, field_order=3)
    say("adjoint full size")
    (px, py, tri, nod), off_t, idx_t, g, tg = setup(wl, seed=7)
    dpx, dpy, dtri, dnod = sb.integrate_backward(wl.kernel, wl.h, px, py, tri, nod, off_t, idx_t, *tg)
    torch.cuda.synchronize()
    dpx, dtri = dpx.cpu().numpy(), dtri.cpu().numpy()
    off, idx = off_t.cpu().numpy(), idx_t.cpu().numpy()
    own = owners(off)
    say(f"  pairs={len(idx)}")
    rng = np.random.default_rng(3)
    e = 1e-3 * wl.h
    worst = 0.0
    for t in rng.choice(wl.n_triangles, 6, replace=False):
        pairs = [(own[q], t) for q in np.nonzero(idx == t)[0]]
        for k in (0, 3):
            def f(s):
                tr = wl.tri.copy()
                tr[k, t] += s * e
                return loss_pairs(wl.kernel, wl.h, wl, pairs, g, tri=tr)
            ref = fd4(f, e)
            worst = max(worst, abs(dtri[k, t] - ref) / max(1.0, abs(ref)))
    for i in rng.choice(wl.n_particles, 6, replace=False):
        pairs = [(i, idx[q]) for q in range(off[i], off[i + 1])]
        def f(s):
            p2 = wl.px.copy()
            p2[i] += s * e
            return loss_pairs(wl.kernel, wl.h, wl, pairs, g, px=p2)
        ref = fd4(f, e)
        worst = max(worst, abs(dpx[i] - ref) / max(1.0, abs(ref)))
    say(f"  worst rel err {worst:.2e}")
    assert worst < 1e-7


def test_adjoint_4096_sampled_pairs_fd():
    """Per-pair gradients on 4,096 pairs sampled from the 262,144-particle C4/P3
    differentiation workload.  Every sampled pair gets its own particle and its
    own copy of the triangle, so the adjoint's per-particle and per-triangle
    outputs are exactly the pair's gradients (same kernels, same per-pair code).
    Positions and vertices: 4th-order central differences of the oracle
    (step 1e-3 h: the oracle's quadrature noise of ~1e-13 relative would be
    amplified to ~1e-7 by a 1e-6 h step), errors on the scale of a pair's
    gradient and bounded by the conditioning law of the closed form (cubic
    fields extrapolated over the particle-anchored pieces); nodal values:
    exact by linearity (unit fields)."""
    wl = W.covering_workload(n_side=512, nx=64, ny=128, seed=4, kernel=1, field_order=3)
    say("adjoint 4096 sampled pairs")
    tpx, tpy, ttri = (torch.as_tensor(np.ascontiguousarray(a), device=DEV) for a in (wl.px, wl.py, wl.tri))
    off_t, idx_t = sb.pairlist(tpx, tpy, ttri, wl.h)
    torch.cuda.synchronize()
    off, idx = off_t.cpu().numpy(), idx_t.cpu().numpy()
    rng = np.random.default_rng(11)
    sel = np.sort(rng.choice(len(idx), 4096, replace=False))
    own = owners(off)
    ip, it = own[sel], idx[sel].astype(np.int64)
    M = len(sel)
    px, py = wl.px[ip].copy(), wl.py[ip].copy()
    tri = np.ascontiguousarray(wl.tri[:, it])
    nod = np.ascontiguousarray(wl.nodal[:, it])
    off1 = np.arange(M + 1, dtype=np.int64)
    idx1 = np.arange(M, dtype=np.int32)
    g = rng.standard_normal((3, M))
    t = [torch.as_tensor(a, device=DEV) for a in (px, py, tri, nod)]
    dpx, dpy, dtri, dnod = sb.integrate_backward(wl.kernel, wl.h, *t, torch.as_tensor(off1, device=DEV),
                                                 torch.as_tensor(idx1, device=DEV),
                                                 *[torch.as_tensor(x, device=DEV) for x in g])
    torch.cuda.synchronize()
    got = np.concatenate([dpx.cpu().numpy()[None], dpy.cpu().numpy()[None], dtri.cpu().numpy()])   # [8, M]

    def loss(px_, py_, tri_, nod_=nod):
        I, Gx, Gy = oracle.integrate(wl.kernel, wl.h, px_, py_, tri_, nod_, off1, idx1, nthreads=NTH)
        return g[0] * I + g[1] * Gx + g[2] * Gy

    e = 1e-3 * wl.h
    ref = np.zeros((8, M))
    for c in range(8):
        vals = {}
        for s_ in (-2, -1, 1, 2):
            px_, py_, tri_ = px.copy(), py.copy(), tri.copy()
            if c == 0:
                px_ += s_ * e
            elif c == 1:
                py_ += s_ * e
            else:
                tri_[c - 2] += s_ * e
            vals[s_] = loss(px_, py_, tri_)
        ref[c] = (8 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12 * e)
    # scale of a pair's position/vertex gradient: d/dx of I is G ~ S_G, of G ~ S_G / h
    sG = metrics.grad_scale(wl.kernel, wl.h)
    amax = 3.0 * np.abs(nod).max(0)
    S = amax * sG * (np.abs(g[0]) + (np.abs(g[1]) + np.abs(g[2])) / wl.h)
    # extrapolation of the cubic field over the particle-anchored pieces (the
    # conditioning law of the forward pass): kappa = (d_max / width)^3
    v = (tri.reshape(3, 2, M) - np.stack([px, py])[None]) / wl.h
    d_max = np.sqrt((v ** 2).sum(1)).max(0)
    Ls = np.stack([np.sqrt(((v[(k + 1) % 3] - v[k]) ** 2).sum(0)) for k in range(3)])
    area2 = np.abs((v[1, 0] - v[0, 0]) * (v[2, 1] - v[0, 1]) - (v[2, 0] - v[0, 0]) * (v[1, 1] - v[0, 1]))
    kappa = (d_max / (area2 / Ls.max(0))) ** 3
    err = np.abs(got - ref) / np.maximum(np.abs(ref), S)
    # floor: the 4th-order differences at 1e-3 h carry up to ~1e-10 of the scale
    # where an edge is nearly tangent to the support circle (the pair integral
    # is less smooth there; refining the step converges onto the adjoint)
    bound = 2e-10 + 16 * 1.1e-16 * 1109.0 * kappa
    say(f"  positions/vertices: worst scaled err {err.max():.2e}, median {np.median(err):.2e}, "
        f"worst err/bound {(err / bound).max():.2e}")
    assert np.all(err <= bound)
    # nodal values: the pair's loss is linear in them
    dn = dnod.cpu().numpy()
    refn = np.zeros_like(dn)
    for n in range(wl.n_nodes):
        unit = np.zeros_like(nod)
        unit[n] = 1.0
        refn[n] = loss(px, py, tri, unit)
    errn = np.abs(dn - refn).max() / np.abs(refn).max()
    say(f"  nodal: scaled err {errn:.2e}")
    assert errn < 1e-13 * 1109.0


def test_pairs_outside_the_csr_range_contribute_nothing():
    """A pair list longer than offsets[-1], or starting after offsets[0] = 0:
    the pairs outside [offsets[0], offsets[N]) belong to no particle, so the
    triangle and nodal gradients equal those of the exact list, bit for bit."""
    say("adjoint stray pairs")
    wl = W.covering_workload(n_side=64, nx=8, ny=16, seed=4, kernel=W.WENDLAND_C4, field_order=3)
    t, off, idx, g, tg = setup(wl)
    ref = sb.integrate_backward(wl.kernel, wl.h, *t, off, idx, *tg)
    T = wl.n_triangles
    rng = np.random.default_rng(1)
    pre = torch.as_tensor(rng.integers(0, T, 50).astype(np.int32), device=DEV)
    post = torch.as_tensor(rng.integers(0, T, 70).astype(np.int32), device=DEV)
    idx2 = torch.cat([pre, idx, post])
    got = sb.integrate_backward(wl.kernel, wl.h, *t, off + 50, idx2, *tg)
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    # no particles at all: nothing reaches the triangles
    z = torch.zeros(0, dtype=torch.float64, device=DEV)
    _, _, dtri, dnod = sb.integrate_backward(wl.kernel, wl.h, z, z, t[2], t[3],
                                             torch.zeros(1, dtype=torch.int64, device=DEV), idx, z, z, z)
    torch.cuda.synchronize()
    assert torch.all(dtri == 0) and torch.all(dnod == 0)


def test_mixed_adjoint_against_fp64_gradient():
    """The adjoint in the mixed precision mode (square roots, reciprocals and,
    for constant and linear fields, sector angles on the FP32 units) on the
    differentiation workload (262,144 particles, Wendland C4, cubic field):
    every particle, triangle and nodal gradient against the FP64 adjoint (to
    1e-6 of the gradient scale), and 4,096 sampled pairs against the oracle's
    FP64 gradient (4th-order central differences of the definition oracle,
    themselves within 1e-9 of the exact gradient), also to 1e-6."""
    wl = W.covering_workload(n_side=512, nx=64, ny=128, seed=4, kernel=1, field_order=3)
    say("mixed adjoint, full size")
    t, off, idx, g, tg = setup(wl)
    a = sb.integrate_backward(wl.kernel, wl.h, *t, off, idx, *tg, precision=sb.MIXED)
    b = sb.integrate_backward(wl.kernel, wl.h, *t, off, idx, *tg)
    torch.cuda.synchronize()
    sG = metrics.grad_scale(wl.kernel, wl.h)
    amax = 3.0 * float(np.abs(wl.nodal).max())
    gmax = float(np.abs(g).max())
    # scales: d(I, G)/dx ~ (S_G, S_G/h), d(I, G)/dA ~ (1, S_G) per unit field, summed over a triangle's pairs
    S_pos = amax * sG * gmax * (1 + 2 / wl.h)
    for k, (x, y) in enumerate(zip(a, b)):
        x, y = x.cpu().numpy(), y.cpu().numpy()
        scale = S_pos * (6.0 if k == 2 else 1.0) if k < 3 else gmax * (1 + 2 * sG) * 6.0
        err = np.abs(x - y).max() / scale
        say(f"  output {k}: max |mixed - fp64| / scale = {err:.2e}")
        assert err <= 1e-6
    # 4,096 sampled pairs, each on its own particle and triangle copy
    off_h, idx_h = off.cpu().numpy(), idx.cpu().numpy()
    rng = np.random.default_rng(12)
    sel = np.sort(rng.choice(len(idx_h), 4096, replace=False))
    own = owners(off_h)
    ip, it = own[sel], idx_h[sel].astype(np.int64)
    M = len(sel)
    px, py = wl.px[ip].copy(), wl.py[ip].copy()
    tri = np.ascontiguousarray(wl.tri[:, it])
    nod = np.ascontiguousarray(wl.nodal[:, it])
    off1 = np.arange(M + 1, dtype=np.int64)
    idx1 = np.arange(M, dtype=np.int32)
    gg = rng.standard_normal((3, M))
    tt = [torch.as_tensor(x, device=DEV) for x in (px, py, tri, nod)]
    dpx, dpy, dtri, dnod = sb.integrate_backward(wl.kernel, wl.h, *tt, torch.as_tensor(off1, device=DEV),
                                                 torch.as_tensor(idx1, device=DEV),
                                                 *[torch.as_tensor(x, device=DEV) for x in gg], precision=sb.MIXED)
    torch.cuda.synchronize()
    got = np.concatenate([dpx.cpu().numpy()[None], dpy.cpu().numpy()[None], dtri.cpu().numpy()])

    def loss(px_, py_, tri_, nod_=nod):
        I, Gx, Gy = oracle.integrate(wl.kernel, wl.h, px_, py_, tri_, nod_, off1, idx1, nthreads=NTH)
        return gg[0] * I + gg[1] * Gx + gg[2] * Gy

    e = 1e-3 * wl.h
    ref = np.zeros((8, M))
    for c in range(8):
        vals = {}
        for s_ in (-2, -1, 1, 2):
            px_, py_, tri_ = px.copy(), py.copy(), tri.copy()
            if c == 0:
                px_ += s_ * e
            elif c == 1:
                py_ += s_ * e
            else:
                tri_[c - 2] += s_ * e
            vals[s_] = loss(px_, py_, tri_)
        ref[c] = (8 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12 * e)
    S = 3.0 * np.abs(nod).max(0) * sG * (np.abs(gg[0]) + (np.abs(gg[1]) + np.abs(gg[2])) / wl.h)
    err = np.abs(got - ref) / np.maximum(np.abs(ref), S)
    say(f"  4096 pairs vs oracle gradient: worst scaled err {err.max():.2e}, median {np.median(err):.2e}")
    assert err.max() <= 1e-6
    dn = dnod.cpu().numpy()
    refn = np.zeros_like(dn)
    for n in range(wl.n_nodes):
        unit = np.zeros_like(nod)
        unit[n] = 1.0
        refn[n] = loss(px, py, tri, unit)
    errn = np.abs(dn - refn).max() / np.abs(refn).max()
    say(f"  nodal vs oracle: scaled err {errn:.2e}")
    assert errn <= 1e-6
