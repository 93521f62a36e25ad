"""Quadrature of the boundary integrals -- TEST INFRASTRUCTURE ONLY (oracle).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; the device library never calls it.

The paper measures its closed form against quadrature rules that cover the
whole triangle (Sec. 6.1-6.2): the same sums as eq. boundaryint and its
gradient, with each triangle's integral replaced by a weighted sum of the
integrand at fixed points.  The rule here is the collapsed (Duffy) product of
two n-point Gauss-Legendre rules (numpy's ``leggauss``): on the reference
triangle L1 = u, L2 = (1 - u) v with weight w_u w_v (1 - u), mapped to a
triangle by its barycentric coordinates with the factor |2 area|.

The integrand is the field (P0 constant, P1 barycentric, P3 cubic Lagrange on
the ten nodes v0, v1, v2, the points at 1/3 and 2/3 of v0v1, v1v2, v2v0, and
the centroid; Sec. 3) times W(|x - x'|) = C_d h^-2 k(q) or times
grad_x W = C_d h^-3 k'(q) (x - x') / (h q), q = |x - x'| / h, with the kernel's
monomial coefficients from the oracle's own kernel tables.
"""
from __future__ import annotations

import numpy as np

from . import kernel_monomials


def collapsed_rule(n):
    """Barycentric points (L0, L1, L2) and weights of the n x n collapsed
    Gauss-Legendre rule on the reference triangle (weights sum to 1/2)."""
    t, w = np.polynomial.legendre.leggauss(n)
    x, w = 0.5 * (t + 1.0), 0.5 * w
    U, V = np.meshgrid(x, x, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    L1 = U
    L2 = (1.0 - U) * V
    return (1.0 - L1 - L2).ravel(), L1.ravel(), L2.ravel(), (WU * WV * (1.0 - U)).ravel()


def basis(n_nodes, L0, L1, L2):
    """Values [n_nodes, ...] of the field's nodal basis at barycentric points."""
    if n_nodes == 1:
        return np.ones((1,) + np.shape(L0))
    if n_nodes == 3:
        return np.stack([L0, L1, L2])
    L = [L0, L1, L2]
    out = [0.5 * L[a] * (3 * L[a] - 1) * (3 * L[a] - 2) for a in range(3)]
    for a, b in ((0, 1), (1, 2), (2, 0)):
        out.append(4.5 * L[a] * L[b] * (3 * L[a] - 1))    # node at 1/3 from a
        out.append(4.5 * L[a] * L[b] * (3 * L[b] - 1))    # node at 2/3 from a
    out.append(27.0 * L0 * L1 * L2)
    return np.stack(out)


def _kernel(kernel_id, q):
    """k(q) and k'(q) of the piecewise polynomial kernel."""
    n_pieces, R, deg, b, cd = kernel_monomials(kernel_id)
    k = np.zeros_like(q)
    dk = np.zeros_like(q)
    for p in range(n_pieces):
        inside = q < R[p]
        c = b[p][: deg[p] + 1]
        k += np.where(inside, np.polynomial.polynomial.polyval(q, c), 0.0)
        dk += np.where(inside, np.polynomial.polynomial.polyval(q, np.polynomial.polynomial.polyder(c)), 0.0)
    return k, dk, cd


def integrate(kernel_id, h, px, py, tri, nodal, offsets, tri_idx, n, chunk=4096):
    """Per-particle (I, Gx, Gy) over a CSR pair list with the n x n collapsed
    rule per pair.  Pairs with an out-of-range triangle index contribute
    nothing."""
    px, py = np.asarray(px, float), np.asarray(py, float)
    tri, nodal = np.asarray(tri, float), np.asarray(nodal, float)
    offsets = np.asarray(offsets, np.int64)
    tri_idx = np.asarray(tri_idx, np.int64)
    N, T = px.shape[0], tri.shape[1]
    P = int(offsets[-1]) if N else 0
    owner = np.repeat(np.arange(N), np.diff(offsets))
    L0, L1, L2, w = collapsed_rule(n)
    B = basis(nodal.shape[0], L0, L1, L2)                        # [nn, n^2]
    out = np.zeros((3, N))
    for s in range(0, P, chunk):
        q = np.arange(s, min(P, s + chunk))
        t = tri_idx[q]
        ok = (t >= 0) & (t < T)
        q, t = q[ok], t[ok]
        if q.size == 0:
            continue
        v = tri[:, t]                                             # [6, m]
        area2 = np.abs((v[2] - v[0]) * (v[5] - v[1]) - (v[3] - v[1]) * (v[4] - v[0]))
        X = L0[None] * v[0][:, None] + L1[None] * v[2][:, None] + L2[None] * v[4][:, None]   # [m, n^2]
        Y = L0[None] * v[1][:, None] + L1[None] * v[3][:, None] + L2[None] * v[5][:, None]
        i = owner[q]
        dx, dy = (px[i][:, None] - X) / h, (py[i][:, None] - Y) / h
        r = np.sqrt(dx * dx + dy * dy)
        k, dk, cd = _kernel(kernel_id, r)
        A = nodal[:, t].T @ B                                     # field at the points [m, n^2]
        Aw = A * w[None] * area2[:, None]
        safe = np.where(r > 0.0, r, 1.0)
        g = np.where(r > 0.0, Aw * dk / safe, 0.0)
        vals = np.stack([(Aw * k).sum(1) * cd / h ** 2, (g * dx).sum(1) * cd / h ** 3,
                         (g * dy).sum(1) * cd / h ** 3])
        for c in range(3):
            out[c] += np.bincount(i, weights=vals[c], minlength=N)
    return out[0], out[1], out[2]
