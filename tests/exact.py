"""Exact reference values written independently of the oracle.

Kernel facts come from sympy on the textbook kernel formulas; 1-D profiles
from mpmath quadrature.  Nothing here calls the oracle or the device library.
"""
from functools import lru_cache

import mpmath as mp
import numpy as np
import sympy as sp

q = sp.symbols("q", nonnegative=True)

# (piece polynomial in q, radius) for each kernel id of the C-ABI
KERNELS = {
    0: [((1 - q) ** 4 * (1 + 4 * q), 1)],
    1: [((1 - q) ** 6 * (1 + 6 * q + sp.Rational(35, 3) * q ** 2), 1)],
    2: [((1 - q) ** 8 * (1 + 8 * q + 25 * q ** 2 + 32 * q ** 3), 1)],
    3: [((1 - q) ** 3, 1), (-4 * (sp.Rational(1, 2) - q) ** 3, sp.Rational(1, 2))],
}


@lru_cache(None)
def c_d(kid):
    s = sum(sp.integrate(k * q, (q, 0, R)) for k, R in KERNELS[kid])
    return sp.nsimplify(1 / (2 * sp.pi * s))


@lru_cache(None)
def int_k(kid):
    """int_0^1 k(q) dq."""
    return sum(sp.integrate(k, (q, 0, R)) for k, R in KERNELS[kid])


@lru_cache(None)
def mu2(kid):
    """Second moment int x^2 W d^2x for support 1: C_d pi int_0^1 k q^3 dq."""
    return sp.nsimplify(c_d(kid) * sp.pi * sum(sp.integrate(k * q ** 3, (q, 0, R)) for k, R in KERNELS[kid]))


@lru_cache(None)
def monomials(kid):
    out = []
    for k, R in KERNELS[kid]:
        p = sp.Poly(sp.expand(k), q)
        out.append(([float(p.coeff_monomial(q ** i)) for i in range(p.degree() + 1)], float(R)))
    return out


def k_num(kid):
    fs = [(sp.lambdify(q, k, "mpmath"), R) for k, R in KERNELS[kid]]
    dfs = [(sp.lambdify(q, sp.diff(k, q), "mpmath"), R) for k, R in KERNELS[kid]]

    def k(r):
        return sum(f(r) for f, R in fs if r < R)

    def dk(r):
        return sum(f(r) for f, R in dfs if r < R)
    return k, dk


def half_plane(kid, s, h=1.0):
    """(I, G_n) for the solid half plane {x . n >= s} (support units, P0 = 1).

    I = C_d int_s^1 k(r) r 2 acos(s/r) dr (for s >= 0) and the gradient along
    the inward normal n: G_n = -(C_d/h) int_s^1 k'(r) r 2 sin(acos(s/r)) dr.
    For s < 0 the complement identity I(s) = 1 - I(-s), G(s) = G(-s) is used.
    """
    mp.mp.dps = 30
    k, dk = k_num(kid)
    cd = mp.mpf(str(sp.N(c_d(kid), 40)))
    a = abs(s)
    pts = [a, 0.5, 1] if a < 0.5 and kid == 3 else [a, 1]
    I = cd * mp.quad(lambda r: k(r) * r * 2 * mp.acos(a / r), pts)
    G = -cd * mp.quad(lambda r: dk(r) * r * 2 * mp.sqrt(1 - (a / r) ** 2), pts) / h
    if s < 0:
        I = 1 - I
    return float(I), float(G)


def rot(t):
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, -s], [s, c]])
