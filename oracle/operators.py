"""SPH operators on the boundary -- TEST INFRASTRUCTURE ONLY (oracle).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; the device library never calls it.

Each operator is taken the way the paper states it, in plain steps:

* Difference and symmetric gradients (Sec. 2, eq. sphdiffops and the
  continuous forms of eq. intsphdiffops): for every (particle, triangle) pair
  the pre-weights f_i are formed at the element's nodes from the nodal values
  and the particle's own values (the paragraph after eq. improper), f is
  interpolated over the triangle with the field's basis, and int_T f grad W is
  taken by the oracle's definition (``oracle.integrate``).  To keep the
  threaded oracle loop, every pair gets a triangle record of its own carrying
  its f.
* Divergence and curl (the equation after eq. improper) from the gradient
  integrals of the two components.
* Boundary normal (App. A): int grad W of the unit field.
* Boundary pressure with one pressure value per contact (App. A): each
  pair's field is the constant rho0 (p_q / rho0^2 + p_i / rho_i^2).

Reading of the symmetric form: eq. intsphdiffops writes the bracket with a
plus (rho [<grad(A/rho)> + A/rho^2 <grad rho>]) and its integral with a
minus; the pre-weights in the text and the pressure term of App. A use the
plus, which is also what the bracket expands to.  The plus is taken.
"""
from __future__ import annotations

import numpy as np

from . import integrate


def _owners(offsets):
    offsets = np.asarray(offsets, dtype=np.int64)
    return np.repeat(np.arange(len(offsets) - 1), np.diff(offsets))


def _pair_gradient(kernel_id, h, px, py, tri, f_pairs, offsets, tri_idx, nthreads):
    """Per-particle sum of int_T f_q grad W over the particle's pairs q, with the
    nodal values f_pairs [n_nodes, P] of each pair.  Pairs whose triangle index
    is out of range contribute nothing."""
    tri = np.asarray(tri, dtype=np.float64)
    tri_idx = np.asarray(tri_idx, dtype=np.int64)
    P = tri_idx.shape[0]
    ok = (tri_idx >= 0) & (tri_idx < tri.shape[1])
    tri_pp = np.zeros((6, P))
    tri_pp[:, ok] = tri[:, tri_idx[ok]]
    f_pp = np.where(ok[None, :], f_pairs, 0.0)
    _, gx, gy = integrate(kernel_id, h, px, py, tri_pp, f_pp, offsets, np.arange(P, dtype=np.int32),
                          nthreads=nthreads)
    return gx, gy


def _pair_nodal(nodal, tri_idx):
    tri_idx = np.asarray(tri_idx, dtype=np.int64)
    T = nodal.shape[1]
    return nodal[:, np.clip(tri_idx, 0, max(T - 1, 0))] if T else np.zeros((nodal.shape[0], len(tri_idx)))


def gradient_difference(kernel_id, h, px, py, A_p, rho_p, tri, A, rho, offsets, tri_idx, nthreads=0):
    """(1/rho(x)) int rho (A - A(x)) grad W: pre-weights f_i = rho_i (A_i - A(x))."""
    own = _owners(offsets)
    Aq, rq = _pair_nodal(np.asarray(A, float), tri_idx), _pair_nodal(np.asarray(rho, float), tri_idx)
    f = rq * (Aq - np.asarray(A_p, float)[own][None, :])
    gx, gy = _pair_gradient(kernel_id, h, px, py, tri, f, offsets, tri_idx, nthreads)
    return gx / rho_p, gy / rho_p


def gradient_symmetric(kernel_id, h, px, py, A_p, rho_p, tri, A, rho, offsets, tri_idx, nthreads=0):
    """rho(x) int rho (A/rho^2 + A(x)/rho(x)^2) grad W: pre-weights
    f_i = rho_i (A_i / rho_i^2 + A(x) / rho(x)^2)."""
    own = _owners(offsets)
    A_p, rho_p = np.asarray(A_p, float), np.asarray(rho_p, float)
    Aq, rq = _pair_nodal(np.asarray(A, float), tri_idx), _pair_nodal(np.asarray(rho, float), tri_idx)
    f = rq * (Aq / rq ** 2 + (A_p / rho_p ** 2)[own][None, :])
    gx, gy = _pair_gradient(kernel_id, h, px, py, tri, f, offsets, tri_idx, nthreads)
    return rho_p * gx, rho_p * gy


def divergence_curl(kernel_id, h, px, py, tri, Ax, Ay, offsets, tri_idx, nthreads=0):
    """div = <grad A_x>_x + <grad A_y>_y, curl = <grad A_y>_x - <grad A_x>_y."""
    _, gxx, gxy = integrate(kernel_id, h, px, py, tri, Ax, offsets, tri_idx, nthreads=nthreads)
    _, gyx, gyy = integrate(kernel_id, h, px, py, tri, Ay, offsets, tri_idx, nthreads=nthreads)
    return gxx + gyy, gyx - gxy


def boundary_normal(kernel_id, h, px, py, tri, offsets, tri_idx, nthreads=0):
    """n(x) = int grad W over the boundary triangles (unit field)."""
    tri = np.asarray(tri, dtype=np.float64)
    _, nx, ny = integrate(kernel_id, h, px, py, tri, np.ones((1, tri.shape[1])), offsets, tri_idx,
                          nthreads=nthreads)
    return nx, ny


def pressure_contact(kernel_id, h, rho0, px, py, p_particle, rho_particle, tri, offsets, tri_idx, p_pair,
                     nthreads=0):
    """Boundary pressure acceleration with one pressure value per contact (App. A, second choice):
    a_i = - sum_q rho0 (p_q / rho0^2 + p_i / rho_i^2) int_T grad W, the field of pair q constant."""
    own = _owners(offsets)
    p_particle, rho_particle = np.asarray(p_particle, float), np.asarray(rho_particle, float)
    f = rho0 * (np.asarray(p_pair, float) / rho0 ** 2 + (p_particle / rho_particle ** 2)[own])
    gx, gy = _pair_gradient(kernel_id, h, px, py, tri, f[None, :], offsets, tri_idx, nthreads)
    return -gx, -gy
