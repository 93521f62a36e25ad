"""Seeded synthetic inputs for the boundary-integral path.

This module only builds geometry and nodal values (particles, triangle
meshes, field samples, cotangents).  It contains none of the integration
arithmetic, so both the device path and the CPU oracle can take their inputs
from here without sharing any of the method.

Conventions shared by every generator (they are interface conventions, not
method arithmetic):

* particle positions ``px``, ``py``: float64 ``[N]``;
* triangles ``tri``: float64 ``[6, T]`` structure-of-arrays holding
  ``x0, y0, x1, y1, x2, y2``;
* nodal field values ``nodal``: float64 ``[n_nodes, T]`` with ``n_nodes`` 1
  (per-triangle constant), 3 (per-vertex, linear) or 10 (cubic Lagrange).
  Cubic node order: v0, v1, v2; the points at 1/3 and 2/3 of edge v0->v1;
  of edge v1->v2; of edge v2->v0; the centroid;
* ``h`` is the support radius of the kernel (the kernel vanishes for
  ``|x - x'| >= h``).

The recipes follow the workloads described for the paper's setting (a wall
band around a box, a covering boundary mesh with perturbed vertices, sliver
triangles with particles placed next to edges and vertices).  All randomness
comes from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

# Kernel identifiers (same numbering as the C header).
WENDLAND_C2 = 0
WENDLAND_C4 = 1
WENDLAND_C6 = 2
CUBIC_BSPLINE = 3
KERNEL_NAMES = {WENDLAND_C2: "wendland_c2", WENDLAND_C4: "wendland_c4",
                WENDLAND_C6: "wendland_c6", CUBIC_BSPLINE: "cubic_bspline"}


@dataclass
class Workload:
    name: str
    px: np.ndarray
    py: np.ndarray
    tri: np.ndarray          # [6, T]
    nodal: np.ndarray        # [n_nodes, T]
    h: float
    kernel: int
    meta: dict = field(default_factory=dict)

    @property
    def n_particles(self) -> int:
        return int(self.px.shape[0])

    @property
    def n_triangles(self) -> int:
        return int(self.tri.shape[1])

    @property
    def n_nodes(self) -> int:
        return int(self.nodal.shape[0])


# ---------------------------------------------------------------------------
# geometry helpers (input construction only)
# ---------------------------------------------------------------------------

def _tri_quality(tri: np.ndarray):
    """Signed doubled area and aspect ratio l_max^2 / (2 area) per triangle."""
    x0, y0, x1, y1, x2, y2 = tri
    area2 = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)
    l2 = np.maximum.reduce([(x1 - x0) ** 2 + (y1 - y0) ** 2,
                            (x2 - x1) ** 2 + (y2 - y1) ** 2,
                            (x0 - x2) ** 2 + (y0 - y2) ** 2])
    with np.errstate(divide="ignore"):
        ar = l2 / np.abs(area2)
    return area2, ar


def _square_ring(lo: float, hi: float, per_side: int) -> np.ndarray:
    """Points on the boundary of [lo,hi]^2, counter-clockwise from (lo,lo)."""
    t = np.arange(per_side) / per_side
    w = hi - lo
    pts = [np.stack([lo + w * t, np.full_like(t, lo)], 1),
           np.stack([np.full_like(t, hi), lo + w * t], 1),
           np.stack([hi - w * t, np.full_like(t, hi)], 1),
           np.stack([np.full_like(t, lo), hi - w * t], 1)]
    return np.concatenate(pts, 0)


def cubic_node_positions(tri: np.ndarray) -> np.ndarray:
    """Positions [10, 2, T] of the cubic Lagrange nodes in the documented order."""
    v = [tri[0:2], tri[2:4], tri[4:6]]
    nodes = [v[0], v[1], v[2]]
    for a, b in ((0, 1), (1, 2), (2, 0)):
        nodes.append(v[a] + (v[b] - v[a]) / 3.0)
        nodes.append(v[a] + 2.0 * (v[b] - v[a]) / 3.0)
    nodes.append((v[0] + v[1] + v[2]) / 3.0)
    return np.stack(nodes, 0)


def vertex_positions(tri: np.ndarray) -> np.ndarray:
    return np.stack([tri[0:2], tri[2:4], tri[4:6]], 0)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def band_wall(seed: int = 1, n_particles: int = 1024, h: float = 0.1,
              per_side: int = 16, width: float = 0.15,
              kernel: int = WENDLAND_C2, field_order: int = 0) -> Workload:
    """Unit box with a wall band of the given width triangulated around it.

    The inner square [0,1]^2 and the outer square [-w,1+w]^2 each carry
    ``4*per_side`` boundary points (counter-clockwise from the corner);
    trapezoid i between inner points I_i, I_{i+1} and outer points O_i,
    O_{i+1} becomes triangles (I_i, O_i, O_{i+1}) and (I_i, O_{i+1}, I_{i+1}).
    Particles are uniform in [0,1]^2.
    """
    rng = np.random.default_rng(seed)
    inner = _square_ring(0.0, 1.0, per_side)
    outer = _square_ring(-width, 1.0 + width, per_side)
    m = inner.shape[0]
    tris = []
    for i in range(m):
        j = (i + 1) % m
        tris.append([*inner[i], *outer[i], *outer[j]])
        tris.append([*inner[i], *outer[j], *inner[j]])
    tri = np.ascontiguousarray(np.array(tris, dtype=np.float64).T)
    p = rng.uniform(0.0, 1.0, size=(n_particles, 2))
    nodal = _field(rng, tri, field_order)
    return Workload("band_wall", np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1]),
                    tri, nodal, float(h), kernel,
                    meta={"seed": seed, "per_side": per_side, "width": width,
                          "field_order": field_order})


def _field(rng, tri: np.ndarray, field_order: int, constant: float = 1.0) -> np.ndarray:
    T = tri.shape[1]
    if field_order == 0:
        return np.full((1, T), constant, dtype=np.float64)
    n = {1: 3, 3: 10}[field_order]
    return rng.standard_normal((n, T))


def covering_mesh(nx: int, ny: int, seed: int, ar_target: float = 20.0,
                  domain=(0.0, 1.0)) -> np.ndarray:
    """Triangulated [lo,hi]^2 (nx*ny cells, 2 triangles each) with perturbed vertices.

    Cell diagonals alternate with the parity of (i + j).  Interior vertices
    move by a seeded uniform offset; boundary vertices slide along the
    boundary and corners stay.  The offset amplitude is bisected so the
    largest aspect ratio l_max^2/(2 area) lands at ``ar_target`` with no
    inverted triangle.
    """
    lo, hi = domain
    rng = np.random.default_rng(seed)
    xs = np.linspace(lo, hi, nx + 1)
    ys = np.linspace(lo, hi, ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="ij")          # [nx+1, ny+1]
    dx, dy = (hi - lo) / nx, (hi - lo) / ny
    nz = rng.uniform(-1.0, 1.0, size=(2, nx + 1, ny + 1))
    nz[0, 0, :] = 0.0
    nz[0, -1, :] = 0.0
    nz[1, :, 0] = 0.0
    nz[1, :, -1] = 0.0

    vid = np.arange((nx + 1) * (ny + 1)).reshape(nx + 1, ny + 1)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    a = vid[i, j]
    b = vid[i + 1, j]
    c = vid[i + 1, j + 1]
    d = vid[i, j + 1]
    even = ((i + j) % 2) == 0
    t1 = np.where(even[:, None], np.stack([a, b, c], 1), np.stack([a, b, d], 1))
    t2 = np.where(even[:, None], np.stack([a, c, d], 1), np.stack([b, c, d], 1))
    conn = np.concatenate([t1, t2], 0)                 # [T, 3] counter-clockwise

    def build(amp):
        VX = (X + amp * dx * nz[0]).ravel()
        VY = (Y + amp * dy * nz[1]).ravel()
        tri = np.stack([VX[conn[:, 0]], VY[conn[:, 0]], VX[conn[:, 1]], VY[conn[:, 1]],
                        VX[conn[:, 2]], VY[conn[:, 2]]], 0)
        area2, ar = _tri_quality(tri)
        return tri, area2, ar

    tri0, _, ar0 = build(0.0)
    if ar_target is None or ar0.max() >= ar_target:
        return np.ascontiguousarray(tri0)
    lo_a, hi_a = 0.0, 0.5
    best = tri0
    for _ in range(60):
        mid = 0.5 * (lo_a + hi_a)
        tri, area2, ar = build(mid)
        if np.all(area2 > 0) and ar.max() <= ar_target:
            lo_a, best = mid, tri
        else:
            hi_a = mid
    return np.ascontiguousarray(best)


def jittered_grid(n_side: int, seed: int, jitter: float = 0.3, domain=(0.0, 1.0)):
    """Particles at cell centres of an n_side^2 grid with uniform jitter (fraction of dx)."""
    lo, hi = domain
    rng = np.random.default_rng(seed)
    dx = (hi - lo) / n_side
    c = lo + (np.arange(n_side) + 0.5) * dx
    X, Y = np.meshgrid(c, c, indexing="ij")
    j = rng.uniform(-jitter * dx, jitter * dx, size=(2, n_side, n_side))
    return (np.ascontiguousarray((X + j[0]).ravel()), np.ascontiguousarray((Y + j[1]).ravel()), dx)


def covering_workload(n_side: int = 1024, nx: int = 128, ny: int = 256, seed: int = 2,
                      kernel: int = WENDLAND_C2, field_order: int = 3,
                      ar_target: float = 20.0, h_factor: float = 2.5) -> Workload:
    """Particles on a jittered grid over [0,1]^2 and a covering perturbed mesh.

    h = h_factor * dx with dx = 1/n_side.  Field values per triangle are
    standard normal (P1/P3) or 1 (P0).
    """
    px, py, dx = jittered_grid(n_side, seed)
    tri = covering_mesh(nx, ny, seed + 1000, ar_target)
    rng = np.random.default_rng(seed + 2000)
    nodal = _field(rng, tri, field_order)
    return Workload(f"covering_{n_side}x{n_side}_{tri.shape[1]}", px, py, tri, nodal,
                    float(h_factor * dx), kernel,
                    meta={"seed": seed, "n_side": n_side, "nx": nx, "ny": ny,
                          "ar_target": ar_target, "field_order": field_order})


def sliver_stress(seed: int = 3, grid: int = 128, h: float = 1.0 / 512,
                  kernel: int = WENDLAND_C2, field_order: int = 0,
                  min_angle_deg: float = 0.5, per_tri_edge: int = 8,
                  per_tri_vertex: int = 8, delta_range=(1e-8, 1e-2)) -> Workload:
    """Sliver triangles (one per 4h cell) with particles hugging edges and vertices.

    Each triangle has a smallest angle of exactly ``min_angle_deg``, a second
    angle uniform in [min_angle, 90] degrees, a longest edge uniform in
    [0.5h, 2h] and a random rotation.  Per triangle, ``per_tri_edge``
    particles sit at normal offset +-delta from a random point (t in
    (0.05, 0.95)) of a random edge and ``per_tri_vertex`` particles at
    distance delta from a random vertex in a random direction; delta is
    log-uniform in ``delta_range`` times h.  Cells are 4h wide, so each
    particle sees exactly one triangle.
    """
    rng = np.random.default_rng(seed)
    n = grid * grid
    cell = 4.0 * h
    A = np.deg2rad(min_angle_deg)
    B = np.deg2rad(rng.uniform(min_angle_deg, 90.0, size=n))
    C = np.pi - A - B
    L = rng.uniform(0.5 * h, 2.0 * h, size=n)
    sA, sB, sC = np.sin(A), np.sin(B), np.sin(C)
    k = L / np.maximum(np.maximum(sA, sB), sC)
    b = k * sB                        # side between P_A and P_C
    c = k * sC                        # side between P_A and P_B
    P = np.zeros((3, 2, n))
    P[1, 0] = c
    P[2, 0] = b * np.cos(A)
    P[2, 1] = b * np.sin(A)
    cen = P.mean(0)
    P -= cen[None]
    rot = rng.uniform(0, 2 * np.pi, size=n)
    cr, sr = np.cos(rot), np.sin(rot)
    R = np.empty_like(P)
    R[:, 0] = cr * P[:, 0] - sr * P[:, 1]
    R[:, 1] = sr * P[:, 0] + cr * P[:, 1]
    gi, gj = np.meshgrid(np.arange(grid), np.arange(grid), indexing="ij")
    ctr = np.stack([(gi.ravel() + 0.5) * cell, (gj.ravel() + 0.5) * cell], 0)
    R += ctr[None]
    tri = np.ascontiguousarray(np.stack([R[0, 0], R[0, 1], R[1, 0], R[1, 1], R[2, 0], R[2, 1]], 0))

    lo, hi = np.log(delta_range[0]), np.log(delta_range[1])
    m = per_tri_edge + per_tri_vertex
    delta = np.exp(rng.uniform(lo, hi, size=(n, m))) * h
    pts = np.empty((n, m, 2))
    # near edges
    e = rng.integers(0, 3, size=(n, per_tri_edge))
    t = rng.uniform(0.05, 0.95, size=(n, per_tri_edge))
    sgn = rng.choice([-1.0, 1.0], size=(n, per_tri_edge))
    idx = np.arange(n)[:, None]
    va = R[e, :, idx]                                  # [n, pe, 2]
    vb = R[(e + 1) % 3, :, idx]
    d = vb - va
    nrm = np.stack([-d[..., 1], d[..., 0]], -1) / np.linalg.norm(d, axis=-1, keepdims=True)
    pts[:, :per_tri_edge] = va + t[..., None] * d + (sgn * delta[:, :per_tri_edge])[..., None] * nrm
    # near vertices
    vv = rng.integers(0, 3, size=(n, per_tri_vertex))
    ang = rng.uniform(0, 2 * np.pi, size=(n, per_tri_vertex))
    vp = R[vv, :, idx]
    dv = delta[:, per_tri_edge:]
    pts[:, per_tri_edge:, 0] = vp[..., 0] + dv * np.cos(ang)
    pts[:, per_tri_edge:, 1] = vp[..., 1] + dv * np.sin(ang)
    px = np.ascontiguousarray(pts[..., 0].ravel())
    py = np.ascontiguousarray(pts[..., 1].ravel())
    nodal = _field(np.random.default_rng(seed + 2000), tri, field_order)
    return Workload(f"sliver_{KERNEL_NAMES[kernel]}_p{field_order}", px, py, tri, nodal, float(h),
                    kernel, meta={"seed": seed, "grid": grid, "min_angle_deg": min_angle_deg,
                                  "field_order": field_order})


def box_mesh_8() -> np.ndarray:
    """[-1,1]^2 split into 8 triangles (4 quadrants, each cut by a diagonal)."""
    tris = []
    for (x0, y0) in ((-1, -1), (0, -1), (-1, 0), (0, 0)):
        a = (x0, y0); b = (x0 + 1, y0); c = (x0 + 1, y0 + 1); d = (x0, y0 + 1)
        tris.append([*a, *b, *c])
        tris.append([*a, *c, *d])
    return np.ascontiguousarray(np.array(tris, dtype=np.float64).T)


def box_mesh_random(mx: int = 6, my: int = 8, seed: int = 0, jitter: float = 0.25) -> np.ndarray:
    """[-1,1]^2 triangulated into 2*mx*my triangles with jittered interior vertices."""
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid(np.linspace(-1, 1, mx + 1), np.linspace(-1, 1, my + 1), indexing="ij")
    dx, dy = 2.0 / mx, 2.0 / my
    J = rng.uniform(-jitter, jitter, size=(2, mx + 1, my + 1))
    J[:, 0, :] = 0; J[:, -1, :] = 0; J[:, :, 0] = 0; J[:, :, -1] = 0
    X = X + J[0] * dx
    Y = Y + J[1] * dy
    tris = []
    for i in range(mx):
        for j in range(my):
            a = (X[i, j], Y[i, j]); b = (X[i + 1, j], Y[i + 1, j])
            c = (X[i + 1, j + 1], Y[i + 1, j + 1]); e = (X[i, j + 1], Y[i, j + 1])
            tris.append([*a, *b, *c])
            tris.append([*a, *c, *e])
    return np.ascontiguousarray(np.array(tris, dtype=np.float64).T)


def random_pairs(n: int, seed: int, spread: float = 1.6, scale_range=(0.05, 2.5)):
    """Random single triangles around a particle at the origin (support 1).

    Returns ``tri`` [6, n] in the support-normalised frame.  Vertex sets mix
    tiny, moderate and large triangles so that every clipping case (0..3
    vertices inside, 0..3 edges crossing, origin inside or outside) occurs.
    """
    rng = np.random.default_rng(seed)
    c = rng.uniform(-spread, spread, size=(n, 2))
    s = np.exp(rng.uniform(np.log(scale_range[0]), np.log(scale_range[1]), size=(n, 1)))
    v = c[:, None, :] + s[:, :, None] * rng.uniform(-1, 1, size=(n, 3, 2))
    return np.ascontiguousarray(v.reshape(n, 6).T)


def surrogate_pairs(n: int, seed: int, n_side: int = 256, nx: int = 32, ny: int = 64):
    """(particle, triangle) candidate geometry for surrogate training/evaluation.

    Builds covering meshes + jittered particles at the given seed; the caller
    enumerates in-support pairs with the library and keeps up to ``n``.
    """
    return covering_workload(n_side=n_side, nx=nx, ny=ny, seed=seed, field_order=0)
