"""Incompressible SPH with the closed-form boundary integrals (App. A).

A small 2D solver in the style of the divergence-free SPH family (Bender and
Koschier's constant-density solver with a Jacobi iteration on the stiffness
kappa = p / rho), whose boundary is a triangle mesh of the solid region handled
by the library's integrals instead of boundary particles:

* density (Sec. 2, the boundary's volume contribution):
  rho_i = sum_j m W_ij + rho_0 int_B W(x_i - x') dx'  (``sphbi_integrate`` with a
  unit P0 field: its I);
* the boundary's share of the density change: rho_0 v_i . int_B grad W (its G);
* the boundary pressure acceleration (App. A, one pressure per contact):
  a_i^b = -rho_0 (p_b / rho_0^2 + p_i / rho_i^2) int_T grad W
  (``sphbi_pressure_contact``), with p_b the contact pressure.  App. A takes p_b
  from a moving-least-squares fit of the fluid pressure at the contact point;
  here it is the particle's own pressure mirrored onto the wall (p_b = p_i), the
  zeroth-order version of that fit.

The fluid-fluid sums are plain tensor arithmetic over a padded neighbour table
(summed along the table, so results are deterministic).  The boundary terms go
through a provider object with two methods, so that a test can substitute the
definition oracle for the library:

    provider.update(px, py)            -> (B, Bx, By) per particle
    provider.pressure_accel(p, rho)    -> (ax, ay) per particle

This is a demonstration of the coupling, not a production solver: no
divergence-free pass, XSPH smoothing in place of a viscosity, a time step
limited by the fastest particle.
"""
from __future__ import annotations

import math

import torch

from . import PairList, integrate, kernel_preset, pressure_contact


class LibraryBoundary:
    """Boundary terms of a static triangle mesh (the solid region) from the
    library: pair list, the unit-field integrals and the contact pressure."""

    def __init__(self, kernel: int, h: float, rho0: float, tri: torch.Tensor):
        self.kernel, self.h, self.rho0 = kernel, float(h), float(rho0)
        self.tri = tri.to(torch.float64)
        self.ones = torch.ones((1, self.tri.shape[1]), dtype=torch.float64, device=self.tri.device)
        self.pairs = PairList(self.tri, self.h)
        self.off = self.idx = None
        self.px = self.py = None

    def update(self, px, py):
        self.px, self.py = px, py
        self.off, self.idx = self.pairs(px, py)
        return integrate(self.kernel, self.h, px, py, self.tri, self.ones, self.off, self.idx)

    def pressure_accel(self, p, rho):
        owner = torch.repeat_interleave(torch.arange(p.numel(), device=p.device), self.off[1:] - self.off[:-1])
        return pressure_contact(self.kernel, self.h, self.rho0, self.px, self.py, p, rho, self.tri, self.off,
                                self.idx, p[owner])


class FluidKernel:
    """W(r) = c_d h^-2 k(r/h) and its gradient from the preset's monomial coefficients."""

    def __init__(self, kernel: int, h: float):
        K = kernel_preset(kernel)
        if K.n_pieces != 1:
            raise ValueError("the fluid kernel must be one polynomial piece")
        self.b = [K.b[0][i] for i in range(K.degree[0] + 1)]
        self.cd, self.h = K.c_d, float(h)

    def w(self, r):
        q = r / self.h
        k = torch.zeros_like(q)
        for c in reversed(self.b):
            k = k * q + c
        return torch.where(q < 1.0, self.cd / self.h ** 2 * k, torch.zeros_like(q))

    def dw_over_r(self, r):
        """W'(r) / r (zero at r = 0 and beyond the support)."""
        q = r / self.h
        dk = torch.zeros_like(q)
        for i in range(len(self.b) - 1, 0, -1):
            dk = dk * q + i * self.b[i]
        safe = torch.where(r > 0, r, torch.ones_like(r))
        return torch.where((q < 1.0) & (r > 0), self.cd / self.h ** 3 * dk / safe, torch.zeros_like(q))


class DFSPH:
    """Particles x [N, 2] with velocities v, spacing dx (mass rho0 dx^2),
    support h, gravity g; the boundary provider supplies the wall terms."""

    def __init__(self, x, dx, h, rho0, boundary, kernel: int = 0, g=(0.0, -9.81), max_iter: int = 100,
                 tol: float = 1e-3, xsph: float = 0.05):
        self.x = x.to(torch.float64).clone()
        self.v = torch.zeros_like(self.x)
        self.h, self.rho0, self.dx = float(h), float(rho0), float(dx)
        self.bnd = boundary
        self.W = FluidKernel(kernel, h)
        self.g = torch.tensor(g, dtype=torch.float64, device=self.x.device)
        self.max_iter, self.tol, self.xsph = max_iter, tol, xsph
        self.w0 = float(self.W.w(torch.zeros(1, dtype=torch.float64)).item())
        # the particle mass that gives an interior particle of the initial
        # lattice the rest density (the kernel sum over a lattice of spacing
        # dx is not exactly 1/dx^2)
        nb, mask = self.neighbours()
        xij = self.x[:, None, :] - self.x[nb]
        rij = torch.sqrt((xij * xij).sum(-1))
        lattice = (torch.where(mask, self.W.w(rij), torch.zeros_like(rij)).sum(1) + self.w0).max()
        self.m = float(rho0 / lattice.item()) if len(self.x) > 1 else rho0 * dx * dx

    # ---------------------------------------------------------------- neighbours
    def neighbours(self):
        """Padded table nb [N, K] of the other particles within h (ascending
        index; padding repeats the particle itself with mask False)."""
        x, h2 = self.x, self.h * self.h
        N = x.shape[0]
        d = x[:, None, :] - x[None, :, :]
        r2 = (d * d).sum(-1)
        close = (r2 < h2) & ~torch.eye(N, dtype=torch.bool, device=x.device)
        cnt = close.sum(1)
        K = max(int(cnt.max().item()), 1)
        i, j = torch.nonzero(close, as_tuple=True)           # row-major: sorted by i, then j
        start = torch.cumsum(cnt, 0) - cnt
        slot = torch.arange(i.numel(), device=x.device) - start[i]
        nb = torch.arange(N, device=x.device)[:, None].repeat(1, K)
        mask = torch.zeros((N, K), dtype=torch.bool, device=x.device)
        nb[i, slot] = j
        mask[i, slot] = True
        return nb, mask

    # ---------------------------------------------------------------- one step
    def relax(self, steps: int, dt: float):
        """Moves the particles towards rest density without gravity, dropping
        the velocity after every step (the usual relaxation of an initial
        lattice: next to a wall the lattice sum and the wall's volume integral
        overlap by a few per cent)."""
        g = self.g
        self.g = torch.zeros_like(g)
        for _ in range(steps):
            self.step(dt)
            self.v.zero_()
        self.g = g

    def step(self, dt: float, cfl: float = 0.25):
        """Advances by dt, or by the shorter step that keeps the fastest
        particle within cfl * dx of its start (dx the lattice spacing);
        returns (step taken, iterations, mean relative density error after
        the solve, largest speed)."""
        x, m = self.x, self.m
        vmax0 = float(torch.sqrt((self.v * self.v).sum(-1)).max().item()) if len(x) else 0.0
        if vmax0 > 0.0:
            dt = min(dt, cfl * self.dx / vmax0)
        nb, mask = self.neighbours()
        xij = x[:, None, :] - x[nb]                            # [N, K, 2]
        rij = torch.sqrt((xij * xij).sum(-1))
        wij = torch.where(mask, self.W.w(rij), torch.zeros_like(rij))
        gij = torch.where(mask[..., None], self.W.dw_over_r(rij)[..., None] * xij, torch.zeros_like(xij))
        B, Bx, By = self.bnd.update(x[:, 0].contiguous(), x[:, 1].contiguous())
        gB = torch.stack([Bx, By], -1)
        rho = m * (wij.sum(1) + self.w0) + self.rho0 * B
        s = m * gij.sum(1) + self.rho0 * gB
        alpha = rho / ((s * s).sum(-1) + (m * m * (gij * gij).sum(-1)).sum(1) + 1e-30)
        v = self.v + dt * self.g
        it, err = 0, 0.0
        for it in range(1, self.max_iter + 1):
            vij = v[:, None, :] - v[nb]
            drho = m * (vij * gij).sum(-1).sum(1) + self.rho0 * (v * gB).sum(-1)
            rho_star = rho + dt * drho
            err = float(torch.clamp(rho_star - self.rho0, min=0.0).mean().item()) / self.rho0
            kappa = torch.clamp(rho_star - self.rho0, min=0.0) / (dt * dt) * alpha
            kr = kappa / rho
            dv = m * ((kr[:, None] + kr[nb])[..., None] * gij).sum(1)
            ax, ay = self.bnd.pressure_accel(kappa * rho, rho)   # p = kappa rho
            v = v - dt * dv + dt * torch.stack([ax, ay], -1)
            if it >= 2 and err < self.tol:
                break
        if self.xsph > 0.0:
            # XSPH velocity smoothing (fluid neighbours only), for the noise
            # of an inviscid solver
            vij = v[nb] - v[:, None, :]
            v = v + self.xsph * (m / rho[nb])[..., None].mul(wij[..., None] * vij).sum(1)
        self.v = v
        self.x = x + dt * v
        return dt, it, err, float(torch.sqrt((v * v).sum(-1)).max().item())


def corner_boundary(width: float, height: float, thickness: float, device="cpu"):
    """The solid region of an open box [0, width] x [0, inf): floor and two
    walls of the given thickness (up to `height`), six triangles, non-
    overlapping.  Returns tri [6, 6] (rows x0 y0 x1 y1 x2 y2)."""
    d = thickness
    rects = [(-d, -d, width + d, 0.0),            # floor, under both walls
             (-d, 0.0, 0.0, height),             # left wall
             (width, 0.0, width + d, height)]    # right wall
    cols = []
    for (x0, y0, x1, y1) in rects:
        cols.append([x0, y0, x1, y0, x1, y1])
        cols.append([x0, y0, x1, y1, x0, y1])
    return torch.tensor(cols, dtype=torch.float64, device=device).T.contiguous()


def fluid_block(x0: float, y0: float, nx: int, ny: int, dx: float, device="cpu"):
    """Particles on a regular grid (cell centres) of nx x ny cells of size dx."""
    gx = x0 + dx * (torch.arange(nx, dtype=torch.float64) + 0.5)
    gy = y0 + dx * (torch.arange(ny, dtype=torch.float64) + 0.5)
    X, Y = torch.meshgrid(gx, gy, indexing="ij")
    return torch.stack([X.reshape(-1), Y.reshape(-1)], -1).to(device)


def stable_dt(dx: float, height: float, g: float = 9.81, cfl: float = 0.25) -> float:
    """A fixed step from the largest free-fall speed over the column height."""
    return cfl * dx / math.sqrt(2.0 * g * height)
