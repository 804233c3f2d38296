"""Plain CPU reference for the steps either side of the pressure solve.

TEST INFRASTRUCTURE ONLY (see the package docstring): only the test suite,
the smoke check and the benchmark's CPU baseline leg may use it.

What it computes, on a periodic n x n grid with the duplicated seam (unique
nodes 0 .. n-2, spacing h = 1/(n-1), x along the columns, y along the rows):

  * the source of the pressure-Poisson equation with zero viscosity
    (Section 2.3, Eq. for f(x, y); the second line of the momentum system in
    Section 2.1): f = -div((u . grad) u);
  * the explicit Euler step of the momentum equation (first line of that
    system): u <- u - dt ((u . grad) u + grad p);
  * the time step that chains them around the pressure solve: the source,
    then p from Laplacian p = f, then the velocity step.  The Poisson solver
    here (as in the library) solves A q = f with A = -Laplacian_h, so the
    pressure of the momentum equation is p = -q.

Readings (the paper gives neither discretisation): every derivative is the
second-order central difference d/dx a[i, j] = (a[i, j+1] - a[i, j-1]) / (2h)
(likewise d/dy along the rows), applied to the nodal velocities; the
convective term c = (u . grad) u has components u_x du_x/dx + u_y du_x/dy
and u_x du_y/dx + u_y du_y/dy; f = -(dc_x/dx + dc_y/dy).  Outputs carry the
seam.  numpy in float64; np.roll supplies the periodic neighbours.
"""

from __future__ import annotations

import numpy as np


def _unique(a: np.ndarray) -> np.ndarray:
    return np.asarray(a, dtype=np.float64)[:-1, :-1]


def _with_seam(a: np.ndarray) -> np.ndarray:
    return np.pad(a, ((0, 1), (0, 1)), mode="wrap")


def ddx(a: np.ndarray, h: float) -> np.ndarray:
    """Central difference along x (columns) of periodic unique nodes."""
    return (np.roll(a, -1, axis=1) - np.roll(a, 1, axis=1)) / (2.0 * h)


def ddy(a: np.ndarray, h: float) -> np.ndarray:
    """Central difference along y (rows) of periodic unique nodes."""
    return (np.roll(a, -1, axis=0) - np.roll(a, 1, axis=0)) / (2.0 * h)


def convection(ux: np.ndarray, uy: np.ndarray, h: float):
    """(u . grad) u on unique nodes: (u_x d/dx + u_y d/dy) applied to each
    component."""
    cx = ux * ddx(ux, h) + uy * ddy(ux, h)
    cy = ux * ddx(uy, h) + uy * ddy(uy, h)
    return cx, cy


def ns_rhs(ux: np.ndarray, uy: np.ndarray) -> np.ndarray:
    """f = -div((u . grad) u) on an (n, n) periodic grid with seam."""
    n = ux.shape[0]
    h = 1.0 / (n - 1)
    cx, cy = convection(_unique(ux), _unique(uy), h)
    return _with_seam(-(ddx(cx, h) + ddy(cy, h)))


def ns_update(ux: np.ndarray, uy: np.ndarray, p: np.ndarray, dt: float):
    """One explicit Euler step u - dt ((u . grad) u + grad p); returns the
    new (u_x, u_y) with seams."""
    n = ux.shape[0]
    h = 1.0 / (n - 1)
    U, V, P = _unique(ux), _unique(uy), _unique(p)
    cx, cy = convection(U, V, h)
    return (_with_seam(U - dt * (cx + ddx(P, h))), _with_seam(V - dt * (cy + ddy(P, h))))


def time_step(ux: np.ndarray, uy: np.ndarray, dt: float, solve):
    """One projection time step (Section 2.1's system with Section 2.3's
    source): f = -div((u . grad) u); q = solve(f), the solution of
    -Laplacian_h q = f; p = -q, so that Laplacian_h p = f; then the
    explicit Euler step with grad p.  Returns (u_x, u_y, p)."""
    f = ns_rhs(ux, uy)
    p = -np.asarray(solve(f), dtype=np.float64)
    vx, vy = ns_update(ux, uy, p, dt)
    return vx, vy, p
