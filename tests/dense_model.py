"""Dense linear-algebra model of the 2-D Poisson multigrid pieces.

Test-only.  Built from library routines and matrix definitions, not from the
oracle's code: the operator is assembled with Kronecker products, a
Gauss-Seidel half-sweep is the block solve of its matrix splitting, full
weighting is a quarter of the transposed bilinear interpolation, the
prolongation is scipy's CubicSpline applied to unit vectors, and the coarsest
solve is numpy's solve / pinv.  Vectors hold the unknown nodes in row-major
order (Dirichlet: interior nodes; periodic: the n-1 unique nodes per side).
"""

from __future__ import annotations

import functools

import numpy as np
import scipy.fft
from scipy.interpolate import CubicSpline

DIRICHLET = 0
PERIODIC = 1


def m_of(n: int, bc: int) -> int:
    """Unknowns per side."""
    return n - 2 if bc == DIRICHLET else n - 1


def to_vec(a: np.ndarray, bc: int) -> np.ndarray:
    return (a[1:-1, 1:-1] if bc == DIRICHLET else a[:-1, :-1]).reshape(-1).copy()


def to_grid(v: np.ndarray, n: int, bc: int) -> np.ndarray:
    m = m_of(n, bc)
    g = np.zeros((n, n), dtype=v.dtype)
    core = v.reshape(m, m)
    if bc == DIRICHLET:
        g[1:-1, 1:-1] = core
    else:
        g[:-1, :-1] = core
        g[-1, :-1] = core[0]
        g[:-1, -1] = core[:, 0]
        g[-1, -1] = core[0, 0]
    return g


@functools.lru_cache(maxsize=None)
def second_difference(m: int, bc: int) -> np.ndarray:
    """1-D matrix of -d^2/dx^2 times h^2: tridiag(-1, 2, -1), circulant if periodic."""
    T = 2.0 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)
    if bc == PERIODIC:
        T[0, -1] -= 1.0
        T[-1, 0] -= 1.0
    return T


@functools.lru_cache(maxsize=None)
def operator(n: int, bc: int) -> np.ndarray:
    """A = -Delta_h = (T x I + I x T) / h^2 on the unknowns."""
    m = m_of(n, bc)
    T = second_difference(m, bc)
    I = np.eye(m)
    return (np.kron(T, I) + np.kron(I, T)) * float(n - 1) ** 2


@functools.lru_cache(maxsize=None)
def colour_mask(n: int, bc: int, colour: int) -> np.ndarray:
    m = m_of(n, bc)
    off = 1 if bc == DIRICHLET else 0
    i, j = np.meshgrid(np.arange(m) + off, np.arange(m) + off, indexing="ij")
    return (((i + j) % 2) == colour).reshape(-1)


def half_sweep(u: np.ndarray, f: np.ndarray, n: int, bc: int, colour: int) -> np.ndarray:
    """Block solve of the matrix splitting for one colour: the colour's rows of
    A u = f are solved exactly with the other colour held fixed."""
    A = operator(n, bc)
    c = colour_mask(n, bc, colour)
    o = ~c
    out = u.copy()
    Acc = A[np.ix_(c, c)]
    out[c] = np.linalg.solve(Acc, f[c] - A[np.ix_(c, o)] @ u[o])
    return out


@functools.lru_cache(maxsize=None)
def bilinear_interp(nc: int, bc: int) -> np.ndarray:
    """Bilinear interpolation from coarse unknowns to fine unknowns."""
    n = 2 * (nc - 1) + 1
    if bc == DIRICHLET:
        P1 = np.zeros((n, nc))
        for k in range(nc):
            P1[2 * k, k] = 1.0
            if k + 1 < nc:
                P1[2 * k + 1, k] = 0.5
                P1[2 * k + 1, k + 1] = 0.5
        P1 = P1[1:-1, 1:-1]
    else:
        mc = nc - 1
        P1 = np.zeros((2 * mc, mc))
        for k in range(mc):
            P1[2 * k, k] = 1.0
            P1[2 * k + 1, k] = 0.5
            P1[2 * k + 1, (k + 1) % mc] = 0.5
    return np.kron(P1, P1)


@functools.lru_cache(maxsize=None)
def full_weighting(n: int, bc: int) -> np.ndarray:
    """Full weighting as a quarter of the transposed bilinear interpolation."""
    nc = (n - 1) // 2 + 1
    return 0.25 * bilinear_interp(nc, bc).T


@functools.lru_cache(maxsize=None)
def spline_1d(nc: int, bc: int) -> np.ndarray:
    """1-D cubic-spline interpolation matrix (coarse unknowns -> fine unknowns)
    by applying scipy's CubicSpline to unit vectors."""
    n = 2 * (nc - 1) + 1
    xc = np.arange(nc, dtype=np.float64)
    xf = np.arange(n, dtype=np.float64) / 2.0
    if bc == DIRICHLET:
        cols = []
        for k in range(1, nc - 1):
            y = np.zeros(nc)
            y[k] = 1.0
            cols.append(CubicSpline(xc, y, bc_type="natural")(xf)[1:-1])
        return np.array(cols).T
    mc = nc - 1
    cols = []
    for k in range(mc):
        y = np.zeros(nc)
        y[k] = 1.0
        if k == 0:
            y[-1] = 1.0
        cols.append(CubicSpline(xc, y, bc_type="periodic")(xf)[:-1])
    return np.array(cols).T


@functools.lru_cache(maxsize=None)
def spline_prolong(nc: int, bc: int) -> np.ndarray:
    P1 = spline_1d(nc, bc)
    return np.kron(P1, P1)


@functools.lru_cache(maxsize=None)
def coarsest_inverse(bc: int) -> np.ndarray:
    A = operator(5, bc)
    return np.linalg.inv(A) if bc == DIRICHLET else np.linalg.pinv(A)


def vcycle(u: np.ndarray, f: np.ndarray, n: int, bc: int, nu1: int = 2, nu2: int = 2,
           prolong=None, levels: int = 0) -> np.ndarray:
    """One V(nu1, nu2) cycle from the dense pieces above.  prolong (optional):
    a function (coarse vector, nc) -> fine vector used instead of the spline
    on the `levels` finest prolongations."""
    if n == 5:
        return coarsest_inverse(bc) @ f
    for _ in range(nu1):
        u = half_sweep(u, f, n, bc, 0)
        u = half_sweep(u, f, n, bc, 1)
    r = f - operator(n, bc) @ u
    fc = full_weighting(n, bc) @ r
    nc = (n - 1) // 2 + 1
    uc = vcycle(np.zeros_like(fc), fc, nc, bc, nu1, nu2, prolong, levels - 1)
    if prolong is not None and levels > 0:
        u = u + prolong(uc, nc)
    else:
        u = u + spline_prolong(nc, bc) @ uc
    for _ in range(nu2):
        u = half_sweep(u, f, n, bc, 0)
        u = half_sweep(u, f, n, bc, 1)
    return u


def vcycle_matrix(n: int, bc: int, nu1: int = 2, nu2: int = 2) -> np.ndarray:
    """Error-propagation matrix of the homogeneous cycle (f = 0)."""
    m = m_of(n, bc) ** 2
    cols = [vcycle(e, np.zeros(m), n, bc, nu1, nu2) for e in np.eye(m)]
    return np.array(cols).T


def exact_discrete_solution(f: np.ndarray, bc: int) -> np.ndarray:
    """Exact solution of the 5-point system by a fast spectral solve.

    Dirichlet: type-I DST diagonalises A on the interior.  Periodic: the 2-D
    real FFT diagonalises A on the unique nodes; the zero mode (the null
    space) is set to 0, giving the zero-mean solution."""
    n = f.shape[0]
    h = 1.0 / (n - 1)
    if bc == DIRICHLET:
        m = n - 2
        k = np.arange(1, m + 1)
        lam1 = (4.0 / h ** 2) * np.sin(k * np.pi * h / 2) ** 2
        lam = lam1[:, None] + lam1[None, :]
        fh = scipy.fft.dstn(f[1:-1, 1:-1], type=1)
        u = np.zeros_like(f)
        u[1:-1, 1:-1] = scipy.fft.idstn(fh / lam, type=1)
        return u
    N = n - 1
    ky = np.fft.fftfreq(N, d=1.0 / N)[:, None]
    kx = np.fft.rfftfreq(N, d=1.0 / N)[None, :]
    lam = (4.0 / h ** 2) * (np.sin(np.pi * kx * h) ** 2 + np.sin(np.pi * ky * h) ** 2)
    fh = np.fft.rfft2(f[:-1, :-1])
    lam[0, 0] = 1.0
    uh = fh / lam
    uh[0, 0] = 0.0
    core = np.fft.irfft2(uh, s=(N, N))
    return to_grid(core.reshape(-1), n, bc)


# ---- factor-F transfers of the two-level experiment (periodic grids) --------

@functools.lru_cache(maxsize=None)
def linear_interp_factor_1d(mc: int, F: int) -> np.ndarray:
    """Periodic piecewise-linear interpolation from mc coarse nodes (spacing F
    fine cells) to the mc * F fine nodes: fine node F k + q lies q/F of the way
    from coarse node k to k + 1."""
    P = np.zeros((mc * F, mc))
    for k in range(mc):
        for q in range(F):
            P[F * k + q, k] += 1.0 - q / F
            P[F * k + q, (k + 1) % mc] += q / F
    return P


@functools.lru_cache(maxsize=None)
def restrict_factor(N: int, F: int) -> np.ndarray:
    """Full weighting widened to the factor F, as the transpose of bilinear
    interpolation divided by F^2 (constants map to constants)."""
    P1 = linear_interp_factor_1d(N // F, F)
    return np.kron(P1.T, P1.T) / float(F * F)


@functools.lru_cache(maxsize=None)
def spline_1d_factor(mc: int, F: int) -> np.ndarray:
    """Periodic cubic-spline interpolation matrix by the factor F (scipy's
    CubicSpline on unit vectors, evaluated at the fine nodes)."""
    nc = mc + 1
    xc = np.arange(nc, dtype=np.float64)
    xf = np.arange(mc * F, dtype=np.float64) / F
    cols = []
    for k in range(mc):
        y = np.zeros(nc)
        y[k] = 1.0
        if k == 0:
            y[-1] = 1.0
        cols.append(CubicSpline(xc, y, bc_type="periodic")(xf))
    return np.array(cols).T


def twolevel(p: np.ndarray, f: np.ndarray, N: int, F: int, n_smooth: int,
             coarse_sweeps: int) -> np.ndarray:
    """One two-level iteration from the dense pieces: n_smooth red/black
    sweeps, residual, factor-F restriction, coarse_sweeps red/black sweeps
    from zero on the coarse 5-point operator, spline prolongation by F, no
    post-smoothing."""
    n, nc = N + 1, N // F + 1
    for _ in range(n_smooth):
        p = half_sweep(p, f, n, PERIODIC, 0)
        p = half_sweep(p, f, n, PERIODIC, 1)
    r = f - operator(n, PERIODIC) @ p
    rc = restrict_factor(N, F) @ r
    d = np.zeros_like(rc)
    for _ in range(coarse_sweeps):
        d = half_sweep(d, rc, nc, PERIODIC, 0)
        d = half_sweep(d, rc, nc, PERIODIC, 1)
    P1 = spline_1d_factor(N // F, F)
    return p + np.kron(P1, P1) @ d
