"""CPU pins of the oracle's two-level experiment (Section 4.1; Table 1;
appendix V-CYCLE with one coarse level that is relaxed, not solved): the
factor-F restriction and prolongation and the two-level iteration, each
against something other than its own code (a dense model built from matrix
definitions and scipy, closed forms, the spectral exact solution)."""

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

import dense_model as dm
import oracle
import workloads

P = oracle.PERIODIC


def rand_periodic(N, rng, zero_mean=False):
    v = rng.standard_normal(N * N)
    if zero_mean:
        v -= v.mean()
    return dm.to_grid(v, N + 1, P)


@pytest.mark.parametrize("N,F", [(32, 2), (32, 4), (32, 8), (64, 16), (192, 32)])
def test_restrict_factor_is_scaled_transpose_of_linear_interpolation(N, F):
    rng = np.random.default_rng(N + F)
    r = rand_periodic(N, rng)
    got = dm.to_vec(oracle.restrict_factor(r, F), P)
    ref = dm.restrict_factor(N, F) @ dm.to_vec(r, P)
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


def test_restrict_factor_two_is_full_weighting():
    rng = np.random.default_rng(3)
    r = rand_periodic(64, rng)
    a, b = oracle.restrict_factor(r, 2), oracle.restrict(r, P)
    assert np.abs(a - b).max() <= 1e-15 * np.abs(b).max()


@pytest.mark.parametrize("F", [4, 16])
def test_restrict_factor_keeps_constants_and_sums(F):
    N = 192
    c = np.full((N + 1, N + 1), 2.5)
    assert np.all(oracle.restrict_factor(c, F) == 2.5)
    r = rand_periodic(N, np.random.default_rng(F))
    rc = oracle.restrict_factor(r, F)
    assert abs(rc[:-1, :-1].sum() * F * F - r[:-1, :-1].sum()) <= 1e-11 * np.abs(r).sum()


@pytest.mark.parametrize("N,F", [(32, 2), (48, 4), (192, 16), (192, 32)])
def test_prolong_factor_matches_scipy_periodic_spline(N, F):
    rng = np.random.default_rng(10 + F)
    mc = N // F
    ec = rand_periodic(mc, rng)
    got = oracle.prolong_factor(ec, F)
    xc = np.arange(mc + 1, dtype=np.float64)
    xf = np.arange(N + 1, dtype=np.float64) / F
    tmp = CubicSpline(xc, ec, axis=1, bc_type="periodic")(xf)
    ref = CubicSpline(xc, tmp, axis=0, bc_type="periodic")(xf)
    assert got.shape == (N + 1, N + 1)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_prolong_factor_keeps_coarse_nodes_and_constants():
    rng = np.random.default_rng(5)
    ec = rand_periodic(12, rng)
    ef = oracle.prolong_factor(ec, 16)
    assert np.abs(ef[::16, ::16] - ec).max() <= 1e-15 * np.abs(ec).max()
    c = np.full((13, 13), -1.25)
    assert np.abs(oracle.prolong_factor(c, 16) + 1.25).max() <= 1e-15


def test_prolong_factor_two_equals_midpoint_spline():
    rng = np.random.default_rng(6)
    ec = rand_periodic(16, rng)
    a, b = oracle.prolong_factor(ec, 2), oracle.prolong(ec, P)
    assert np.abs(a - b).max() <= 1e-15 * np.abs(b).max()


@pytest.mark.parametrize("N,F,ns,cs", [(32, 4, 3, 2), (32, 8, 2, 10), (64, 16, 1, 3)])
def test_twolevel_matches_dense_model(N, F, ns, cs):
    rng = np.random.default_rng(N * F + ns)
    p = rand_periodic(N, rng)
    f = rand_periodic(N, rng, zero_mean=True)
    got = dm.to_vec(oracle.twolevel(p, f, F, ns, cs), P)
    ref = dm.twolevel(dm.to_vec(p, P), dm.to_vec(f, P), N, F, ns, cs)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_twolevel_exact_solution_is_a_fixed_point():
    f = workloads.rhs_twolevel_periodic(192, 7)
    ps = dm.exact_discrete_solution(f, P)
    out = oracle.twolevel(ps, f, 16, 20, 10)
    assert np.linalg.norm(out - ps) <= 1e-12 * np.linalg.norm(ps)


def test_twolevel_rate_matches_spectral_radius():
    """The change between iterates shrinks asymptotically by the spectral
    radius of the homogeneous iteration matrix (the constant mode, which
    every step keeps, excluded)."""
    N, F, ns, cs = 32, 8, 2, 10
    m = N * N
    cols = [dm.twolevel(e, np.zeros(m), N, F, ns, cs) for e in np.eye(m)]
    M = np.array(cols).T
    ev = np.linalg.eigvals(M)
    ev = ev[np.abs(ev - 1.0) > 1e-8]
    rho = np.abs(ev).max()
    rng = np.random.default_rng(9)
    f = rand_periodic(N, rng, zero_mean=True)
    p0 = rand_periodic(N, rng)
    _, it, hist = oracle.twolevel_solve(f, p0, F, ns, cs, n_pre=0, tol=0.0, max_iter=60)
    ratio = hist[-1] / hist[-2]
    assert abs(ratio - rho) <= 0.02 * rho, (ratio, rho)


def test_twolevel_solve_reaches_the_exact_solution():
    """The paper's fiducial setting (192 -> 12, N_smooth 20, coarse relaxed
    10 times, N_smooth,pre 10, stop when the change is <= 1e-10): the result,
    mean removed, is the exact discrete solution (FFT) to within what the
    last change and the observed rate allow."""
    f = workloads.rhs_twolevel_periodic(192, 2000)
    p0 = workloads.initial_grid_periodic(192, 3000)
    p, it, hist = oracle.twolevel_solve(f, p0, 16)
    assert hist[-1] <= 1e-10 and it < 300
    rho = hist[-1] / hist[-2]
    ps = dm.exact_discrete_solution(f, P)
    e = dm.to_vec(p, P) - dm.to_vec(p, P).mean() - dm.to_vec(ps, P)
    assert np.linalg.norm(e) <= 2 * hist[-1] * rho / (1 - rho) + 1e-13 * np.linalg.norm(
        dm.to_vec(ps, P))
