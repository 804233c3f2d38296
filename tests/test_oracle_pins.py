"""Pins of the CPU oracle against things other than itself.

Each part of the oracle is checked against a closed form, a library routine,
a dense matrix model built from definitions (``dense_model``), or an
invariant, so that a dropped term, a wrong sign, index or weight, or a
transposed operand anywhere in it fails at least one test here.
"""

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

import dense_model as dm
import oracle
import workloads

D, P = oracle.DIRICHLET, oracle.PERIODIC
BCS = [D, P]


def rand_grid(n, bc, rng, dtype=np.float64):
    """Random grid function respecting the boundary convention."""
    m = dm.m_of(n, bc)
    return dm.to_grid(rng.standard_normal(m * m), n, bc).astype(dtype)


def zero_mean(a):
    core = a[:-1, :-1] - a[:-1, :-1].mean()
    return dm.to_grid(core.reshape(-1), a.shape[0], P)


# ---------------------------------------------------------------- operator --

@pytest.mark.parametrize("n", [9, 33, 65])
def test_operator_sine_eigenpairs(n):
    """A sin(a pi x) sin(b pi y) = lambda sin sin, lambda = 4/h^2 (sin^2(a pi h/2)
    + sin^2(b pi h/2)) (closed form of the 5-point operator)."""
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    for a, b in [(1, 1), (2, 5), (n - 2, 1), (3, n - 3)]:
        u = np.outer(np.sin(b * np.pi * x), np.sin(a * np.pi * x))
        u[0, :] = u[-1, :] = u[:, 0] = u[:, -1] = 0.0
        lam = 4 / h ** 2 * (np.sin(a * np.pi * h / 2) ** 2 + np.sin(b * np.pi * h / 2) ** 2)
        r = oracle.residual(u, np.zeros_like(u), D)  # r = -A u
        np.testing.assert_allclose(-r[1:-1, 1:-1], lam * u[1:-1, 1:-1], rtol=0,
                                   atol=1e-12 * lam)
        assert np.all(r[0, :] == 0) and np.all(r[:, 0] == 0)


@pytest.mark.parametrize("n", [9, 33])
def test_operator_fourier_eigenpairs(n):
    """Periodic: A cos(2 pi (k x + l y)) = 4/h^2 (sin^2(pi k h) + sin^2(pi l h)) cos(...)."""
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    for k, l in [(1, 0), (2, 3), ((n - 1) // 2, 1)]:
        u = np.cos(2 * np.pi * (k * x[None, :] + l * x[:, None]))
        lam = 4 / h ** 2 * (np.sin(np.pi * k * h) ** 2 + np.sin(np.pi * l * h) ** 2)
        r = oracle.residual(u, np.zeros_like(u), P)
        np.testing.assert_allclose(-r, lam * u, rtol=0, atol=1e-11 * max(lam, 1.0))


@pytest.mark.parametrize("bc", BCS)
def test_residual_matches_kron_operator(bc):
    rng = np.random.default_rng(1)
    n = 17
    u, f = rand_grid(n, bc, rng), rand_grid(n, bc, rng)
    r = oracle.residual(u, f, bc)
    ref = dm.to_vec(f, bc) - dm.operator(n, bc) @ dm.to_vec(u, bc)
    np.testing.assert_allclose(dm.to_vec(r, bc), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_array_equal(r, dm.to_grid(dm.to_vec(r, bc), n, bc))  # boundary / seam


# ---------------------------------------------------------------- smoother --

@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("colour", [0, 1])
def test_half_sweep_matches_matrix_splitting(bc, colour):
    rng = np.random.default_rng(2 + colour)
    n = 17
    u, f = rand_grid(n, bc, rng), rand_grid(n, bc, rng)
    got = oracle.relax(u, f, bc, colour)
    ref = dm.half_sweep(dm.to_vec(u, bc), dm.to_vec(f, bc), n, bc, colour)
    np.testing.assert_allclose(dm.to_vec(got, bc), ref, rtol=1e-13, atol=1e-13)
    np.testing.assert_array_equal(got, dm.to_grid(dm.to_vec(got, bc), n, bc))


@pytest.mark.parametrize("bc", BCS)
def test_half_sweep_zeroes_residual_on_its_colour(bc):
    """Invariant: right after a half-sweep the residual vanishes (to rounding)
    at every node of that colour, and the other colour is untouched."""
    rng = np.random.default_rng(4)
    n = 33
    u, f = rand_grid(n, bc, rng), rand_grid(n, bc, rng)
    for colour in (0, 1):
        u2 = oracle.relax(u, f, bc, colour)
        r = dm.to_vec(oracle.residual(u2, f, bc), bc)
        c = dm.colour_mask(n, bc, colour)
        scale = np.abs(dm.to_vec(f, bc)).max() + 8 * (n - 1) ** 2 * np.abs(u2).max()
        assert np.abs(r[c]).max() <= 1e-14 * scale
        np.testing.assert_array_equal(dm.to_vec(u2, bc)[~c], dm.to_vec(u, bc)[~c])
        u = u2


# ------------------------------------------------------------- restriction --

@pytest.mark.parametrize("bc", BCS)
def test_restrict_is_quarter_transposed_bilinear(bc):
    rng = np.random.default_rng(5)
    for n in (9, 17):
        r = rand_grid(n, bc, rng)
        fc = oracle.restrict(r, bc)
        ref = dm.full_weighting(n, bc) @ dm.to_vec(r, bc)
        nc = (n - 1) // 2 + 1
        np.testing.assert_allclose(dm.to_vec(fc, bc), ref, rtol=1e-14, atol=1e-15)
        np.testing.assert_array_equal(fc, dm.to_grid(dm.to_vec(fc, bc), nc, bc))


def test_restrict_exact_on_bilinear():
    """Full weighting reproduces bilinear functions at interior coarse nodes."""
    n = 33
    x = np.arange(n) / (n - 1)
    X, Y = np.meshgrid(x, x)
    r = 0.3 + 1.7 * X - 0.9 * Y + 2.5 * X * Y
    fc = oracle.restrict(r, D)
    np.testing.assert_allclose(fc[1:-1, 1:-1], r[2:-2:2, 2:-2:2], rtol=0, atol=1e-14)


def test_restrict_periodic_preserves_sum_over_four():
    rng = np.random.default_rng(6)
    r = rand_grid(65, P, rng)
    fc = oracle.restrict(r, P)
    assert abs(fc[:-1, :-1].sum() - r[:-1, :-1].sum() / 4) < 1e-12


# ------------------------------------------------------------ prolongation --

@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("nc", [5, 9, 33])
def test_prolong_matches_scipy_cubicspline(bc, nc):
    """Tensor-product CubicSpline (natural / periodic), x then y."""
    rng = np.random.default_rng(nc + 10 * bc)
    ec = rand_grid(nc, bc, rng)
    ef = oracle.prolong(ec, bc)
    n = 2 * (nc - 1) + 1
    xc = np.arange(nc, dtype=float)
    xf = np.arange(n) / 2.0
    kind = "natural" if bc == D else "periodic"
    along_x = CubicSpline(xc, ec, axis=1, bc_type=kind)(xf)
    ref = CubicSpline(xc, along_x, axis=0, bc_type=kind)(xf)
    np.testing.assert_allclose(ef, ref, rtol=0, atol=2e-15 * np.abs(ec).max() * 4)


@pytest.mark.parametrize("bc", BCS)
def test_prolong_interpolates_and_matches_dense(bc):
    rng = np.random.default_rng(7)
    nc = 9
    ec = rand_grid(nc, bc, rng)
    ef = oracle.prolong(ec, bc)
    np.testing.assert_allclose(ef[::2, ::2], ec, rtol=0, atol=1e-15)
    ref = dm.spline_prolong(nc, bc) @ dm.to_vec(ec, bc)
    np.testing.assert_allclose(dm.to_vec(ef, bc), ref, rtol=0, atol=1e-14)


def test_prolong_periodic_reproduces_constants():
    ec = np.full((17, 17), 3.25)
    np.testing.assert_allclose(oracle.prolong(ec, P), 3.25, rtol=0, atol=1e-14)


# ---------------------------------------------------------- coarsest solve --

@pytest.mark.parametrize("bc", BCS)
def test_coarse_solve_matches_numpy(bc):
    rng = np.random.default_rng(8)
    f = rand_grid(5, bc, rng)
    u = oracle.coarse_solve(f, bc)
    A = dm.operator(5, bc)
    fv = dm.to_vec(f, bc)
    ref = np.linalg.solve(A, fv) if bc == D else np.linalg.pinv(A) @ fv
    np.testing.assert_allclose(dm.to_vec(u, bc), ref, rtol=1e-13, atol=1e-15)
    np.testing.assert_array_equal(u, dm.to_grid(dm.to_vec(u, bc), 5, bc))
    if bc == P:
        assert abs(u[:-1, :-1].mean()) < 1e-15


# ------------------------------------------------------------ whole cycle --

@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", [9, 17, 33])
def test_vcycle_matches_dense_model(bc, n):
    """One V(2,2) cycle from random (u, f) equals the dense model's cycle."""
    rng = np.random.default_rng(n + bc)
    u, f = rand_grid(n, bc, rng), rand_grid(n, bc, rng)
    if bc == P:
        f = zero_mean(f)
    got = oracle.vcycle(u, f, bc)
    ref = dm.vcycle(dm.to_vec(u, bc), dm.to_vec(f, bc), n, bc)
    scale = np.abs(ref).max()
    np.testing.assert_allclose(dm.to_vec(got, bc), ref, rtol=0, atol=1e-12 * scale)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", [9, 17])
def test_asymptotic_rate_equals_iteration_matrix_radius(bc, n):
    """The oracle's measured asymptotic contraction equals the spectral radius
    of the dense model's error-propagation matrix (numpy eigvals)."""
    M = dm.vcycle_matrix(n, bc)
    rho = np.abs(np.linalg.eigvals(M)).max() if bc == D else None
    if bc == P:
        # constants are the null space of A: the cycle leaves them alone.
        # Deflate the constant mode before taking the radius.
        m = M.shape[0]
        Q = np.eye(m) - np.full((m, m), 1.0 / m)
        rho = np.abs(np.linalg.eigvals(Q @ M @ Q)).max()
    rng = np.random.default_rng(9)
    e = rand_grid(n, bc, rng)
    zero = np.zeros_like(e)
    ratios = []
    for _ in range(60):
        e2 = oracle.vcycle(e, zero, bc)
        if bc == P:
            e2 = zero_mean(e2)
        ratios.append(np.linalg.norm(e2) / np.linalg.norm(e))
        e = e2 / np.linalg.norm(e2)
    measured = np.exp(np.mean(np.log(ratios[-20:])))
    assert rho < 0.1
    assert abs(measured - rho) <= 0.03 * rho


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", [9, 17, 33])
def test_solve_reaches_dense_direct_solution(bc, n):
    rng = np.random.default_rng(11)
    f = rand_grid(n, bc, rng)
    if bc == P:
        f = zero_mean(f)
    u, cycles, hist = oracle.solve(f, bc, rtol=1e-12, max_cycles=40)
    assert hist[-1] <= 1e-12
    A = dm.operator(n, bc)
    fv = dm.to_vec(f, bc)
    ref = np.linalg.solve(A, fv) if bc == D else np.linalg.pinv(A) @ fv
    got = dm.to_vec(u, bc)
    if bc == P:
        got = got - got.mean()
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("bc,n", [(D, 65), (D, 257), (P, 65), (P, 257)])
def test_solve_reaches_exact_spectral_solution(bc, n):
    """Converged cycles reach the exact discrete solution (DST / FFT solve)."""
    rng = np.random.default_rng(12)
    if bc == D:
        f = workloads.rhs_divu_dirichlet(n, 3)
    else:
        f = workloads.rhs_divu_periodic(n, 3)
    u, cycles, hist = oracle.solve(f, bc, rtol=1e-11, max_cycles=40)
    assert hist[-1] <= 1e-11
    ref = dm.exact_discrete_solution(f, bc)
    if bc == P:
        u = zero_mean(u)
    assert np.linalg.norm(u - ref) <= 1e-9 * np.linalg.norm(ref)
    del rng


def test_manufactured_solution_closed_form():
    """f = 2 pi^2 sin(pi x) sin(pi y) on 65^2: the discrete solution is
    c sin(pi x) sin(pi y) with c = (pi h/2)^2 / sin^2(pi h/2) = 1.000200822...
    (closed form of the 5-point operator's lowest eigenvalue)."""
    n = 65
    h = 1.0 / (n - 1)
    s = workloads.manufactured_solution(n)
    f = 2 * np.pi ** 2 * s
    u, cycles, hist = oracle.solve(f, D, rtol=1e-12, max_cycles=30)
    c = (np.pi * h / 2) ** 2 / np.sin(np.pi * h / 2) ** 2
    assert abs(c - 1.000200822) < 1e-9
    np.testing.assert_allclose(u, c * s, rtol=0, atol=1e-12)
    # second-order discretisation error against the continuous solution:
    # c - 1 = (pi h)^2 / 12 + O(h^4)
    assert np.abs(u - s).max() <= np.pi ** 2 * h ** 2 / 12 * 1.001


@pytest.mark.parametrize("name,n,bc", [("dirichlet", 65, D), ("dirichlet", 513, D),
                                       ("periodic", 129, P), ("periodic", 513, P)])
def test_textbook_rate_and_independence_of_n(name, n, bc):
    """V(2,2) with red-black Gauss-Seidel contracts the residual by <= ~0.1 per
    cycle, roughly independently of the grid size (textbook multigrid)."""
    f = (workloads.rhs_divu_dirichlet(n, 0) if bc == D else workloads.rhs_divu_periodic(n, 0))
    u, cycles, hist = oracle.solve(f, bc, rtol=1e-10, max_cycles=20)
    assert hist[-1] <= 1e-10
    rates = hist[1:] / hist[:-1]
    assert np.max(rates[1:]) < 0.1
    assert cycles <= 10


# ------------------------------------------------------- mixed precision --

@pytest.mark.parametrize("bc", BCS)
def test_fp32_build_tracks_fp64_build(bc):
    """The FP32 build of each step agrees with the FP64 build to FP32 rounding."""
    rng = np.random.default_rng(13)
    n = 33
    u, f = rand_grid(n, bc, rng), rand_grid(n, bc, rng)
    for fn in (lambda a, b: oracle.relax(a, b, bc, 0),
               lambda a, b: oracle.residual(a, b, bc),
               lambda a, b: oracle.vcycle(a, b, bc)):
        r64 = fn(u, f)
        r32 = fn(u.astype(np.float32), f.astype(np.float32))
        assert r32.dtype == np.float32
        err = np.linalg.norm(r32 - r64) / np.linalg.norm(r64)
        # really rounded to FP32, and only that (the cycle's coarse correction
        # amplifies rounding of a random residual by up to ~100 eps32)
        assert 1e-10 < err < 1e-4


@pytest.mark.parametrize("bc", BCS)
def test_mixed_solve_reaches_fp64_solution(bc):
    n = 257
    f = workloads.rhs_divu_dirichlet(n, 1) if bc == D else workloads.rhs_divu_periodic(n, 1)
    u64, c64, h64 = oracle.solve(f, bc, rtol=1e-10, max_cycles=30)
    um, cm, hm = oracle.solve_mixed(f, bc, rtol=1e-10, max_steps=30)
    assert hm[-1] <= 1e-10
    assert cm <= c64 + 1
    if bc == P:
        u64, um = zero_mean(u64), zero_mean(um)
    assert np.linalg.norm(um - u64) <= 1e-9 * np.linalg.norm(u64)


def test_refine_step_is_fp64_update_of_fp32_cycle():
    """One refinement step equals u + e, e = FP32 cycle on fl32(f - A u)."""
    rng = np.random.default_rng(14)
    n, bc = 33, D
    u, f = rand_grid(n, bc, rng), rand_grid(n, bc, rng)
    got = oracle.refine_step(u, f, bc)
    r = (dm.to_vec(f, bc) - dm.operator(n, bc) @ dm.to_vec(u, bc))
    e = oracle.vcycle(np.zeros((n, n), np.float32), dm.to_grid(r, n, bc).astype(np.float32), bc)
    ref = u + e.astype(np.float64)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-6 * np.abs(e).max())


def test_oracle_is_bitwise_thread_count_independent():
    """The oracle's OpenMP loops have disjoint outputs and its reductions run
    in a fixed order, so its results are the same bits at 1 thread and at 8:
    an FP64 cycle, a mixed refinement step and a solve, both boundary
    conditions (each thread count in a process of its own)."""
    import os
    import subprocess
    import sys

    code = (
        "import hashlib, numpy as np, oracle, workloads\n"
        "h = hashlib.sha256()\n"
        "for bc, f in ((0, workloads.rhs_divu_dirichlet(257, 5)),"
        " (1, workloads.rhs_divu_periodic(257, 6))):\n"
        "    u = oracle.vcycle(np.zeros_like(f), f, bc)\n"
        "    h.update(u.tobytes())\n"
        "    h.update(oracle.refine_step(u, f, bc).tobytes())\n"
        "    us, c, hist = oracle.solve(f, bc, rtol=1e-10, max_cycles=30)\n"
        "    h.update(us.tobytes()); h.update(hist.tobytes())\n"
        "print(h.hexdigest())\n"
    )
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    digests = []
    for threads in ("1", "8"):
        env = dict(os.environ, OMP_NUM_THREADS=threads, PYTHONPATH=root)
        out = subprocess.run([sys.executable, "-c", code], env=env, cwd=root, check=True,
                             capture_output=True, text=True, timeout=300)
        digests.append(out.stdout.strip())
    assert len(digests[0]) == 64 and digests[0] == digests[1], digests
