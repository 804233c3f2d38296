"""Pins of the pressure-projection oracle (oracle/projection.py): closed
forms for the Taylor-Green vortex and a shear flow, the same discrete
operators evaluated through their Fourier symbols, and the telescoping sum
of a divergence."""

import numpy as np
import pytest

import workloads
from oracle import projection as pj


def nodes(n):
    h = 1.0 / (n - 1)
    X = np.arange(n) * h
    return np.meshgrid(X, X, indexing="xy"), h  # x varies along columns


@pytest.mark.parametrize("n", [17, 65])
def test_taylor_green_source_closed_form(n):
    """u = sin x cos y, v = -cos x sin y (x = 2 pi X): the central
    differences give c = (s/2) (sin 2x, sin 2y) with s = sin(2 pi h)/h, so
    f = -(s/2) sin(4 pi h)/h (cos 2x + cos 2y)."""
    (X, Y), h = nodes(n)
    x, y = 2 * np.pi * X, 2 * np.pi * Y
    ux, uy = np.sin(x) * np.cos(y), -np.cos(x) * np.sin(y)
    s = np.sin(2 * np.pi * h) / h
    want = -(s / 2) * np.sin(4 * np.pi * h) / h * (np.cos(2 * x) + np.cos(2 * y))
    got = pj.ns_rhs(ux, uy)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11 * np.abs(want).max())


def test_shear_flow_has_no_source():
    """u = (sin 2 pi Y, 0): the convective term vanishes node by node."""
    (X, Y), h = nodes(33)
    ux = np.sin(2 * np.pi * Y) + 0.3 * np.cos(6 * np.pi * Y)
    uy = np.zeros_like(ux)
    assert np.all(pj.ns_rhs(ux, uy) == 0.0)


def spectral_d(a, h, axis):
    """Central difference through its Fourier symbol i sin(2 pi k h)/h."""
    N = a.shape[axis]
    k = np.fft.fftfreq(N, d=1.0 / N)
    sym = 1j * np.sin(2 * np.pi * k * h) / h
    shape = [1, 1]
    shape[axis] = N
    return np.real(np.fft.ifft(np.fft.fft(a, axis=axis) * sym.reshape(shape), axis=axis))


def test_source_matches_fourier_symbol_evaluation():
    n = 65
    ux, uy = workloads.velocity_periodic(n, 3)
    h = 1.0 / (n - 1)
    U, V = ux[:-1, :-1], uy[:-1, :-1]
    dx = lambda a: spectral_d(a, h, 1)  # noqa: E731
    dy = lambda a: spectral_d(a, h, 0)  # noqa: E731
    cx = U * dx(U) + V * dy(U)
    cy = U * dx(V) + V * dy(V)
    want = -(dx(cx) + dy(cy))
    got = pj.ns_rhs(ux, uy)
    np.testing.assert_allclose(got[:-1, :-1], want, rtol=0, atol=1e-11 * np.abs(want).max())
    np.testing.assert_array_equal(got[-1, :], got[0, :])
    np.testing.assert_array_equal(got[:, -1], got[:, 0])


def test_source_sums_to_zero():
    ux, uy = workloads.velocity_periodic(129, 4)
    f = pj.ns_rhs(ux, uy)[:-1, :-1]
    assert abs(f.sum()) <= 1e-12 * np.sqrt((f * f).sum()) * f.shape[0]


def test_update_closed_form():
    """Taylor-Green velocity and p = cos x: u_x - dt ((s/2) sin 2x - s sin x),
    u_y - dt (s/2) sin 2y."""
    (X, Y), h = nodes(33)
    x, y = 2 * np.pi * X, 2 * np.pi * Y
    ux, uy = np.sin(x) * np.cos(y), -np.cos(x) * np.sin(y)
    p = np.cos(x)
    s = np.sin(2 * np.pi * h) / h
    dt = 0.01
    vx, vy = pj.ns_update(ux, uy, p, dt)
    np.testing.assert_allclose(vx, ux - dt * (s / 2 * np.sin(2 * x) - s * np.sin(x)), rtol=0, atol=1e-13)
    np.testing.assert_allclose(vy, uy - dt * (s / 2 * np.sin(2 * y)), rtol=0, atol=1e-13)


def test_update_with_zero_step_is_identity():
    ux, uy = workloads.velocity_periodic(33, 5)
    p = workloads.rhs_divu_periodic(33, 6)
    vx, vy = pj.ns_update(ux, uy, p, 0.0)
    np.testing.assert_array_equal(vx, ux)
    np.testing.assert_array_equal(vy, uy)


def test_velocity_generator_is_divergence_free_spectrally():
    """The generated field has zero spectral divergence and unit RMS speed
    (input sanity, not the method)."""
    n = 65
    ux, uy = workloads.velocity_periodic(n, 7)
    U, V = ux[:-1, :-1], uy[:-1, :-1]
    N = n - 1
    k = np.fft.fftfreq(N, d=1.0 / N)
    div = np.fft.fft2(U) * 1j * k[None, :] + np.fft.fft2(V) * 1j * k[:, None]
    assert np.abs(div).max() <= 1e-9 * np.abs(np.fft.fft2(U)).max()
    assert abs(np.mean(U * U + V * V) - 1.0) < 1e-12


def _solve_q(f):
    """The oracle's Poisson solve, A q = f with A = -Laplacian_h (q = -p)."""
    import oracle

    return oracle.solve(f, oracle.PERIODIC, rtol=1e-13, max_cycles=80)[0]


def test_time_step_pressure_closed_form():
    """Taylor-Green: the source is a multiple of cos 2x + cos 2y, an
    eigenfunction of the 5-point Laplacian with eigenvalue
    -(4/h^2) sin^2(2 pi h), so the step's p is that multiple divided by the
    eigenvalue (p > 0 where cos 2x + cos 2y > 0, as the continuous
    (cos 2x + cos 2y)/4).  A flipped sign on p fails here."""
    n = 65
    (X, Y), h = nodes(n)
    x, y = 2 * np.pi * X, 2 * np.pi * Y
    ux, uy = np.sin(x) * np.cos(y), -np.cos(x) * np.sin(y)
    s = np.sin(2 * np.pi * h) / h
    fc = -(s / 2) * np.sin(4 * np.pi * h) / h
    lam = -(4 / h**2) * np.sin(2 * np.pi * h) ** 2
    want = fc / lam * (np.cos(2 * x) + np.cos(2 * y))
    _, _, p = pj.time_step(ux, uy, 1e-3, _solve_q)
    pm = p - p[:-1, :-1].mean()
    np.testing.assert_allclose(pm, want, rtol=0, atol=1e-9 * np.abs(want).max())
    assert abs(want.max() - 0.5) < 0.01  # (cos 2x + cos 2y)/4 peaks at 1/2


@pytest.mark.parametrize("n,bound", [(65, 0.05), (129, 0.0125)])
def test_time_step_keeps_taylor_green_steady(n, bound):
    """Taylor-Green is a steady solution of the Euler equations, so one
    source -> solve -> update step changes it only by the discretisation
    error: max |du| / dt = O(h^2).  With the pressure force reversed the
    rate is about 2 |grad p| = 2 pi instead."""
    (X, Y), h = nodes(n)
    x, y = 2 * np.pi * X, 2 * np.pi * Y
    ux, uy = np.sin(x) * np.cos(y), -np.cos(x) * np.sin(y)
    dt = 1e-3
    vx, vy, p = pj.time_step(ux, uy, dt, _solve_q)
    rate = max(np.abs(vx - ux).max(), np.abs(vy - uy).max()) / dt
    assert rate <= bound, rate
    wx, wy = pj.ns_update(ux, uy, -p, dt)  # the reversed pressure force
    wrong = max(np.abs(wx - ux).max(), np.abs(wy - uy).max()) / dt
    assert wrong > 5.0, wrong


def test_time_step_reduces_divergence_of_increment():
    """On a divergence-free random field the pressure term removes most of
    the divergence that the convective term alone puts into the increment
    (the central-difference divergence of the central-difference gradient is
    the wide Laplacian, not the 5-point one the solve inverts, so the
    removal is not exact)."""
    n = 129
    h = 1.0 / (n - 1)
    ux, uy = workloads.velocity_periodic(n, 21)
    dt = 1e-3

    def div_inc(vx, vy):
        dx = (vx - ux)[:-1, :-1]
        dy = (vy - uy)[:-1, :-1]
        return np.abs(pj.ddx(dx, h) + pj.ddy(dy, h)).max()

    vx, vy, p = pj.time_step(ux, uy, dt, _solve_q)
    with_p = div_inc(vx, vy)
    nx, ny = pj.ns_update(ux, uy, np.zeros_like(p), dt)
    without = div_inc(nx, ny)
    rx, ry = pj.ns_update(ux, uy, -p, dt)
    reversed_ = div_inc(rx, ry)
    assert with_p < 0.5 * without < reversed_, (with_p, without, reversed_)
