"""GPU parity of the pressure-projection steps (mg_ns_rhs, mg_ns_update)
against the oracle (oracle/projection.py), through the C ABI.

mg_ns_update takes the Poisson solve's output q = -p (the library solves
-Laplacian_h q = f); the oracle's update takes the paper's p, so every
comparison hands the oracle p = -q (negation is exact, so FP64 stays
bit-exact).

Tolerances: FP64 bit-exact (the kernels evaluate the same expressions in the
same order without contraction, and 1/(2h) is a power of two); FP32 against
the FP64 oracle on the FP32-rounded inputs within 1e-5 of the largest
intermediate term (the differences of convective terms cancel, so the bound
is taken on their size, not on the result); a whole time step (source,
mg_solve to 1e-12, update) within 1e-6 of the velocity change (both
solves stop at 1e-12, so their pressures differ by the solve error).
"""

import numpy as np
import pytest

import oracle
import workloads
from oracle import projection as pj

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F64, F32 = 0, 1


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def B():
    from paper_2403_07936_amd import binding
    binding.lib()
    return binding


def say(msg):
    print(msg, flush=True)


def padded(a, pitch, dev, dtype):
    t = torch.zeros((a.shape[0], pitch), dtype=dtype, device=dev)
    t[:, :a.shape[1]] = torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype)
    return t


def gpu_rhs(B, dev, ux, uy, pitch, dt_):
    tdt = torch.float64 if dt_ == F64 else torch.float32
    n = ux.shape[0]
    a, b = padded(ux, pitch, dev, tdt), padded(uy, pitch, dev, tdt)
    f = torch.full((n, pitch), 7.0, dtype=tdt, device=dev)
    B.mg_ns_rhs(n, a.data_ptr(), b.data_ptr(), f.data_ptr(), pitch, dt_)
    torch.cuda.synchronize()
    out = f.cpu().numpy()
    assert np.all(out[:, n:] == 7.0)  # padding untouched
    return out[:, :n]


def gpu_update(B, dev, ux, uy, q, dt, pitch, dt_):
    """mg_ns_update with the solver-sign pressure q (= -p)."""
    tdt = torch.float64 if dt_ == F64 else torch.float32
    n = ux.shape[0]
    a, b, q = (padded(x, pitch, dev, tdt) for x in (ux, uy, q))
    ox = torch.full((n, pitch), 7.0, dtype=tdt, device=dev)
    oy = torch.full((n, pitch), 7.0, dtype=tdt, device=dev)
    B.mg_ns_update(n, a.data_ptr(), b.data_ptr(), q.data_ptr(), dt, ox.data_ptr(), oy.data_ptr(),
                   pitch, dt_)
    torch.cuda.synchronize()
    return ox.cpu().numpy()[:, :n], oy.cpu().numpy()[:, :n]


CASES = [(5, 0), (17, 3), (65, 0), (257, 5), (1025, 0)]


@pytest.mark.parametrize("n,pad", CASES)
def test_rhs_bit_exact_fp64(B, dev, n, pad):
    ux, uy = workloads.velocity_periodic(n, 11)
    got = gpu_rhs(B, dev, ux, uy, n + pad, F64)
    want = pj.ns_rhs(ux, uy)
    say(f"ns_rhs n={n} pitch={n + pad}: max |diff| {np.abs(got - want).max():.3e}")
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("n,pad", CASES)
def test_update_bit_exact_fp64(B, dev, n, pad):
    ux, uy = workloads.velocity_periodic(n, 12)
    q = workloads.rhs_divu_periodic(n, 13) * 1e-3
    gx, gy = gpu_update(B, dev, ux, uy, q, 1e-3, n + pad, F64)
    wx, wy = pj.ns_update(ux, uy, -q, 1e-3)
    say(f"ns_update n={n}: max |diff| {max(np.abs(gx - wx).max(), np.abs(gy - wy).max()):.3e}")
    np.testing.assert_array_equal(gx, wx)
    np.testing.assert_array_equal(gy, wy)


@pytest.mark.parametrize("n", [17, 257])
def test_fp32_within_rounding(B, dev, n):
    ux, uy = workloads.velocity_periodic(n, 14)
    q = workloads.rhs_divu_periodic(n, 15) * 1e-3
    r32 = [x.astype(np.float32).astype(np.float64) for x in (ux, uy, q)]
    h = 1.0 / (n - 1)
    cx, cy = pj.convection(r32[0][:-1, :-1], r32[1][:-1, :-1], h)
    scale = (np.abs(cx).max() + np.abs(cy).max()) / (2 * h)
    got = gpu_rhs(B, dev, ux, uy, n, F32)
    want = pj.ns_rhs(r32[0], r32[1])
    err = np.abs(got - want).max()
    say(f"ns_rhs fp32 n={n}: max err {err:.3e} of scale {scale:.3e}")
    assert err <= 1e-5 * scale
    dt = 1e-3
    gx, gy = gpu_update(B, dev, ux, uy, q, dt, n, F32)
    wx, wy = pj.ns_update(r32[0], r32[1], -r32[2], dt)
    sc = 1.0 + dt * (np.abs(cx).max() + np.abs(cy).max() + np.abs(q).max() / h)
    err = max(np.abs(gx - wx).max(), np.abs(gy - wy).max())
    say(f"ns_update fp32 n={n}: max err {err:.3e} of scale {sc:.3e}")
    assert err <= 1e-6 * sc


def test_full_size_fp64_bit_exact(B, dev):
    """At the benchmark's size (4097^2), bit-exact on every node."""
    n = 4097
    ux, uy = workloads.velocity_periodic(n, 16)
    got = gpu_rhs(B, dev, ux, uy, n, F64)
    np.testing.assert_array_equal(got, pj.ns_rhs(ux, uy))
    q = workloads.rhs_divu_periodic(n, 17) * 1e-3
    gx, gy = gpu_update(B, dev, ux, uy, q, 1e-4, n, F64)
    wx, wy = pj.ns_update(ux, uy, -q, 1e-4)
    np.testing.assert_array_equal(gx, wx)
    np.testing.assert_array_equal(gy, wy)


def test_time_step_with_solve_matches_oracle(B, dev):
    """Source, pressure solve to 1e-12 and velocity step on the GPU (the
    solver's output handed to mg_ns_update unchanged) against the oracle's
    time step, which takes p = -q; plus the physics: on a steady
    Taylor-Green flow the same GPU chain changes u only by O(h^2)."""
    n, dt = 257, 1e-3
    ux, uy = workloads.velocity_periodic(n, 18)
    a, b = padded(ux, n, dev, torch.float64), padded(uy, n, dev, torch.float64)
    f = torch.zeros((n, n), dtype=torch.float64, device=dev)
    p = torch.zeros_like(f)
    ox, oy = torch.zeros_like(f), torch.zeros_like(f)
    o = B.mg_options_default()
    ctx = B.mg_setup([(n, oracle.PERIODIC, 0)], o, torch.cuda.current_stream().cuda_stream)
    try:
        B.mg_ns_rhs(n, a.data_ptr(), b.data_ptr(), f.data_ptr(), n, F64,
                    torch.cuda.current_stream().cuda_stream)
        st, cyc, rel = B.mg_solve(ctx, [p.data_ptr()], [f.data_ptr()], 1e-12, 60)
        B.mg_ns_update(n, a.data_ptr(), b.data_ptr(), p.data_ptr(), dt, ox.data_ptr(),
                       oy.data_ptr(), n, F64, torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
    finally:
        B.mg_destroy(ctx)
    wx, wy, _ = pj.time_step(
        ux, uy, dt, lambda fo: oracle.solve(fo, oracle.PERIODIC, rtol=1e-12, max_cycles=60)[0])
    gx, gy = ox.cpu().numpy(), oy.cpu().numpy()
    err = max(np.abs(gx - wx).max(), np.abs(gy - wy).max()) / np.abs(wx - ux).max()
    say(f"time step n={n}: solve {cyc[0]} cycles relres {rel[0]:.2e}; step error {err:.3e}")
    assert st == 0 and rel[0] <= 1e-12
    assert err <= 1e-6


def test_rejections(B, dev):
    x = torch.zeros((17, 17), dtype=torch.float64, device=dev)
    y = torch.zeros_like(x)
    with pytest.raises(B.MGError):
        B.mg_ns_rhs(17, x.data_ptr(), y.data_ptr(), x.data_ptr(), 17, F64)  # f aliases u_x
    with pytest.raises(B.MGError):
        B.mg_ns_rhs(18, x.data_ptr(), y.data_ptr(), y.data_ptr() + 8, 18, F64)
    with pytest.raises(B.MGError):
        B.mg_ns_update(17, x.data_ptr(), y.data_ptr(), x.data_ptr(), 0.1, x.data_ptr(),
                       y.data_ptr(), 17, F64)


def test_gpu_time_step_keeps_taylor_green_steady(B, dev):
    """The GPU chain mg_ns_rhs -> mg_solve -> mg_ns_update on the steady
    Taylor-Green flow: max |du| / dt = O(h^2) (<= 0.05 at 65^2), the same
    bound the oracle's time step is pinned to."""
    n, dt = 65, 1e-3
    X = np.arange(n) / (n - 1)
    x, y = np.meshgrid(2 * np.pi * X, 2 * np.pi * X, indexing="xy")
    ux, uy = np.sin(x) * np.cos(y), -np.cos(x) * np.sin(y)
    a, b = padded(ux, n, dev, torch.float64), padded(uy, n, dev, torch.float64)
    f = torch.zeros((n, n), dtype=torch.float64, device=dev)
    q = torch.zeros_like(f)
    ox, oy = torch.zeros_like(f), torch.zeros_like(f)
    stream = torch.cuda.current_stream().cuda_stream
    ctx = B.mg_setup([(n, oracle.PERIODIC, 0)], B.mg_options_default(), stream)
    try:
        B.mg_ns_rhs(n, a.data_ptr(), b.data_ptr(), f.data_ptr(), n, F64, stream)
        st, cyc, rel = B.mg_solve(ctx, [q.data_ptr()], [f.data_ptr()], 1e-12, 60)
        B.mg_ns_update(n, a.data_ptr(), b.data_ptr(), q.data_ptr(), dt, ox.data_ptr(),
                       oy.data_ptr(), n, F64, stream)
        torch.cuda.synchronize()
    finally:
        B.mg_destroy(ctx)
    rate = max(np.abs(ox.cpu().numpy() - ux).max(), np.abs(oy.cpu().numpy() - uy).max()) / dt
    say(f"Taylor-Green step n={n}: max |du|/dt {rate:.3e}")
    assert st == 0 and rate <= 0.05
