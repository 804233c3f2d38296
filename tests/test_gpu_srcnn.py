"""GPU parity of the SR-CNN prolongation (HIP library through the C ABI)
against the oracle (oracle/srcnn.py).

Tolerances:
  * hand-set weights that make the network a dyadic linear interpolation:
    bit-exact (every product and sum is exact in bf16/FP32);
  * random weights, one prolongation: relative L2 error <= 2e-2 (bf16
    re-rounding of the activations where the GPU's FP32 accumulation order
    and the oracle's exact sums straddle a rounding boundary; observed
    values are printed);
  * one cycle: ||u_gpu - u_oracle|| <= 2e-2 ||u_oracle - u_in||;
  * solve: cycles to tolerance within +-1 of the oracle's run with the same
    weights and the same switching rule;
  * hybrid schedule (N_GAN, S_thres) with the linear-interpolation weights:
    the same prolongation in every cycle both ran, the per-cycle change of
    the iterate within 1e-6 (FP64) / 1e-3 (mixed) relative, plus 1e-12 of
    the first change (the rounding floor of FP64 iterates), cycles to
    tolerance within +-1.
"""

import numpy as np
import pytest

import oracle
import workloads
from oracle import srcnn
from srcnn_weights import linear_blob, linear_interp, random_blob

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P = oracle.PERIODIC
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


def setup(B, sizes, blob, levels, precision=0, kernel_path=0, **kw):
    o = B.mg_options_default()
    o.precision = precision
    o.kernel_path = kernel_path
    o.prolong = B.MG_PROLONG_SRCNN
    o.cnn_levels = levels
    keep = np.ascontiguousarray(blob, dtype=np.float32)
    o.cnn_weights = keep.ctypes.data
    o.cnn_weights_bytes = keep.nbytes
    for k, v in kw.items():
        setattr(o, k, v)
    ctx = B.mg_setup([(n, P, 0) for n in sizes], o, torch.cuda.current_stream().cuda_stream)
    return ctx


def periodic_field(nc, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((nc - 1, nc - 1))
    # a smooth-ish correction: low-pass in Fourier space
    k = np.fft.fftfreq(nc - 1)
    damp = np.exp(-(k[:, None] ** 2 + k[None, :] ** 2) * 60.0)
    a = np.real(np.fft.ifft2(np.fft.fft2(a) * damp))
    a -= a.mean()
    return srcnn.with_seam(a)


def gpu_prolong(B, ctx, dev, ec, coarse_level, dtype):
    tdt = torch.float64 if dtype == F64 else torch.float32
    ct = torch.from_numpy(np.ascontiguousarray(ec)).to(dev, tdt)
    n = 2 * (ec.shape[0] - 1) + 1
    ft = torch.full((n, n), float("nan"), dtype=tdt, device=dev)
    B.mg_prolong(ctx, 0, coarse_level, B.MG_PROLONG_SRCNN, ct.data_ptr(), ft.data_ptr(), dtype)
    torch.cuda.synchronize()
    return ft.cpu().numpy().astype(np.float64)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_hand_set_weights_bit_exact(B, dev):
    """Layout pin: with the dyadic linear-interpolation weights the GPU output
    equals the closed form exactly (tap orientation, shuffle order, seam)."""
    n = 257
    ctx = setup(B, [n], linear_blob(), 0)
    try:
        for lvl, dtype in ((1, F64), (1, F32), (2, F64)):
            nc = (n - 1) // 2 ** lvl + 1
            rng = np.random.default_rng(lvl)
            e = rng.integers(-16, 17, (nc - 1, nc - 1)).astype(np.float64)
            e[3, 4] = 16.0
            got = gpu_prolong(B, ctx, dev, srcnn.with_seam(e), lvl, dtype)
            want = srcnn.with_seam(linear_interp(e))
            say(f"hand-set level {lvl} dtype {dtype}: max diff {np.abs(got - want).max():.3e}")
            np.testing.assert_array_equal(got, want)
    finally:
        B.mg_destroy(ctx)


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("n,lvl", [(257, 1), (257, 2), (513, 1)])
def test_prolong_matches_oracle(B, dev, dtype, n, lvl):
    blob = random_blob(11)
    layers = srcnn.unpack_weights(blob)
    ctx = setup(B, [n], blob, 0)
    try:
        nc = (n - 1) // 2 ** lvl + 1
        ec = periodic_field(nc, 100 + lvl)
        if dtype == F32:
            ec = ec.astype(np.float32)
        got = gpu_prolong(B, ctx, dev, ec, lvl, dtype)
        want = srcnn.prolong(ec, layers).astype(np.float64)
        err = rel_l2(got, want)
        say(f"prolong n={n} level {lvl} dtype {dtype}: rel L2 {err:.3e}")
        assert err <= 2e-2
        np.testing.assert_array_equal(got[-1], got[0])
        np.testing.assert_array_equal(got[:, -1], got[:, 0])
    finally:
        B.mg_destroy(ctx)


def test_prolong_full_size_sampled(B, dev):
    """1025 periodic (the network's finest prolongation, 512^2 -> 1024^2) in the
    launch configuration of the cycle, checked on windows the oracle
    computes one by one (corners across the wrap, interior)."""
    n = 1025
    blob = random_blob(12)
    layers = srcnn.unpack_weights(blob)
    ctx = setup(B, [n], blob, 2)
    try:
        ec = periodic_field(513, 7)
        got = gpu_prolong(B, ctx, dev, ec, 1, F64)
        eu = srcnn.to_unique(ec)
        for y0, x0 in ((0, 0), (508, 3), (250, 509), (131, 377)):
            h = w = 6
            want = srcnn.forward_window(eu, layers, y0, x0, h, w).astype(np.float64)
            rows = np.arange(2 * y0, 2 * (y0 + h)) % 1024
            cols = np.arange(2 * x0, 2 * (x0 + w)) % 1024
            err = rel_l2(got[np.ix_(rows, cols)], want)
            say(f"window ({y0},{x0}): rel L2 {err:.3e}")
            assert err <= 2e-2
    finally:
        B.mg_destroy(ctx)


@pytest.mark.parametrize("precision,kernel_path,n,levels",
                         [(F64, 0, 257, 1), (F64, 1, 257, 1), (F32, 0, 257, 1), (F64, 0, 513, 2)])
def test_cycle_matches_oracle(B, dev, precision, kernel_path, n, levels):
    blob = random_blob(13, scale=0.7)
    layers = srcnn.unpack_weights(blob)
    f = workloads.rhs_divu_periodic(n, 3)
    u0 = periodic_field(n, 9) * 1e-3
    ctx = setup(B, [n], blob, levels, precision, kernel_path)
    try:
        ut = torch.from_numpy(u0).to(dev)
        ft = torch.from_numpy(f).to(dev)
        B.mg_vcycle(ctx, [ut.data_ptr()], [ft.data_ptr()], 1)
        got = ut.cpu().numpy()
    finally:
        B.mg_destroy(ctx)
    if precision == F64:
        want = srcnn.vcycle(u0, f, layers, levels)
    else:
        want = srcnn.refine_step(u0, f, layers, levels)
    err = np.linalg.norm(got - want) / np.linalg.norm(want - u0)
    say(f"cycle n={n} precision={precision} path={kernel_path} levels={levels}: {err:.3e}")
    assert err <= 2e-2


def oracle_schedule(f, layers, levels, rtol, max_cycles, ratio=0.5, floor=1e-7):
    u = np.zeros_like(f)
    rel = oracle.relres(u, f, P)
    cnn, cycles, used = True, 0, 0
    while rel > rtol and cycles < max_cycles:
        u = srcnn.vcycle(u, f, layers, levels) if cnn else oracle.vcycle(u, f, P)
        used += cnn
        new = oracle.relres(u, f, P)
        if cnn and (new / rel > ratio or new <= floor):
            cnn = False
        rel, cycles = new, cycles + 1
    return cycles, used, rel


@pytest.mark.parametrize("scale", [0.7, 0.05])
def test_solve_with_network_schedule(B, dev, scale):
    """mg_solve with the network prolongation and the spline fallback reaches
    the tolerance in the oracle's number of cycles (+-1) for the same
    weights and rule."""
    n, levels, rtol = 257, 1, 1e-8
    blob = random_blob(14, scale)
    layers = srcnn.unpack_weights(blob)
    f = workloads.rhs_divu_periodic(n, 4)
    co, used, ro = oracle_schedule(f, layers, levels, rtol, 40)
    ctx = setup(B, [n], blob, levels)
    try:
        ft = torch.from_numpy(f).to(dev)
        ut = torch.zeros_like(ft)
        st, cyc, rel = B.mg_solve(ctx, [ut.data_ptr()], [ft.data_ptr()], rtol, 40)
    finally:
        B.mg_destroy(ctx)
    say(f"scale {scale}: GPU {cyc[0]} cycles relres {rel[0]:.2e}; oracle {co} cycles "
        f"({used} with the network) relres {ro:.2e}")
    assert st == 0 and rel[0] <= rtol
    assert abs(cyc[0] - co) <= 1


def test_setup_rejections(B, dev):
    blob = random_blob(15)
    with pytest.raises(B.MGError) as ei:
        setup(B, [257], blob, 2)  # level 2 of 257 is 65 < 129
    assert ei.value.status == B.MG_ERR_UNSUPPORTED
    with pytest.raises(B.MGError) as ei:
        setup(B, [257], blob[:-1], 1)
    assert ei.value.status == B.MG_ERR_INVALID_ARG
    o = B.mg_options_default()
    ctx = B.mg_setup([(129, P, 0)], o, torch.cuda.current_stream().cuda_stream)
    try:
        t = torch.zeros((65, 65), dtype=torch.float64, device=dev)
        u = torch.zeros((129, 129), dtype=torch.float64, device=dev)
        with pytest.raises(B.MGError) as ei:
            B.mg_prolong(ctx, 0, 1, B.MG_PROLONG_SRCNN, t.data_ptr(), u.data_ptr(), F64)
        assert ei.value.status == B.MG_ERR_UNSUPPORTED
    finally:
        B.mg_destroy(ctx)


N_ITER = 300


def gpu_schedule(B, dev, f, blob, levels, precision, n_gan, s_thres, rtol, cap):
    ctx = setup(B, [f.shape[0]], blob, levels, precision, n_gan=n_gan, s_thres=s_thres,
                check_every=1)
    try:
        ft = torch.from_numpy(f).to(dev)
        ut = torch.zeros_like(ft)
        st, cyc, rel = B.mg_solve(ctx, [ut.data_ptr()], [ft.data_ptr()], rtol, cap)
        ops, dif = B.mg_solve_history(ctx, 0)
    finally:
        B.mg_destroy(ctx)
    return st, cyc[0], rel[0], [o == B.MG_PROLONG_SRCNN for o in ops], dif


@pytest.mark.parametrize("n_gan,levels", [(1.0, 1), (3.0, 1), (1 / 3, 1)])
def test_solve_hybrid_schedule_matches_oracle(B, dev, n_gan, levels):
    """N_GAN network prolongations per spline one (no switch): the GPU takes
    the oracle's operator in every cycle and reaches the tolerance in its
    number of cycles (+-1)."""
    n, rtol, cap = 257, 1e-8, 40
    blob = linear_blob()
    layers = srcnn.unpack_weights(blob)
    f = workloads.rhs_divu_periodic(n, 4)
    _, ops_o, _, rel_o = srcnn.solve_schedule(f, layers, levels, rtol, cap, n_gan, 0.0)
    st, cyc, rel, ops, dif = gpu_schedule(B, dev, f, blob, levels, F64, n_gan, 0.0, rtol, cap)
    say(f"N_GAN={n_gan:.3g} levels={levels}: GPU {cyc} cycles {rel:.2e}; oracle {len(ops_o)} "
        f"cycles {rel_o:.2e}; ops {''.join('N' if o else 's' for o in ops)}")
    assert st == 0 and rel <= rtol and abs(cyc - len(ops_o)) <= 1
    k = min(cyc, len(ops_o))
    assert len(ops) == cyc and ops[:k] == ops_o[:k]
    assert all(np.isnan(dif))


@pytest.mark.parametrize("precision,n_gan", [(F64, N_ITER), (F64, 1 / N_ITER), (F64, 1.0),
                                             (F32, 1.0)])
def test_solve_switch_threshold_matches_oracle(B, dev, precision, n_gan):
    """S_thres between the changes the 3rd and 4th cycles make: the GPU
    switches after the same cycle as the oracle, and the changes it
    measures agree with the oracle's."""
    n, levels, rtol, cap = 257, 1, 1e-9, 40
    mixed = precision == F32
    blob = linear_blob()
    layers = srcnn.unpack_weights(blob)
    f = workloads.rhs_divu_periodic(n, 6)
    _, _, d0, _ = srcnn.solve_schedule(f, layers, levels, rtol, cap, n_gan, 0.0, mixed=mixed)
    assert d0[3] < 0.5 * d0[2]
    s = float(np.sqrt(d0[2] * d0[3]))
    _, ops_o, d_o, rel_o = srcnn.solve_schedule(f, layers, levels, rtol, cap, n_gan, s,
                                                mixed=mixed)
    st, cyc, rel, ops, dif = gpu_schedule(B, dev, f, blob, levels, precision, n_gan, s, rtol, cap)
    say(f"S_thres={s:.3e} N_GAN={n_gan:.3g} mixed={mixed}: GPU {cyc} cycles {rel:.2e}; oracle "
        f"{len(ops_o)} cycles {rel_o:.2e}; ops {''.join('N' if o else 's' for o in ops)}")
    assert st == 0 and rel <= rtol and abs(cyc - len(ops_o)) <= 1
    k = min(cyc, len(ops_o))
    assert ops[:k] == ops_o[:k]
    first = n_gan >= 1.0
    if n_gan != 1.0:
        assert ops_o[:5] == [first] * 4 + [not first]
    # Relative, plus an absolute floor at the rounding noise of the FP64
    # iterates (a few ulps of u summed over 256^2 nodes: ~1e-13 of the first
    # change).
    tol = 1e-3 if mixed else 1e-6
    np.testing.assert_allclose(dif[:k], d_o[:k], rtol=tol, atol=1e-12 * d_o[0])
