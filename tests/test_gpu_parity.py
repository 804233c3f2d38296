"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Every test feeds both sides the same seeded inputs and compares element by
element.  Tolerances:
  * FP64 steps: 1e-13 relative to the output's max (rounding-order and FMA
    contraction differences only);
  * FP64 whole cycle: ||u_gpu - u_oracle|| / ||u_oracle|| <= 1e-12 per cycle
    from identical inputs;
  * FP32 steps: 2e-6 relative to the output's max (a few FP32 ulps);
  * mixed refinement step: ||u_gpu - u_oracle|| <= 1e-5 ||e||, e the step's
    correction, against the oracle's FP32 emulation.
"""

import numpy as np
import pytest

import dense_model as dm
import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

D, P = oracle.DIRICHLET, oracle.PERIODIC
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


def rand_grid(n, bc, rng):
    m = dm.m_of(n, bc)
    return dm.to_grid(rng.standard_normal(m * m), n, bc)


def zero_mean(a):
    core = a[:-1, :-1] - a[:-1, :-1].mean()
    return dm.to_grid(core.reshape(-1), a.shape[0], P)


def ctx_for(B, n, bc, precision=0, use_graph=1, kernel_path=0):
    o = B.mg_options_default()
    o.precision = precision
    o.use_graph = use_graph
    o.kernel_path = kernel_path
    return B.mg_setup([(n, bc, 0)], o, torch.cuda.current_stream().cuda_stream)


def gpu(a, dev, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(msg):
    print(msg, flush=True)


def assert_close(got, ref, rel):
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(got - ref).max() / scale
    assert err <= rel, f"max rel. diff {err:.3e} > {rel:.1e}"


SIZES = [5, 9, 33, 65, 129, 257]


# ------------------------------------------------------------ single steps --

@pytest.mark.parametrize("bc", [D, P])
@pytest.mark.parametrize("n", SIZES[1:])
@pytest.mark.parametrize("dt", [F64, F32])
def test_relax_parity(B, dev, bc, n, dt):
    say(f"relax bc={bc} n={n} dt={dt}")
    rng = np.random.default_rng(100 + n)
    u, f = rand_grid(n, bc, rng), rand_grid(n, bc, rng)
    npdt = np.float64 if dt == F64 else np.float32
    tdt = torch.float64 if dt == F64 else torch.float32
    ctx = ctx_for(B, n, bc)
    try:
        for colour in (0, 1):
            ut, ft = gpu(u, dev, tdt), gpu(f, dev, tdt)
            B.mg_relax(ctx, 0, 0, ut.data_ptr(), ft.data_ptr(), colour, 3, dt)
            ref = u.astype(npdt)
            for k in range(3):
                ref = oracle.relax(ref, f.astype(npdt), bc, (colour + k) % 2)
            assert_close(host(ut), ref, 1e-13 if dt == F64 else 2e-6)
    finally:
        B.mg_destroy(ctx)


@pytest.mark.parametrize("bc", [D, P])
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("dt", [F64, F32])
def test_residual_parity(B, dev, bc, n, dt):
    say(f"residual bc={bc} n={n} dt={dt}")
    rng = np.random.default_rng(200 + n)
    # keep r O(f): u scaled by h^2 so A u is comparable to f
    u, f = rand_grid(n, bc, rng) / (n - 1) ** 2, rand_grid(n, bc, rng)
    npdt = np.float64 if dt == F64 else np.float32
    tdt = torch.float64 if dt == F64 else torch.float32
    ctx = ctx_for(B, n, bc)
    try:
        ut, ft = gpu(u, dev, tdt), gpu(f, dev, tdt)
        rt = torch.full_like(ut, 7.0)
        B.mg_residual(ctx, 0, 0, ut.data_ptr(), ft.data_ptr(), rt.data_ptr(), dt)
        ref = oracle.residual(u.astype(npdt), f.astype(npdt), bc)
        assert_close(host(rt), ref, 1e-13 if dt == F64 else 2e-6)
    finally:
        B.mg_destroy(ctx)


@pytest.mark.parametrize("bc", [D, P])
@pytest.mark.parametrize("n", SIZES[1:])
@pytest.mark.parametrize("dt", [F64, F32])
def test_restrict_parity(B, dev, bc, n, dt):
    say(f"restrict bc={bc} n={n} dt={dt}")
    rng = np.random.default_rng(300 + n)
    r = rand_grid(n, bc, rng)
    nc = (n - 1) // 2 + 1
    npdt = np.float64 if dt == F64 else np.float32
    tdt = torch.float64 if dt == F64 else torch.float32
    ctx = ctx_for(B, n, bc)
    try:
        rt = gpu(r, dev, tdt)
        fct = torch.full((nc, nc), 7.0, device=dev, dtype=tdt)
        B.mg_restrict(ctx, 0, 0, rt.data_ptr(), fct.data_ptr(), dt)
        ref = oracle.restrict(r.astype(npdt), bc)
        assert_close(host(fct), ref, 1e-14 if dt == F64 else 2e-7)
    finally:
        B.mg_destroy(ctx)


@pytest.mark.parametrize("bc", [D, P])
@pytest.mark.parametrize("n", SIZES[1:])
@pytest.mark.parametrize("dt", [F64, F32])
def test_prolong_parity(B, dev, bc, n, dt):
    say(f"prolong bc={bc} n={n} dt={dt}")
    rng = np.random.default_rng(400 + n)
    nc = (n - 1) // 2 + 1
    e = rand_grid(nc, bc, rng)
    npdt = np.float64 if dt == F64 else np.float32
    tdt = torch.float64 if dt == F64 else torch.float32
    ctx = ctx_for(B, n, bc)
    try:
        et = gpu(e, dev, tdt)
        ft = torch.full((n, n), 7.0, device=dev, dtype=tdt)
        B.mg_prolong(ctx, 0, 1, B.MG_PROLONG_SPLINE, et.data_ptr(), ft.data_ptr(), dt)
        ref = oracle.prolong(e.astype(npdt), bc)
        assert_close(host(ft), ref, 1e-13 if dt == F64 else 2e-6)
    finally:
        B.mg_destroy(ctx)


@pytest.mark.parametrize("bc", [D, P])
@pytest.mark.parametrize("dt", [F64, F32])
def test_coarse_solve_parity(B, dev, bc, dt):
    say(f"coarse bc={bc} dt={dt}")
    rng = np.random.default_rng(500)
    f = rand_grid(5, bc, rng)
    if bc == P:
        f = zero_mean(f)
    tdt = torch.float64 if dt == F64 else torch.float32
    ctx = ctx_for(B, 5, bc)
    try:
        ft = gpu(f, dev, tdt)
        ut = torch.full_like(ft, 7.0)
        B.mg_coarse_solve(ctx, 0, ft.data_ptr(), ut.data_ptr(), dt)
        fin = f.astype(np.float32).astype(np.float64) if dt == F32 else f
        ref = oracle.coarse_solve(fin, bc)
        assert_close(host(ut), ref, 1e-14 if dt == F64 else 2e-7)
    finally:
        B.mg_destroy(ctx)


# ------------------------------------------------------------ whole cycles --

def make_rhs(n, bc, seed):
    if bc == D:
        return workloads.rhs_manufactured_dirichlet(n, seed) if n <= 65 else \
            workloads.rhs_divu_dirichlet(n, seed)
    return workloads.rhs_divu_periodic(n, seed)


CYCLE_CASES = [(D, 5), (D, 9), (D, 33), (D, 65), (D, 129), (D, 257), (D, 513),
               (P, 5), (P, 9), (P, 33), (P, 65), (P, 129), (P, 257), (P, 513)]


@pytest.mark.parametrize("bc,n", CYCLE_CASES)
@pytest.mark.parametrize("kernel_path,use_graph", [(0, 1), (0, 0), (1, 1), (2, 1)])
def test_fp64_cycle_parity_per_cycle(B, dev, bc, n, kernel_path, use_graph):
    """From identical inputs each GPU cycle matches the oracle's to 1e-12."""
    say(f"fp64 cycle bc={bc} n={n} path={kernel_path} graph={use_graph}")
    f = make_rhs(n, bc, 0)
    ctx = ctx_for(B, n, bc, 0, use_graph, kernel_path)
    try:
        ft = gpu(f, dev)
        u = np.zeros_like(f)
        for c in range(3):
            ut = gpu(u, dev)
            B.mg_vcycle(ctx, [ut.data_ptr()], [ft.data_ptr()], 1)
            ref = oracle.vcycle(u, f, bc)
            got = host(ut)
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            say(f"  cycle {c + 1}: {err:.2e}")
            assert err <= 1e-12
            u = ref
    finally:
        B.mg_destroy(ctx)


@pytest.mark.parametrize("bc,n", [(D, 65), (P, 65), (D, 257), (P, 257), (P, 513)])
@pytest.mark.parametrize("kernel_path", [0, 1, 2])
def test_mixed_step_parity(B, dev, bc, n, kernel_path):
    """One refinement step against the oracle's FP32 emulation.  The GPU's
    FP32 inner cycle rounds in its own order, so the bar comes from the
    oracle's own spread: D = the larger of the distances of its FP32 step
    from the step with an FP64 inner cycle and from its FP32 step on the
    transposed problem (transposed back), relative to the update e; the GPU
    step must lie within 3 D (L2), and within 1e-6 |e| where D is smaller."""
    say(f"mixed step bc={bc} n={n} path={kernel_path}")
    f = make_rhs(n, bc, 1)
    ctx = ctx_for(B, n, bc, 1, 1, kernel_path)
    try:
        ft = gpu(f, dev)
        u = np.zeros_like(f)
        for c in range(3):
            ut = gpu(u, dev)
            B.mg_vcycle(ctx, [ut.data_ptr()], [ft.data_ptr()], 1)
            ref = oracle.refine_step(u, f, bc)
            e = ref - u
            e64 = oracle.vcycle(np.zeros_like(f), oracle.residual(u, f, bc), bc)
            tr = np.ascontiguousarray(oracle.refine_step(
                np.ascontiguousarray(u.T), np.ascontiguousarray(f.T), bc).T)
            d = max(np.linalg.norm(ref - (u + e64)), np.linalg.norm(ref - tr)) / np.linalg.norm(e)
            err = np.linalg.norm(host(ut) - ref) / np.linalg.norm(e)
            say(f"  step {c + 1}: {err:.2e} (oracle spread D {d:.2e})")
            assert err <= max(1e-6, 3.0 * d)
            u = ref
    finally:
        B.mg_destroy(ctx)


@pytest.mark.parametrize("bc,n", [(D, 5), (P, 5), (P, 9), (D, 17), (P, 129), (D, 257),
                                  (P, 1025)])
def test_mixed_relres_matches_oracle_norm(B, dev, bc, n):
    """The mixed path's norm check (FP64 residual by rows, per-wavefront
    partial sums, fixed-order reduction) against the oracle's residual norm
    of the iterate it returns, on grids from the coarsest up: a dropped row,
    column or seam node shows as a relative difference far above 1e-12."""
    say(f"mixed relres bc={bc} n={n}")
    f = make_rhs(n, bc, 3)
    ctx = ctx_for(B, n, bc, 1)
    try:
        ut = gpu(np.zeros_like(f), dev)
        ft = gpu(f, dev)
        for c in range(2):
            rel = B.mg_vcycle(ctx, [ut.data_ptr()], [ft.data_ptr()], 1, want_relres=True)[0]
            ref = oracle.relres(host(ut), f, bc)
            say(f"  cycle {c + 1}: relres {rel:.6e} oracle {ref:.6e}")
            assert abs(rel - ref) <= 1e-12 * ref + 1e-300
    finally:
        B.mg_destroy(ctx)


@pytest.mark.parametrize("bc,n", [(D, 257), (P, 257), (D, 1025), (P, 1025)])
def test_mixed_step_residual_in_down_pass_is_bitwise(B, dev, bc, n):
    """A mixed step whose level-0 down pass makes the FP64 residual itself
    (mg_vcycle) against the same step started from the residual pass's
    output (mg_solve's first step follows its norm check): the right-hand
    side is the same arithmetic, so the iterates agree bit for bit (periodic:
    up to the mean mg_solve removes)."""
    from paper_2403_07936_amd.solver import Solver
    say(f"residual in down pass bc={bc} n={n}")
    f = make_rhs(n, bc, 4)
    u0 = oracle.vcycle(np.zeros_like(f), f, bc)
    ft = gpu(f, dev)
    sa = Solver([(n, bc)], precision="mixed")
    ua = gpu(u0, dev)
    sa.vcycle([ua], [ft], 1)
    sa.close()
    sb = Solver([(n, bc)], precision="mixed", check_every=1)
    ub = gpu(u0, dev)
    st, cyc, rel = sb.solve([ub], [ft], rtol=1e-300, max_cycles=1)
    sb.close()
    assert cyc[0] == 1
    a, b = host(ua), host(ub)
    if bc == P:
        # mg_solve removes the mean of a periodic u on exit: compare both
        # with the mean removed here (the subtraction rounds differently).
        a, b = zero_mean(a), zero_mean(b)
        say(f"  max |diff| {np.abs(a - b).max():.3e}")
        assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()
    else:
        say(f"  max |diff| {np.abs(a - b).max():.3e}")
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("use_graph", [1, 0])
@pytest.mark.parametrize("bc,n", [(D, 257), (P, 257), (D, 1025), (P, 1025)])
def test_solve_norm_from_next_down_pass(B, dev, bc, n, use_graph, precision):
    """mg_solve takes each norm check from the next step's level-0 down pass
    (mixed: the pass makes the FP64 residual of the iterate anyway; FP64: the
    pass forms the residual of the rows it reads before smoothing them) and
    queues the rest of that step only while the problem is unconverged.
    Checked for 1, 2 and 3 steps (check_every 1): the iterate it returns
    against the same number of mg_vcycle steps, bit for bit (periodic: after
    the mean mg_solve removes on exit), so the down pass of the final check
    left the iterate as it was; and the relative residual it returns against
    the oracle's norm of that iterate before the mean removal (the
    mg_vcycle result), 1e-12 relative.  With and without captured graphs
    (the head and the rest of a step queued eagerly)."""
    from paper_2403_07936_amd.solver import Solver
    say(f"norm from the next down pass {precision} bc={bc} n={n} use_graph={use_graph}")
    f = make_rhs(n, bc, 6)
    ft = gpu(f, dev)
    for steps in (1, 2, 3):
        sa = Solver([(n, bc)], precision=precision, check_every=1, use_graph=bool(use_graph))
        ua = torch.zeros_like(ft)
        st, cyc, rel = sa.solve([ua], [ft], rtol=1e-300, max_cycles=steps)
        sa.close()
        sb = Solver([(n, bc)], precision=precision, use_graph=bool(use_graph))
        ub = torch.zeros_like(ft)
        sb.vcycle([ub], [ft], steps)
        sb.close()
        a, b = host(ua), host(ub)
        ref = oracle.relres(b, f, bc)
        say(f"  {steps} steps: status {st} cycles {cyc[0]} relres {rel[0]:.6e} oracle {ref:.6e}")
        assert cyc[0] == steps
        assert abs(rel[0] - ref) <= 1e-12 * ref
        if bc == P:
            a, b = zero_mean(a), zero_mean(b)
            assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()
        else:
            assert np.array_equal(a, b)


@pytest.mark.parametrize("bc,n", [(D, 513), (P, 513)])
def test_solve_of_a_converged_iterate_changes_nothing(B, dev, bc, n):
    """An mg_solve started from an iterate that already meets the tolerance
    stops at its initial check, which is the next step's level-0 down pass:
    zero cycles, status 0, and the iterate bit for bit as it was; FP64 and
    mixed single problems, and a mixed batch of the same problem twice
    (schedule 3)."""
    from paper_2403_07936_amd.solver import Solver
    say(f"solve of a converged iterate bc={bc} n={n}")
    f = make_rhs(n, bc, 8)
    ft = gpu(f, dev)
    for precision in ("fp64", "mixed"):
        s = Solver([(n, bc)], precision=precision)
        u = torch.zeros_like(ft)
        st, cyc, rel = s.solve([u], [ft], rtol=1e-10, max_cycles=30)
        assert st == 0 and cyc[0] > 0
        before = host(u)
        st, cyc, rel2 = s.solve([u], [ft], rtol=1e-10, max_cycles=30)
        s.close()
        say(f"  {precision} again: status {st} cycles {cyc[0]} relres {rel2[0]:.3e}")
        assert st == 0 and cyc[0] == 0 and rel2[0] <= 1e-10
        assert np.array_equal(host(u), before)
    ctx = batch_ctx(B, [(n, bc), (n, bc)], 1, 3)
    try:
        us = [gpu(before, dev), gpu(before, dev)]
        st, cyc, rel3 = B.mg_solve(ctx, [t.data_ptr() for t in us], [ft.data_ptr()] * 2,
                                   1e-10, 30)
    finally:
        B.mg_destroy(ctx)
    say(f"  batch: status {st} cycles {cyc} relres {rel3}")
    assert st == 0 and cyc == [0, 0]
    for t in us:
        assert np.array_equal(host(t), before)


@pytest.mark.parametrize("name", ["dirichlet4097", "periodic1025"])
def test_full_size_cycle_parity(B, dev, name):
    """The benchmark configurations at full size, in the launch configuration
    the benchmark times (fused kernels, graph): one FP64 cycle and one mixed
    step from the same state, against the oracle, on every grid point (the
    largest element-wise difference as well as the 2-norm)."""
    say(f"full size {name}")
    n, bc, f = workloads.workload(name, 0)
    ft = gpu(f, dev)
    u1 = oracle.vcycle(np.zeros_like(f), f, bc)   # a nonzero starting state
    for precision in (0, 1):
        ctx = ctx_for(B, n, bc, precision)
        try:
            ut = gpu(u1, dev)
            B.mg_vcycle(ctx, [ut.data_ptr()], [ft.data_ptr()], 1)
            got = host(ut)
        finally:
            B.mg_destroy(ctx)
        # Both bars: the 2-norm, and element-wise against the largest value
        # (an error confined to one band-edge column would be diluted ~64x
        # in the 2-norm at 4097^2, but not in the max).
        if precision == 0:
            ref = oracle.vcycle(u1, f, bc)
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            mx = np.abs(got - ref).max() / np.abs(ref).max()
            say(f"  fp64 cycle: l2 {err:.2e} max {mx:.2e}")
            assert err <= 1e-12 and mx <= 1e-12
        else:
            ref = oracle.refine_step(u1, f, bc)
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref - u1)
            mx = np.abs(got - ref).max() / np.abs(ref - u1).max()
            say(f"  mixed step: l2 {err:.2e} max {mx:.2e}")
            assert err <= 1e-5 and mx <= 1e-5


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("bc,n,seed", [(D, 65, 0), (D, 65, 7), (P, 129, 0), (D, 257, 2)])
def test_solve_matches_oracle_solution(B, dev, precision, bc, n, seed):
    say(f"solve precision={precision} bc={bc} n={n} seed={seed}")
    f = make_rhs(n, bc, seed)
    from paper_2403_07936_amd.solver import Solver
    s = Solver([(n, bc)], precision="fp64" if precision == 0 else "mixed")
    ft = gpu(f, dev)
    ut = torch.zeros_like(ft)
    st, cyc, rel = s.solve([ut], [ft], rtol=1e-10, max_cycles=30)
    s.close()
    if precision == 0:
        uo, co, ho = oracle.solve(f, bc, rtol=1e-10, max_cycles=30)
    else:
        uo, co, ho = oracle.solve_mixed(f, bc, rtol=1e-10, max_steps=30)
    say(f"  status={st} cycles={cyc[0]} (oracle {co}) relres={rel[0]:.3e}")
    assert st == 0
    assert rel[0] <= 1e-10
    assert abs(cyc[0] - co) <= 1
    got = host(ut)
    if bc == P:
        uo = zero_mean(uo)
        assert abs(got[:-1, :-1].mean()) <= 1e-14 * np.abs(got).max()
    assert np.linalg.norm(got - uo) <= 1e-9 * np.linalg.norm(uo)


def test_batch_matches_individual_solves(B, dev):
    say("batch of mixed sizes")
    specs = [(33, D, 3), (65, P, 4), (129, P, 5), (17, D, 6)]
    from paper_2403_07936_amd.solver import Solver
    fs = [make_rhs(n, bc, s) for n, bc, s in specs]
    s = Solver([(n, bc) for n, bc, _ in specs], precision="fp64")
    fts = [gpu(f, dev) for f in fs]
    uts = [torch.zeros_like(t) for t in fts]
    s.vcycle(uts, fts, 2)
    for (n, bc, _), f, ut in zip(specs, fs, uts):
        ref = oracle.vcycle(oracle.vcycle(np.zeros_like(f), f, bc), f, bc)
        assert np.linalg.norm(host(ut) - ref) <= 1e-12 * np.linalg.norm(ref)
    s.close()


def test_determinism_bitwise(B, dev):
    say("determinism")
    n, bc = 257, P
    f = make_rhs(n, bc, 9)
    outs = []
    for rep in range(2):
        ctx = ctx_for(B, n, bc, 1)
        ft = gpu(f, dev)
        ut = torch.zeros_like(ft)
        rel = B.mg_vcycle(ctx, [ut.data_ptr()], [ft.data_ptr()], 3, True)
        outs.append((host(ut), rel[0]))
        B.mg_destroy(ctx)
    assert np.array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]


# ----------------------------------------------------------- failure paths --

def test_periodic_nonzero_mean_rhs_is_rejected(B, dev):
    n = 65
    f = make_rhs(n, P, 0) + 0.5
    ctx = ctx_for(B, n, P)
    try:
        ft = gpu(f, dev)
        ut = torch.zeros_like(ft)
        st, cyc, rel = B.mg_solve(ctx, [ut.data_ptr()], [ft.data_ptr()], 1e-10, 10)
        assert st == B.MG_ERR_INCOMPATIBLE_RHS
        assert float(ut.abs().max()) == 0.0
    finally:
        B.mg_destroy(ctx)


def test_nan_rhs_reports_nonfinite(B, dev):
    n = 65
    f = make_rhs(n, D, 0)
    f[10, 10] = np.nan
    ctx = ctx_for(B, n, D)
    try:
        ft = gpu(f, dev)
        ut = torch.zeros_like(ft)
        st, _, _ = B.mg_solve(ctx, [ut.data_ptr()], [ft.data_ptr()], 1e-10, 10)
        assert st == B.MG_ERR_NONFINITE
    finally:
        B.mg_destroy(ctx)


def test_max_cycles_reports_not_converged_with_valid_u(B, dev):
    n = 129
    f = make_rhs(n, D, 0)
    ctx = ctx_for(B, n, D)
    try:
        ft = gpu(f, dev)
        ut = torch.zeros_like(ft)
        st, cyc, rel = B.mg_solve(ctx, [ut.data_ptr()], [ft.data_ptr()], 1e-10, 1)
        assert st == B.MG_ERR_NOT_CONVERGED and cyc[0] == 1
        ref = oracle.vcycle(np.zeros_like(f), f, D)
        assert np.linalg.norm(host(ut) - ref) <= 1e-12 * np.linalg.norm(ref)
        assert abs(rel[0] - oracle.relres(ref, f, D)) <= 1e-9 * rel[0]
    finally:
        B.mg_destroy(ctx)


def test_unreachable_tolerance_reports_stagnation(B, dev):
    n = 129
    f = make_rhs(n, D, 0)
    ctx = ctx_for(B, n, D)
    try:
        ft = gpu(f, dev)
        ut = torch.zeros_like(ft)
        st, cyc, rel = B.mg_solve(ctx, [ut.data_ptr()], [ft.data_ptr()], 1e-18, 60)
        assert st == B.MG_ERR_STAGNATED
        assert rel[0] < 1e-12 and cyc[0] < 60
    finally:
        B.mg_destroy(ctx)


# ------------------------------------------------------- persistent schedule --

def batch_ctx(B, specs, precision, schedule, check_every=0, use_graph=1):
    o = B.mg_options_default()
    o.precision = precision
    o.schedule = schedule
    o.check_every = check_every
    o.use_graph = use_graph
    return B.mg_setup([(n, bc, 0) for n, bc in specs], o, torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("schedule", [2, 3])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("bc,sizes", [(P, [33, 129, 65, 257, 513, 9]), (D, [257, 65, 1025, 129])])
def test_persistent_batch_step_parity(B, dev, schedule, precision, bc, sizes):
    """One persistent launch (schedule 2), or one launch per phase (3),
    steps every problem of an uneven batch; each problem's step matches the
    oracle's."""
    say(f"batch schedule={schedule} precision={precision} bc={bc} sizes={sizes}")
    specs = [(n, bc) for n in sizes]
    fs = [make_rhs(n, bc, 20 + k) for k, n in enumerate(sizes)]
    ctx = batch_ctx(B, specs, precision, schedule)
    try:
        fts = [gpu(f, dev) for f in fs]
        us = [np.zeros_like(f) for f in fs]
        for step in range(2):
            uts = [gpu(u, dev) for u in us]
            B.mg_vcycle(ctx, [t.data_ptr() for t in uts], [t.data_ptr() for t in fts], 1)
            for k, (n, _) in enumerate(specs):
                got = host(uts[k])
                if precision == 0:
                    ref = oracle.vcycle(us[k], fs[k], bc)
                    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
                    bound = 1e-12
                else:
                    ref = oracle.refine_step(us[k], fs[k], bc)
                    err = np.linalg.norm(got - ref) / np.linalg.norm(ref - us[k])
                    bound = 1e-5
                say(f"  step {step + 1} n={n}: {err:.2e}")
                assert err <= bound
                us[k] = ref
    finally:
        B.mg_destroy(ctx)


@pytest.mark.parametrize("schedule", [2, 3])
@pytest.mark.parametrize("precision", [0, 1])
def test_persistent_batch_solve(B, dev, schedule, precision):
    """Batched solve with the persistent (or phased) schedule: every problem
    reaches 1e-10 in the oracle's number of cycles (+-1), problems stopping
    independently, and matches the oracle's solution."""
    sizes = [129, 1025, 257, 129, 513, 257, 1025, 513]
    say(f"batch solve schedule={schedule} precision={precision}")
    specs = [(n, P) for n in sizes]
    fs = [workloads.rhs_divu_periodic(n, 1000 + k) for k, n in enumerate(sizes)]
    ctx = batch_ctx(B, specs, precision, schedule)
    try:
        fts = [gpu(f, dev) for f in fs]
        uts = [torch.zeros_like(t) for t in fts]
        st, cyc, rel = B.mg_solve(ctx, [t.data_ptr() for t in uts], [t.data_ptr() for t in fts],
                                  1e-10, 30)
        assert st == 0
        for k, f in enumerate(fs):
            if precision == 0:
                uo, co, ho = oracle.solve(f, P, rtol=1e-10, max_cycles=30)
            else:
                uo, co, ho = oracle.solve_mixed(f, P, rtol=1e-10, max_steps=30)
            say(f"  n={sizes[k]} cycles={cyc[k]} (oracle {co}) relres={rel[k]:.2e}")
            assert rel[k] <= 1e-10 and abs(cyc[k] - co) <= 1
            got = host(uts[k])
            uo = zero_mean(uo)
            assert np.linalg.norm(got - uo) <= 1e-9 * np.linalg.norm(uo)
    finally:
        B.mg_destroy(ctx)


@pytest.mark.parametrize("use_graph", [1, 0])
@pytest.mark.parametrize("schedule", [2, 3])
@pytest.mark.parametrize("bc,sizes", [(P, [257, 129, 513]), (D, [129, 257, 513]),
                                      (P, [65, 257])])
def test_batch_solve_norm_from_next_down_pass(B, dev, schedule, bc, sizes, use_graph):
    """Mixed batched mg_solve: when every problem's level 0 lies above the
    tail (sizes from 129 on), each check is the next step's down phases,
    whose level-0 items also write their sums of r^2, and the rest of that
    step runs only for the problems still unconverged; otherwise (a 65 x 65
    problem, its level 0 in the tail) the batched residual norm runs.  For 1,
    2 and 3 steps (check_every 1): each problem's iterate against the same
    number of mg_vcycle steps of the same batch, bit for bit (periodic: after
    the mean mg_solve removes), and its relative residual against the
    oracle's norm of the mg_vcycle iterate (1e-12 relative).  With and without
    captured launches."""
    say(f"batch norm from the next down pass schedule={schedule} bc={bc} sizes={sizes} "
        f"use_graph={use_graph}")
    specs = [(n, bc) for n in sizes]
    fs = [make_rhs(n, bc, 40 + k) for k, n in enumerate(sizes)]
    fts = [gpu(f, dev) for f in fs]
    for steps in (1, 2, 3):
        ctx = batch_ctx(B, specs, 1, schedule, check_every=1, use_graph=use_graph)
        uas = [torch.zeros_like(t) for t in fts]
        try:
            st, cyc, rel = B.mg_solve(ctx, [t.data_ptr() for t in uas],
                                      [t.data_ptr() for t in fts], 1e-300, steps)
        finally:
            B.mg_destroy(ctx)
        assert st == B.MG_ERR_NOT_CONVERGED
        ctx = batch_ctx(B, specs, 1, schedule, use_graph=use_graph)
        ubs = [torch.zeros_like(t) for t in fts]
        try:
            B.mg_vcycle(ctx, [t.data_ptr() for t in ubs], [t.data_ptr() for t in fts], steps)
        finally:
            B.mg_destroy(ctx)
        for k, n in enumerate(sizes):
            a, b = host(uas[k]), host(ubs[k])
            ref = oracle.relres(b, fs[k], bc)
            say(f"  {steps} steps n={n}: cycles {cyc[k]} relres {rel[k]:.6e} oracle {ref:.6e}")
            assert cyc[k] == steps
            assert abs(rel[k] - ref) <= 1e-12 * ref
            if bc == P:
                a, b = zero_mean(a), zero_mean(b)
                assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()
            else:
                assert np.array_equal(a, b)


def test_persistent_matches_per_problem_schedule(B, dev):
    sizes = [257, 65, 513]
    specs = [(n, P) for n in sizes]
    fs = [workloads.rhs_divu_periodic(n, 7 + k) for k, n in enumerate(sizes)]
    outs = []
    for schedule in (1, 2, 3):
        ctx = batch_ctx(B, specs, 1, schedule)
        fts = [gpu(f, dev) for f in fs]
        uts = [torch.zeros_like(t) for t in fts]
        rel = B.mg_vcycle(ctx, [t.data_ptr() for t in uts], [t.data_ptr() for t in fts], 3, True)
        outs.append(([host(t) for t in uts], rel))
        B.mg_destroy(ctx)
    for other in outs[1:]:
        for a, b in zip(outs[0][0], other[0]):
            assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(a)
        np.testing.assert_allclose(outs[0][1], other[1], rtol=1e-6)
    # The persistent and phased schedules run the same device functions on
    # the same items: bitwise equal.
    for a, b in zip(outs[1][0], outs[2][0]):
        assert np.array_equal(a, b)


def test_persistent_rejects_mixed_boundary_conditions(B, dev):
    o = B.mg_options_default()
    o.schedule = 2
    with pytest.raises(B.MGError) as ei:
        B.mg_setup([(65, P, 0), (65, D, 0)], o, 0)
    assert ei.value.status == B.MG_ERR_UNSUPPORTED


# ----------------------------------------------------------------- autotuner --

def device_arch():
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def read_tune_file(path):
    lines = [ln.split() for ln in open(path).read().splitlines() if ln.strip()]
    return [ln for ln in lines if ln[0] == "L"], [ln for ln in lines if ln[0] == "S"]


def run_cycles(B, ctx, fs, dev, k):
    fts = [gpu(f, dev) for f in fs]
    uts = [torch.zeros_like(t) for t in fts]
    B.mg_vcycle(ctx, [t.data_ptr() for t in uts], [t.data_ptr() for t in fts], k)
    return [host(t) for t in uts]


def test_autotune_writes_and_reuses_cache(B, dev, tmp_path):
    """schedule 0 measures a kernel choice for every streamed level and a
    schedule for the batch, records them in the cache file, reuses them on
    the next setup, and steps the same as the untuned per-problem schedule."""
    path = str(tmp_path / "tune.txt")
    sizes = [1025, 257, 513]
    specs = [(n, D) for n in sizes]
    fs = [make_rhs(n, D, 40 + k) for k, n in enumerate(sizes)]
    o = B.mg_options_default()
    o.tune_cache_path = path.encode()
    ctx = B.mg_setup([(n, bc, 0) for n, bc in specs], o, torch.cuda.current_stream().cuda_stream)
    try:
        tuned = run_cycles(B, ctx, fs, dev, 2)
    finally:
        B.mg_destroy(ctx)
    lv, sc = read_tune_file(path)
    arch = device_arch()
    tuned_sides = {int(ln[4]) for ln in lv if ln[1] == arch and ln[2] == "fp64" and ln[3] == "0"}
    # Every level above the single-workgroup tail (65) was measured, unless an
    # earlier setup in this process already had it.
    assert tuned_sides <= {1025, 513, 257, 129}
    for ln in lv:
        assert ln[5] in ("0", "1") and ln[7] in ("0", "1", "2")
        for hs in (int(ln[6]), int(ln[8])):  # rows per segment: 0 = default, else even
            assert hs == 0 or (hs > 0 and hs % 2 == 0 and hs <= int(ln[4]))
    assert len(sc) == 1 and sc[0][1] == arch and sc[0][4].startswith("B3:")
    assert sc[0][5] in ("1", "2", "3")
    say(f"tuned: {[' '.join(ln) for ln in lv + sc]}")
    # Second setup: everything comes from the cache, nothing is appended.
    before = open(path).read()
    ctx = B.mg_setup([(n, bc, 0) for n, bc in specs], o, torch.cuda.current_stream().cuda_stream)
    B.mg_destroy(ctx)
    assert open(path).read() == before
    ctx = batch_ctx(B, specs, 0, 1)
    try:
        ref = run_cycles(B, ctx, fs, dev, 2)
    finally:
        B.mg_destroy(ctx)
    for a, b in zip(tuned, ref):
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("bc", [D, P])
def test_tile_up_with_own_prefilter(B, dev, tmp_path, precision, bc):
    """Up-pass variant 2 (the LDS tiles prefilter their own coarse support,
    no separate prefilter pass), forced from a cache file on every level
    where it applies, gives the oracle's cycle."""
    n = 1025
    prec = "fp64" if precision == 0 else "fp32"
    top = "fp32a" if precision == 1 else prec
    path = tmp_path / "tune.txt"
    # Level-0 lines for the mixed path stay streaming (it adds into FP64).
    text = "".join(f"L {device_arch()} {top if m == n else prec} {bc} {m} 0 0 "
                   f"{0 if (m == n and precision == 1) else 2} 0 0\n"
                   for m in (1025, 513, 257, 129))
    path.write_text(text)
    o = B.mg_options_default()
    o.precision = precision
    o.tune_cache_path = str(path).encode()
    f = make_rhs(n, bc, 91)
    u0 = rand_grid(n, bc, np.random.default_rng(92)) * 1e-3
    ctx = B.mg_setup([(n, bc, 0)], o, torch.cuda.current_stream().cuda_stream)
    try:
        ut, ft = gpu(u0, dev), gpu(f, dev)
        B.mg_vcycle(ctx, [ut.data_ptr()], [ft.data_ptr()], 1)
        got = host(ut)
    finally:
        B.mg_destroy(ctx)
    assert path.read_text() == text  # nothing measured: all came from the file
    if precision == 0:
        ref = oracle.vcycle(u0, f, bc)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        bound = 1e-12
    else:
        ref = oracle.refine_step(u0, f, bc)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref - u0)
        bound = 1e-5
    say(f"tile up with own prefilter precision={precision} bc={bc}: {err:.2e}")
    assert err <= bound


@pytest.mark.parametrize("precision", [0, 1])
def test_autotune_cache_forces_variants(B, dev, tmp_path, precision):
    """Choices read from a cache file are applied: the LDS-tiled down pass
    and fixed segment heights on the streamed levels give the oracle's
    cycle."""
    n, bc = 2049, P
    prec = "fp64" if precision == 0 else "fp32"
    # The mixed path's level-0 up pass adds into the FP64 iterate, a kernel
    # variant of its own, tuned under the key "fp32a".
    top = "fp32a" if precision == 1 else prec
    path = tmp_path / "tune.txt"
    text = "".join(f"L {device_arch()} {top if m == n else prec} {bc} {m} 1 0 0 {hs} 0\n"
                   for m, hs in ((2049, 16), (1025, 8), (513, 32), (257, 64), (129, 8)))
    path.write_text(text)
    o = B.mg_options_default()
    o.precision = precision
    o.tune_cache_path = str(path).encode()
    f = make_rhs(n, bc, 77)
    u0 = zero_mean(make_rhs(n, bc, 78))
    ctx = B.mg_setup([(n, bc, 0)], o, torch.cuda.current_stream().cuda_stream)
    try:
        ut, ft = gpu(u0, dev), gpu(f, dev)
        B.mg_vcycle(ctx, [ut.data_ptr()], [ft.data_ptr()], 1)
        got = host(ut)
    finally:
        B.mg_destroy(ctx)
    assert path.read_text() == text  # nothing measured: all came from the file
    if precision == 0:
        ref = oracle.vcycle(u0, f, bc)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        bound = 1e-12
    else:
        ref = oracle.refine_step(u0, f, bc)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref - u0)
        bound = 1e-5
    say(f"forced variants n={n} precision={precision}: {err:.2e}")
    assert err <= bound
