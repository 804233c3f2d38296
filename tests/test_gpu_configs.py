"""GPU parity for configurations the C ABI accepts beyond the defaults:
caller row pitches other than n, several FP32 cycles per refinement step,
smoothing counts other than two, the full 256-problem batch in one
persistent launch, the periodic 4097 x 4097 grid, and the persistent
schedule's barrier-timeout report.

Bars (as in test_gpu_parity.py): one FP64 cycle within 1e-12 of the
oracle's (relative 2-norm, and element-wise against the largest value);
one mixed refinement step within 1e-5 of the step's correction (FP32
rounding order against the oracle's FP32 emulation); solves to 1e-10 within
1e-9 of the oracle's FP64 solution and within one cycle of its count.
"""

import functools

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

D, P = oracle.DIRICHLET, oracle.PERIODIC


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


@functools.lru_cache(maxsize=8)
def rhs(n, bc, seed):
    if bc == D:
        return workloads.rhs_manufactured_dirichlet(n, seed) if n <= 65 else \
            workloads.rhs_divu_dirichlet(n, seed)
    return workloads.rhs_divu_periodic(n, seed)


def zero_mean(a):
    out = a.copy()
    core = a[:-1, :-1] - a[:-1, :-1].mean()
    out[:-1, :-1] = core
    out[-1, :-1] = core[0]
    out[:-1, -1] = core[:, 0]
    out[-1, -1] = core[0, 0]
    return out


def pitched(a, pitch, dev, fill=7.0):
    """(n, pitch) device array holding a in its first n columns and `fill`
    in the padding; returns the (n, n) view and the backing tensor."""
    n = a.shape[0]
    t = torch.full((n, pitch), fill, dtype=torch.float64, device=dev)
    t[:, :n] = torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return t[:, :n], t


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def check_cycle(got, ref, prev, fp64):
    """FP64: 2-norm and element-wise bars against the new iterate; mixed:
    against the step's correction ref - prev."""
    if fp64:
        l2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        mx = np.abs(got - ref).max() / np.abs(ref).max()
        assert l2 <= 1e-12 and mx <= 1e-12, (l2, mx)
    else:
        e = ref - prev
        l2 = np.linalg.norm(got - ref) / np.linalg.norm(e)
        mx = np.abs(got - ref).max() / np.abs(e).max()
        assert l2 <= 1e-5 and mx <= 1e-5, (l2, mx)
    return l2, mx


# ------------------------------------------------------------- caller pitch --

PITCH_CASES = [(257, 259), (257, 320), (4097, 4099), (4097, 4160)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("bc", [D, P])
@pytest.mark.parametrize("n,pitch", PITCH_CASES)
def test_pitched_cycle_parity(B, dev, n, pitch, bc, precision):
    """mg_vcycle on level-0 arrays whose rows are `pitch` elements apart (odd:
    odd rows start at odd elements; padded: a multiple of 64), one cycle from
    a nonzero state, against the oracle; the padding is never written."""
    from paper_2403_07936_amd.solver import Solver
    say(f"pitched cycle n={n} pitch={pitch} bc={bc} {precision}")
    f = rhs(n, bc, 31)
    u1 = oracle.vcycle(np.zeros_like(f), f, bc)
    uv, ub = pitched(u1, pitch, dev)
    fv, fb = pitched(f, pitch, dev, fill=-3.0)
    s = Solver([(n, bc)], precision=precision, pitch=[pitch])
    try:
        s.vcycle([uv], [fv], 1)
        got_full = host(ub)
    finally:
        s.close()
    assert np.all(got_full[:, n:] == 7.0)
    assert np.all(host(fb)[:, n:] == -3.0)
    got = got_full[:, :n]
    ref = oracle.vcycle(u1, f, bc) if precision == "fp64" else oracle.refine_step(u1, f, bc)
    l2, mx = check_cycle(got, ref, u1, precision == "fp64")
    say(f"  l2 {l2:.2e} max {mx:.2e}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("bc", [D, P])
@pytest.mark.parametrize("n,pitch", PITCH_CASES)
def test_pitched_solve_matches_oracle(B, dev, n, pitch, bc, precision):
    """mg_solve to 1e-10 on pitched arrays reaches the oracle's solution."""
    from paper_2403_07936_amd.solver import Solver
    say(f"pitched solve n={n} pitch={pitch} bc={bc} {precision}")
    f = rhs(n, bc, 32)
    uv, ub = pitched(np.zeros_like(f), pitch, dev)
    fv, _ = pitched(f, pitch, dev, fill=-3.0)
    s = Solver([(n, bc)], precision=precision, pitch=[pitch])
    try:
        st, cyc, rel = s.solve([uv], [fv], rtol=1e-10, max_cycles=30)
        got_full = host(ub)
    finally:
        s.close()
    if precision == "fp64":
        uo, co, _ = oracle.solve(f, bc, rtol=1e-10, max_cycles=30)
    else:
        uo, co, _ = oracle.solve_mixed(f, bc, rtol=1e-10, max_steps=30)
    if bc == P:
        uo = zero_mean(uo)
    got = got_full[:, :n]
    err = np.linalg.norm(got - uo) / np.linalg.norm(uo)
    say(f"  status {st} cycles {cyc[0]} (oracle {co}) relres {rel[0]:.2e} err {err:.2e}")
    assert st == 0 and rel[0] <= 1e-10 and abs(cyc[0] - co) <= 1
    assert err <= 1e-9
    assert np.all(got_full[:, n:] == 7.0)


# ------------------------------------------------ inner cycles, sweep counts --

@pytest.mark.parametrize("inner", [2, 3])
@pytest.mark.parametrize("kernel_path", [0, 1])
@pytest.mark.parametrize("bc,n", [(D, 257), (P, 257), (D, 1025), (P, 1025)])
def test_inner_cycles_parity(B, dev, inner, kernel_path, bc, n):
    """MG_MIXED with `inner` FP32 cycles per refinement step (the first from
    e = 0, the last adding into the FP64 iterate) against the oracle's
    refine_step with the same count, three steps in a row.

    Bar.  From the second inner cycle on, the FP32 cycle restarts from the
    FP32 residual r - A e, whose smooth part is mostly rounding (A scales by
    1/h^2 and the terms cancel), so the step depends on the rounding order at
    the level of FP32 noise amplified by the cycle.  The natural spread D is
    measured here on the oracle itself, as the larger of two distances: its
    FP32 step from the same step with FP64 inner cycles, and its FP32 step
    from the FP32 step of the transposed problem transposed back (the same
    operations with x and y swapped, so only the rounding order differs).
    At 257^2 and 1025^2 the second is 1-4x the first (e.g. 1.6e-5 against
    1.25e-5 of |e|, periodic 1025^2, 3 inner cycles), and an FMA-contracted
    build of the oracle lies as far.  The GPU step (contracted, its own
    order) must lie within 3 D of the oracle's step, L2 and max norm, and
    never further than 1e-5 |e| when D is smaller; its FP64 residual must be
    as small as the oracle's (within 5 %)."""
    from paper_2403_07936_amd.solver import Solver
    say(f"inner cycles {inner} path {kernel_path} bc={bc} n={n}")
    f = rhs(n, bc, 33)
    s = Solver([(n, bc)], precision="mixed", inner_cycles=inner, kernel_path=kernel_path)
    try:
        ft = torch.from_numpy(f).to(dev)
        u = np.zeros_like(f)
        for step in range(3):
            ut = torch.from_numpy(u.copy()).to(dev)
            s.vcycle([ut], [ft], 1)
            got = host(ut)
            ref = oracle.refine_step(u, f, bc, inner=inner)
            r = oracle.residual(u, f, bc)
            e64 = np.zeros_like(f)
            for _ in range(inner):
                e64 = oracle.vcycle(e64, r, bc)
            tr = np.ascontiguousarray(oracle.refine_step(
                np.ascontiguousarray(u.T), np.ascontiguousarray(f.T), bc, inner=inner).T)
            e = ref - u

            def dist(a, b):
                return (np.linalg.norm(a - b) / np.linalg.norm(e),
                        np.abs(a - b).max() / np.abs(e).max())

            d64, dtr = dist(ref, u + e64), dist(ref, tr)
            d_l2, d_mx = max(d64[0], dtr[0]), max(d64[1], dtr[1])
            l2, mx = dist(got, ref)
            rg, ro = oracle.relres(got, f, bc), oracle.relres(ref, f, bc)
            say(f"  step {step + 1}: l2 {l2:.2e} max {mx:.2e} (oracle FP32 vs FP64 inner: "
                f"{d64[0]:.2e} / {d64[1]:.2e}, vs transposed order: {dtr[0]:.2e} / "
                f"{dtr[1]:.2e}); relres {rg:.3e} oracle {ro:.3e}")
            assert l2 <= max(1e-5, 3.0 * d_l2) and mx <= max(1e-5, 3.0 * d_mx)
            assert rg <= 1.05 * ro
            u = ref
    finally:
        s.close()


@pytest.mark.parametrize("nu", [(1, 1), (3, 3), (1, 3), (0, 2), (3, 0)])
@pytest.mark.parametrize("bc,n", [(D, 129), (P, 129), (D, 513), (P, 513)])
def test_sweep_counts_fp64_parity(B, dev, nu, bc, n):
    """V(nu_pre, nu_post) cycles with sweep counts other than two (the
    per-operation schedule) against the oracle's vcycle(nu1, nu2)."""
    from paper_2403_07936_amd.solver import Solver
    say(f"sweeps {nu} bc={bc} n={n}")
    f = rhs(n, bc, 34)
    s = Solver([(n, bc)], precision="fp64", nu_pre=nu[0], nu_post=nu[1])
    try:
        ft = torch.from_numpy(f).to(dev)
        u = np.zeros_like(f)
        for c in range(3):
            ut = torch.from_numpy(u.copy()).to(dev)
            s.vcycle([ut], [ft], 1)
            ref = oracle.vcycle(u, f, bc, nu[0], nu[1])
            l2, mx = check_cycle(host(ut), ref, u, True)
            say(f"  cycle {c + 1}: l2 {l2:.2e} max {mx:.2e}")
            u = ref
    finally:
        s.close()


@pytest.mark.parametrize("nu", [(1, 1), (3, 3)])
@pytest.mark.parametrize("bc", [D, P])
def test_sweep_counts_mixed_parity(B, dev, nu, bc):
    from paper_2403_07936_amd.solver import Solver
    n = 257
    say(f"mixed sweeps {nu} bc={bc} n={n}")
    f = rhs(n, bc, 35)
    s = Solver([(n, bc)], precision="mixed", nu_pre=nu[0], nu_post=nu[1])
    try:
        ft = torch.from_numpy(f).to(dev)
        u = np.zeros_like(f)
        for step in range(2):
            ut = torch.from_numpy(u.copy()).to(dev)
            s.vcycle([ut], [ft], 1)
            ref = oracle.refine_step(u, f, bc, nu1=nu[0], nu2=nu[1])
            l2, mx = check_cycle(host(ut), ref, u, False)
            say(f"  step {step + 1}: l2 {l2:.2e} max {mx:.2e}")
            u = ref
    finally:
        s.close()


# ------------------------------------------------------- periodic 4097^2 --

@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_periodic4097_cycle_parity(B, dev, precision):
    """One cycle of the periodic 4097 x 4097 grid (1024 wavenumbers) from a
    nonzero state, in the benchmark's launch configuration."""
    from paper_2403_07936_amd.solver import Solver
    n, bc = 4097, P
    say(f"periodic 4097 {precision}")
    f = rhs(n, bc, 36)
    u1 = oracle.vcycle(np.zeros_like(f), f, bc)
    s = Solver([(n, bc)], precision=precision)
    try:
        ut = torch.from_numpy(u1.copy()).to(dev)
        ft = torch.from_numpy(f).to(dev)
        s.vcycle([ut], [ft], 1)
        got = host(ut)
    finally:
        s.close()
    ref = oracle.vcycle(u1, f, bc) if precision == "fp64" else oracle.refine_step(u1, f, bc)
    l2, mx = check_cycle(got, ref, u1, precision == "fp64")
    say(f"  l2 {l2:.2e} max {mx:.2e}")


# -------------------------------------------------- the 256-problem batch --

@functools.lru_cache(maxsize=1)
def batch256():
    return workloads.workload("batch256", 0)


@pytest.mark.parametrize("schedule", [2, 3])
def test_batch256_persistent_step_parity(B, dev, schedule):
    """One persistent launch (schedule 2) or one launch per phase (3) steps
    all 256 problems of the batched workload (sides 129..1025, mixed
    precision); each problem's new iterate is checked element-wise against
    the oracle's refinement step from the same nonzero state."""
    probs = batch256()
    say(f"batch256 schedule {schedule}: {len(probs)} problems, "
        f"{sum((n - 1) ** 2 for n, _, _ in probs)} unknowns")
    o = B.mg_options_default()
    o.precision = B.MG_MIXED
    o.schedule = schedule
    ctx = B.mg_setup([(n, bc, 0) for n, bc, _ in probs], o,
                     torch.cuda.current_stream().cuda_stream)
    try:
        # A nonzero start: one oracle FP64 cycle per problem.
        starts = [oracle.vcycle(np.zeros_like(f), f, bc) for n, bc, f in probs]
        uts = [torch.from_numpy(u.copy()).to(dev) for u in starts]
        fts = [torch.from_numpy(f).to(dev) for _, _, f in probs]
        B.mg_vcycle(ctx, [t.data_ptr() for t in uts], [t.data_ptr() for t in fts], 1)
        worst = (0.0, 0.0)
        for k, (n, bc, f) in enumerate(probs):
            ref = oracle.refine_step(starts[k], f, bc)
            l2, mx = check_cycle(host(uts[k]), ref, starts[k], False)
            worst = (max(worst[0], l2), max(worst[1], mx))
        say(f"  worst over the batch: l2 {worst[0]:.2e} max {worst[1]:.2e}")
    finally:
        B.mg_destroy(ctx)


# ------------------------------------------------ barrier timeout report --

def test_phased_schedule_has_no_barrier_to_mark(B, dev):
    """The phased schedule (3) orders its phases by kernel boundaries; the
    diagnostic that marks the device barrier refuses it."""
    o = B.mg_options_default()
    o.precision = B.MG_MIXED
    o.schedule = 3
    ctx = B.mg_setup([(n, P, 0) for n in (129, 257)], o, torch.cuda.current_stream().cuda_stream)
    try:
        with pytest.raises(B.MGError) as ei:
            B.mg_persistent_mark_timeout(ctx)
        assert ei.value.status == B.MG_ERR_UNSUPPORTED
    finally:
        B.mg_destroy(ctx)


@pytest.mark.parametrize("call", ["vcycle", "solve"])
def test_persistent_barrier_timeout_is_reported(B, dev, call):
    """A timed-out device barrier (marked from the host, so every workgroup
    exits at entry and nothing spins) makes the call that queued the launch
    return MG_ERR_HIP, also without a residual request; the mark is then
    cleared and the next call steps normally."""
    sizes = [129, 257, 65]
    fs = [rhs(n, P, 40 + k) for k, n in enumerate(sizes)]
    o = B.mg_options_default()
    o.precision = B.MG_MIXED
    o.schedule = 2
    ctx = B.mg_setup([(n, P, 0) for n in sizes], o, torch.cuda.current_stream().cuda_stream)
    try:
        fts = [torch.from_numpy(f).to(dev) for f in fs]
        uts = [torch.zeros_like(t) for t in fts]
        B.mg_persistent_mark_timeout(ctx)
        with pytest.raises(B.MGError) as ei:
            if call == "vcycle":
                B.mg_vcycle(ctx, [t.data_ptr() for t in uts], [t.data_ptr() for t in fts], 1)
            else:
                B.mg_solve(ctx, [t.data_ptr() for t in uts], [t.data_ptr() for t in fts],
                           1e-10, 5)
        assert ei.value.status == B.MG_ERR_HIP
        for t in uts:  # the launch exited at entry: nothing was written
            assert np.abs(host(t)).max() == 0.0
        B.mg_vcycle(ctx, [t.data_ptr() for t in uts], [t.data_ptr() for t in fts], 1)
        for k, f in enumerate(fs):
            ref = oracle.refine_step(np.zeros_like(f), f, P)
            check_cycle(host(uts[k]), ref, np.zeros_like(f), False)
    finally:
        B.mg_destroy(ctx)
    o.schedule = 1
    ctx = B.mg_setup([(65, P, 0)], o, torch.cuda.current_stream().cuda_stream)
    try:
        with pytest.raises(B.MGError) as ei:
            B.mg_persistent_mark_timeout(ctx)
        assert ei.value.status == B.MG_ERR_UNSUPPORTED
    finally:
        B.mg_destroy(ctx)
