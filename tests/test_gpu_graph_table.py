"""Captured steps read the caller's arrays through a device table.

mg_vcycle captures a problem's step into a hipGraph on its first call.  With
the default kernels that graph takes u and f from a per-problem device slot
that a call rewrites when its arrays differ from the last call's, so calls
that alternate between buffers reuse the one graph.  Checked here through
the C ABI: ten calls alternating two u buffers and two right-hand sides
(FP64 cycles and mixed refinement steps, both boundary conditions), each
call at the per-step parity bar against the oracle started from what that
buffer held, and no capture or instantiation after the first call
(mg_graph_stats).  The per-operation kernels take the arrays as kernel
arguments, so there a change of arrays captures the step again; that path
is checked for the same parity and for the captures it makes.

Bars as in the cycle parity tests: FP64 cycle <= 1e-12 relative to the
oracle's result; mixed step <= 1e-5 of the oracle's update (the FP32 inner
cycle rounds differently from the oracle's FP32 emulation)."""

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

D, P = 0, 1


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


def rhs(n, bc, seed):
    if bc == D:
        return workloads.rhs_divu_dirichlet(n, seed)
    return workloads.rhs_divu_periodic(n, seed)


def alternate(B, dev, n, bc, precision, kernel_path, calls=10):
    """Runs `calls` single-step calls alternating u buffers A/B and
    right-hand sides 1/2; returns the graph statistics after the first and
    after the last call."""
    o = B.mg_options_default()
    o.precision = precision
    o.use_graph = 1
    o.kernel_path = kernel_path
    ctx = B.mg_setup([(n, bc, 0)], o, torch.cuda.current_stream().cuda_stream)
    try:
        fs = [rhs(n, bc, 11), rhs(n, bc, 12)]
        ft = [torch.from_numpy(f).to(dev) for f in fs]
        us = [np.zeros_like(fs[0]), np.zeros_like(fs[0])]
        ut = [torch.zeros_like(ft[0]), torch.zeros_like(ft[0])]
        first = None
        for c in range(calls):
            a, b = c % 2, (c // 2) % 2
            B.mg_vcycle(ctx, [ut[a].data_ptr()], [ft[b].data_ptr()], 1)
            torch.cuda.synchronize()
            got = ut[a].cpu().numpy()
            if precision == 0:
                ref = oracle.vcycle(us[a], fs[b], bc)
                err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
                bar = 1e-12
            else:
                ref = oracle.refine_step(us[a], fs[b], bc)
                err = np.linalg.norm(got - ref) / np.linalg.norm(ref - us[a])
                bar = 1e-5
            say(f"  call {c}: u buffer {a}, f {b}: rel. diff {err:.2e}")
            assert err <= bar
            us[a] = got
            if c == 0:
                first = B.mg_graph_stats(ctx)
        return first, B.mg_graph_stats(ctx)
    finally:
        B.mg_destroy(ctx)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("bc,n", [(D, 257), (P, 257), (D, 1025), (P, 513)])
def test_one_graph_serves_alternating_buffers(B, dev, precision, bc, n):
    say(f"graph table: precision={precision} bc={bc} n={n}")
    first, last = alternate(B, dev, n, bc, precision, 0)
    say(f"  captures/instantiations after call 0: {first}, after call 9: {last}")
    assert first[0] >= 1 and first[1] >= 1
    assert last == first


def test_per_operation_path_captures_again(B, dev):
    say("graph table: per-operation path, alternating buffers")
    first, last = alternate(B, dev, 129, D, 0, 1)
    say(f"  captures/instantiations after call 0: {first}, after call 9: {last}")
    assert last[0] > first[0] and last[1] > first[1]
