"""mg_prolong_noalloc (spline prolongation with its scratch in a static
device array, for callers that cannot allocate) against mg_prolong (the same
operator with a context's workspace), through the C ABI.

Both run the same two kernels on the same inputs, so the outputs must be
equal bit for bit; they are also checked against the oracle's prolongation
at the operator's parity bar.  Two calls in a row on one device, the second
on a smaller grid, so the second starts from the first call's scratch
contents."""

import numpy as np
import pytest

import dense_model as dm
import oracle

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


def say(msg):
    print(msg, flush=True)


def coarse_grid(nc, bc, seed):
    rng = np.random.default_rng(seed)
    m = dm.m_of(nc, bc)
    return dm.to_grid(rng.standard_normal(m * m), nc, bc)


@pytest.mark.parametrize("dt", [F64, F32])
@pytest.mark.parametrize("bc", [D, P])
def test_noalloc_prolong_matches_mg_prolong(B, dev, bc, dt):
    npdt = np.float64 if dt == F64 else np.float32
    tdt = torch.float64 if dt == F64 else torch.float32
    stream = torch.cuda.current_stream().cuda_stream
    for call, nc in enumerate((1025, 129)):
        n = 2 * nc - 1
        say(f"no-alloc prolong call {call + 1}: bc={bc} dt={dt} nc={nc} -> n={n}")
        e = coarse_grid(nc, bc, 900 + 10 * call + bc).astype(npdt)
        et = torch.from_numpy(e).to(dev)
        got = torch.full((n, n), 7.0, device=dev, dtype=tdt)
        ref = torch.full((n, n), -7.0, device=dev, dtype=tdt)
        o = B.mg_options_default()
        ctx = B.mg_setup([(n, bc, 0)], o, stream)
        try:
            B.mg_prolong(ctx, 0, 1, B.MG_PROLONG_SPLINE, et.data_ptr(), ref.data_ptr(), dt)
            B.mg_prolong_noalloc(nc, bc, et.data_ptr(), got.data_ptr(), dt, stream)
            torch.cuda.synchronize()
        finally:
            B.mg_destroy(ctx)
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(g, r), np.abs(g - r).max()
        o_ref = oracle.prolong(e, bc)
        err = np.abs(g - o_ref).max() / np.abs(o_ref).max()
        say(f"  bitwise equal to mg_prolong; max diff vs oracle {err:.2e}")
        assert err <= (1e-13 if dt == F64 else 2e-6)


def test_noalloc_prolong_rejects_sizes_beyond_the_scratch(B, dev):
    a = torch.zeros((2049, 2049), device=dev, dtype=torch.float64)
    b = torch.zeros((4097, 4097), device=dev, dtype=torch.float64)
    with pytest.raises(B.MGError) as ei:
        B.mg_prolong_noalloc(2049, D, a.data_ptr(), b.data_ptr(), F64)
    assert ei.value.status == B.MG_ERR_UNSUPPORTED
    assert "1025" in ei.value.detail
