"""Pins of the SR-CNN prolongation oracle (oracle/srcnn.py).

Each check ties the oracle to something other than itself: the bfloat16
rounding to torch's conversion, the convolution to a brute-force loop and
to torch's own padding, the pixel shuffle to torch's, the whole network to
the closed form of hand-set weights that make it a known linear
interpolation (exact in dyadic arithmetic), and the CNN V-cycle to the dense
matrix model with the same prolongation plugged in.
"""

import numpy as np
import pytest

import dense_model as dm
import oracle
from oracle import srcnn
from srcnn_weights import linear_interp, linear_layers, random_layers

torch = pytest.importorskip("torch")
P = oracle.PERIODIC


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** rng.integers(-30, 30, 20000),
        # exact ties: the bf16 value plus half its ulp, for even and odd bf16 mantissas
        (np.arange(1, 2000, dtype=np.uint32) << 16 | 0x8000).view(np.float32),
        np.array([0.0, -0.0, 1e-40, -3e-39, 3.3895e38], dtype=np.float32),
    ])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(srcnn.bf16_round(x), want)


def brute_conv(x, w, circular):
    cin, h, wd = x.shape
    cout = w.shape[0]
    if circular:
        out = np.zeros((cout, h, wd))
        for o in range(cout):
            for y in range(h):
                for xx in range(wd):
                    s = 0.0
                    for i in range(cin):
                        for ky in range(3):
                            for kx in range(3):
                                s += float(w[o, i, ky, kx]) * float(x[i, (y + ky - 1) % h, (xx + kx - 1) % wd])
                    out[o, y, xx] = s
        return out
    out = np.zeros((cout, h - 2, wd - 2))
    for o in range(cout):
        for y in range(h - 2):
            for xx in range(wd - 2):
                out[o, y, xx] = sum(float(w[o, i, ky, kx]) * float(x[i, y + ky, xx + kx])
                                    for i in range(cin) for ky in range(3) for kx in range(3))
    return out


@pytest.mark.parametrize("circular", [True, False])
def test_conv3x3_matches_brute_force(circular):
    rng = np.random.default_rng(1)
    x = srcnn.bf16_round(rng.standard_normal((3, 6, 5)).astype(np.float32))
    w = srcnn.bf16_round(rng.standard_normal((4, 3, 3, 3)).astype(np.float32))
    got = srcnn.conv3x3(x, w, circular)
    want = brute_conv(x, w, circular)
    np.testing.assert_allclose(got, want.astype(np.float32), rtol=1e-6, atol=1e-6)
    # Orientation: a single tap at (ky, kx) = (2, 0) reads x[y + 1, x - 1].
    w1 = np.zeros((1, 1, 3, 3), np.float32)
    w1[0, 0, 2, 0] = 1.0
    got = srcnn.conv3x3(x[:1], w1, True)[0]
    np.testing.assert_array_equal(got, np.roll(np.roll(x[0], -1, axis=0), 1, axis=1))


def test_pixel_shuffle_matches_torch():
    rng = np.random.default_rng(2)
    y = rng.standard_normal((12, 4, 5)).astype(np.float32)
    want = torch.nn.functional.pixel_shuffle(torch.from_numpy(y)[None], 2)[0].numpy()
    np.testing.assert_array_equal(srcnn.pixel_shuffle(y), want)


def test_weight_count():
    # stem 1*64*9, 16 body convs 64*64*9, up 64*256*9, final 64*9
    assert srcnn.WEIGHT_COUNT == 576 + 16 * 36864 + 147456 + 576


# --------------------------------------------------- hand-set weights pins --

def test_network_closed_form_with_hand_set_weights():
    rng = np.random.default_rng(3)
    e = rng.integers(-16, 17, (12, 12)).astype(np.float64)
    e[5, 7] = -16.0
    got = srcnn.forward(e, linear_layers())
    np.testing.assert_array_equal(got, linear_interp(e).astype(np.float32))
    # Scaling by s = max|e|: any power-of-two multiple gives the same
    # interpolant times that multiple.
    got = srcnn.forward(e * 2.0 ** -20, linear_layers())
    np.testing.assert_array_equal(got, (linear_interp(e) * 2.0 ** -20).astype(np.float32))


def test_network_is_homogeneous_and_shift_equivariant():
    rng = np.random.default_rng(4)
    layers = random_layers(5)
    e = rng.standard_normal((16, 16))
    base = srcnn.forward(e, layers)
    assert np.abs(base).max() > 0
    np.testing.assert_array_equal(srcnn.forward(e * 8.0, layers), base * 8.0)
    shifted = srcnn.forward(np.roll(e, (3, -2), axis=(0, 1)), layers)
    np.testing.assert_allclose(shifted, np.roll(base, (6, -4), axis=(0, 1)), rtol=1e-6,
                               atol=1e-6 * np.abs(base).max())
    assert not np.any(srcnn.forward(np.zeros((8, 8)), layers))


def test_window_matches_whole_forward():
    rng = np.random.default_rng(6)
    layers = random_layers(7)
    e = rng.standard_normal((24, 24))
    whole = srcnn.forward(e, layers)
    for y0, x0, h, w in ((0, 0, 4, 3), (21, 22, 3, 5), (10, 3, 2, 2)):
        got = srcnn.forward_window(e, layers, y0, x0, h, w)
        rows = np.arange(2 * y0, 2 * (y0 + h)) % 48
        cols = np.arange(2 * x0, 2 * (x0 + w)) % 48
        np.testing.assert_allclose(got, whole[np.ix_(rows, cols)], rtol=1e-5,
                                   atol=1e-6 * np.abs(whole).max())


@pytest.mark.parametrize("levels", [1, 2])
def test_cnn_vcycle_matches_dense_model(levels):
    """The oracle's cycle with the network on the finest prolongations equals
    the dense model's cycle with the same prolongation plugged in."""
    n = 17
    layers = random_layers(8, scale=0.5)
    rng = np.random.default_rng(9)
    f = dm.to_grid(rng.standard_normal(dm.m_of(n, P) ** 2), n, P)
    f = f - f[:-1, :-1].mean()
    f = dm.to_grid(dm.to_vec(f, P), n, P)
    u0 = dm.to_grid(rng.standard_normal(dm.m_of(n, P) ** 2), n, P)
    got = srcnn.vcycle(u0, f, layers, levels)

    def plug(uc_vec, nc):
        return dm.to_vec(srcnn.prolong(dm.to_grid(uc_vec, nc, P), layers), P)

    want = dm.vcycle(dm.to_vec(u0, P), dm.to_vec(f, P), n, P, prolong=plug, levels=levels)
    np.testing.assert_allclose(dm.to_vec(got, P), want, rtol=0, atol=1e-10 * np.abs(want).max())


def test_mixed_refine_step_with_zero_network_levels_is_plain():
    n = 33
    rng = np.random.default_rng(10)
    f = dm.to_grid(rng.standard_normal(dm.m_of(n, P) ** 2), n, P)
    f = dm.to_grid(dm.to_vec(f - f[:-1, :-1].mean(), P), n, P)
    u = np.zeros_like(f)
    np.testing.assert_array_equal(srcnn.refine_step(u, f, None, 0), oracle.refine_step(u, f, P))


# Hybrid prolongation schedule (Table 1's N_GAN and S_thres; appendix
# V-CYCLE).  The pins restate what Sections 3 and 4 say the parameters do.

N_ITER = 300  # the paper's iteration cap (Table 1)


@pytest.mark.parametrize("n_gan", [1.0, 5.0, 10.0, 1 / 5, 1 / 10])
def test_schedule_n_gan_counts_network_per_spline(n_gan):
    """N_GAN network prolongations per spline one (N_GAN >= 1), or 1/N_GAN
    spline ones per network one; the first iteration uses the first
    operator."""
    ops = [srcnn.prolongation_choice(i, n_gan, False) for i in range(1, 121)]
    first = n_gan >= 1.0
    N = round(n_gan if first else 1.0 / n_gan)
    assert ops[0] == first
    for k in range(0, 120 - N):
        window = ops[k:k + N + 1]
        assert window.count(first) == N and window.count(not first) == 1


def test_schedule_n_gan_one_alternates():
    ops = [srcnn.prolongation_choice(i, 1.0, False) for i in range(1, 11)]
    assert ops == [True, False] * 5


@pytest.mark.parametrize("n_gan,only", [(N_ITER, True), (1 / N_ITER, False)])
def test_schedule_edge_values_use_one_operator(n_gan, only):
    """N_GAN = N_iter is network-only and 1/N_iter spline-only over N_iter
    iterations; a set switch always selects the second operator."""
    assert all(srcnn.prolongation_choice(i, n_gan, False) == only for i in range(1, N_ITER + 1))
    assert all(srcnn.prolongation_choice(i, n_gan, True) == (not only) for i in range(1, 50))


def schedule_rhs(n, scale=1.0):
    import workloads
    return workloads.rhs_divu_periodic(n, 5) * scale


def test_schedule_single_operator_solves_are_plain_cycles():
    """Network-only and spline-only schedules reproduce repeated network and
    spline cycles bit for bit."""
    n, levels, cycles = 65, 1, 4
    layers = linear_layers()
    f = schedule_rhs(n)
    u_net, ops, _, _ = srcnn.solve_schedule(f, layers, levels, 0.0, cycles, N_ITER, 0.0)
    u_spl, ops_s, _, _ = srcnn.solve_schedule(f, layers, levels, 0.0, cycles, 1 / N_ITER, 0.0)
    a = np.zeros_like(f)
    b = np.zeros_like(f)
    for _ in range(cycles):
        a = srcnn.vcycle(a, f, layers, levels)
        b = oracle.vcycle(b, f, P)
    assert ops == [True] * cycles and ops_s == [False] * cycles
    np.testing.assert_array_equal(u_net, a)
    np.testing.assert_array_equal(u_spl, b)


@pytest.mark.parametrize("n_gan", [N_ITER, 1 / N_ITER, 1.0])
def test_schedule_threshold_one_switches_after_the_first_iteration(n_gan):
    """S_thres = 1 switches to the second operator right after the first
    iteration when the iterates change by less than 1 (pressure-sized
    values, Section 4)."""
    layers = linear_layers()
    f = schedule_rhs(65, 1e-4)
    _, ops, diffs, _ = srcnn.solve_schedule(f, layers, 1, 0.0, 6, n_gan, 1.0)
    assert diffs[0] <= 1.0
    first = n_gan >= 1.0
    assert ops == [first] + [not first] * 5


def test_schedule_switch_follows_the_previous_iteration_change():
    """The switch is set by the change the previous iteration made: with
    S_thres between the changes of iterations 3 and 4 the first four
    iterations use the network and the rest the spline."""
    layers = linear_layers()
    f = schedule_rhs(65)
    _, ops0, d0, _ = srcnn.solve_schedule(f, layers, 1, 0.0, 8, N_ITER, 0.0)
    assert all(ops0) and d0[3] < d0[2]
    s = float(np.sqrt(d0[2] * d0[3]))
    _, ops, d, _ = srcnn.solve_schedule(f, layers, 1, 0.0, 8, N_ITER, s)
    assert ops == [True] * 4 + [False] * 4
    assert d[:4] == d0[:4]


@pytest.mark.parametrize("mixed", [False, True])
def test_schedule_alternating_solve_converges(mixed):
    layers = linear_layers()
    f = schedule_rhs(65)
    _, ops, _, rel = srcnn.solve_schedule(f, layers, 1, 1e-9, 40, 1.0, 0.0, mixed=mixed)
    assert rel <= 1e-9 and len(ops) < 40
    assert ops == [True, False] * (len(ops) // 2) + [True] * (len(ops) % 2)
