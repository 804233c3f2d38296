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
