"""CPU pins of the adversarial-training oracle (Section 2.3's losses after
Ledig et al.; Fig. 2b's discriminator) and parity of the trainer's PyTorch
versions against it.

Pins: the convolution against torch.nn.functional.conv2d (a library routine)
and a one-tap orientation check; the whole discriminator against the closed
form of hand-set weights (centre taps, identity and weighted dense layers:
it reads x at the strided positions in channel-first order); the losses
against closed forms (log 2, c^2, N log 2, the 1e-3 weight)."""

import numpy as np
import pytest

import oracle.gan as G

torch = pytest.importorskip("torch")


def rand_params(rng, widths, window, dense):
    return [rng.standard_normal(s) * (0.5 / np.sqrt(np.prod(s[1:])) if len(s) > 1 else 0.1)
            for s in G.param_shapes(widths, window, dense)]


@pytest.mark.parametrize("stride", [1, 2])
@pytest.mark.parametrize("side", [5, 8, 24])
def test_conv_matches_torch(stride, side):
    rng = np.random.default_rng(side + stride)
    x = rng.standard_normal((3, side, side))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    got = G.conv2d(x, w, b, stride)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x)[None], torch.from_numpy(w),
                                     torch.from_numpy(b), stride=stride, padding=1)[0].numpy()
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 1e-12


def test_conv_is_a_cross_correlation():
    x = np.zeros((1, 5, 5))
    x[0, 2, 3] = 1.0          # one node right of the centre
    w = np.zeros((1, 1, 3, 3))
    w[0, 0, 1, 2] = 7.0       # the tap that reads the right neighbour
    out = G.conv2d(x, w, np.zeros(1), 1)
    assert out[0, 2, 2] == 7.0 and np.count_nonzero(out) == 1


def test_discriminator_closed_form():
    """Centre taps of 1, zero biases, positive input: every conv passes its
    input through (stride 2 keeps the even nodes), so the last 2 x 2 map of
    a 24 x 24 window holds x at rows and columns 0 and 16; an identity dense
    layer and output weights (1, 2, 3, 4) give sigmoid(x00 + 2 x0,16 +
    3 x16,0 + 4 x16,16), which fixes the strides, the padding and the
    channel-first flatten order."""
    widths = (1,) * 8
    params = []
    for _ in widths:
        w = np.zeros((1, 1, 3, 3))
        w[0, 0, 1, 1] = 1.0
        params += [w, np.zeros(1)]
    params += [np.eye(4), np.zeros(4), np.array([[1.0, 2.0, 3.0, 4.0]]), np.zeros(1)]
    rng = np.random.default_rng(3)
    x = rng.uniform(0.1, 1.0, (2, 1, 24, 24)) * 0.2
    got = G.discriminator(params, x)
    for b in range(2):
        z = x[b, 0, 0, 0] + 2 * x[b, 0, 0, 16] + 3 * x[b, 0, 16, 0] + 4 * x[b, 0, 16, 16]
        assert abs(got[b] - 1.0 / (1.0 + np.exp(-z))) <= 1e-15


def test_discriminator_zero_weights_is_one_half():
    shapes = G.param_shapes((4, 4, 8, 8, 8, 8, 8, 8), 24, 16)
    params = [np.zeros(s) for s in shapes]
    x = np.random.default_rng(1).standard_normal((3, 1, 24, 24))
    assert np.all(G.discriminator(params, x) == 0.5)


def test_leaky_relu_slope():
    assert np.array_equal(G.leaky_relu(np.array([-2.0, 0.0, 3.0])), np.array([-0.4, 0.0, 3.0]))


def test_losses_closed_forms():
    assert abs(G.bce(np.full(5, 0.5), 1.0) - np.log(2)) <= 1e-15
    assert abs(G.bce(np.full(5, 0.5), 0.0) - np.log(2)) <= 1e-15
    assert abs(G.bce(np.array([np.exp(-1.0)]), 1.0) - 1.0) <= 1e-15
    assert abs(G.dis_loss(np.full(3, 0.5), np.full(3, 0.5)) - 2 * np.log(2)) <= 1e-15
    assert G.dis_loss(np.full(3, 1 - 1e-12), np.full(3, 1e-12)) <= 1e-11
    hr = np.random.default_rng(0).standard_normal((2, 1, 8, 8))
    assert G.mse_loss(hr, hr) == 0.0
    assert abs(G.mse_loss(hr, hr + 0.25) - 0.0625) <= 1e-15
    assert G.gen_loss(np.ones(4)) == 0.0
    assert abs(G.gen_loss(np.full(4, 0.5)) - 4 * np.log(2)) <= 1e-14
    d = np.array([0.3, 0.9])
    assert abs(G.sr_loss(hr, hr + 0.5, d) - (0.25 + 1e-3 * (-np.log(0.3) - np.log(0.9)))) <= 1e-15


# ---- the trainer's PyTorch versions against the oracle (CPU, float64) ----

def test_trainer_discriminator_matches_oracle():
    from paper_2403_07936_amd import srcnn_train as T
    widths, window, dense = (4, 4, 8, 8, 8, 8, 16, 16), 24, 32
    rng = np.random.default_rng(7)
    params = rand_params(rng, widths, window, dense)
    D = T.build_discriminator(torch, widths, window, dense).double()
    T.set_discriminator_params(torch, D, params)
    x = rng.standard_normal((3, 1, window, window))
    got = D(torch.from_numpy(x)).detach().numpy().reshape(-1)
    ref = G.discriminator(params, x)
    assert np.abs(got - ref).max() <= 1e-13


def test_trainer_losses_match_oracle():
    from paper_2403_07936_amd import srcnn_train as T
    rng = np.random.default_rng(8)
    hr = rng.standard_normal((4, 1, 16, 16))
    sr = rng.standard_normal((4, 1, 16, 16))
    dr = rng.uniform(0.05, 0.95, 4)
    df = rng.uniform(0.05, 0.95, 4)
    t = torch.from_numpy
    assert abs(float(T.dis_loss(torch, t(dr), t(df))) - G.dis_loss(dr, df)) <= 1e-14
    assert abs(float(T.mse_loss(torch, t(hr), t(sr))) - G.mse_loss(hr, sr)) <= 1e-14
    assert abs(float(T.gen_loss(torch, t(df))) - G.gen_loss(df)) <= 1e-14
    assert abs(float(T.sr_loss(torch, t(hr), t(sr), t(df))) - G.sr_loss(hr, sr, df)) <= 1e-14


def test_adversarial_step_on_cpu():
    """A few alternating steps on tiny synthetic pairs (CPU): the losses stay
    finite, both networks' parameters move, and the discriminator step
    raises D on real windows relative to generated ones."""
    from paper_2403_07936_amd import srcnn_train as T
    torch.manual_seed(0)
    rng = np.random.default_rng(9)
    N = 16
    x = torch.from_numpy(rng.standard_normal((4, 1, N, N)).astype(np.float32))
    y = torch.nn.functional.interpolate(x, scale_factor=2, mode="bilinear", align_corners=False)
    gen = T.build_model(torch)
    disc = T.build_discriminator(torch, (4, 4, 8, 8, 8, 8, 16, 16), 24, 32)
    og = torch.optim.Adam(gen.parameters(), lr=1e-3)
    od = torch.optim.Adam(disc.parameters(), lr=1e-3)
    g0 = [p.detach().clone() for p in gen.parameters()]
    d0 = [p.detach().clone() for p in disc.parameters()]
    crops = T.crop_windows(torch, y.shape[-1], 24, 2, np.random.default_rng(1))
    for _ in range(5):
        ld, lg, before, after = T.adversarial_step(torch, gen, disc, og, od, x, y, crops,
                                                   content="mse")
        assert np.isfinite(ld) and np.isfinite(lg)
        assert after > before
    assert any(not torch.equal(a, b) for a, b in zip(g0, gen.parameters()))
    assert any(not torch.equal(a, b) for a, b in zip(d0, disc.parameters()))
