"""The adversarial training of the SR model (Section 2.3: l_Dis, and l^SR =
l_MSE + 1e-3 l_Gen; Fig. 2b) on the GPU, and the trained generator in the
library's SR-CNN prolongation.

Training pairs come from the library's own solver (as in the trainer).  The
steps are checked for what the paper's alternation must do: finite losses,
each discriminator step separating real from generated windows further, both
networks moving.  The generator it leaves runs through the HIP SR-CNN kernels
at the SR-CNN parity bar (relative L2 <= 2e-2 against the oracle's forward
pass with the same weights)."""

import os

import numpy as np
import pytest

from oracle import srcnn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
W_MSE = os.path.join(ROOT, "paper_2403_07936_amd", "weights", "srcnn_divu_periodic.npy")
W_GAN = os.path.join(ROOT, "paper_2403_07936_amd", "weights", "srcnn_gan_divu_periodic.npy")


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


@pytest.fixture(scope="module")
def trained(dev, B):
    """Six adversarial steps from the supervised weights on solver pairs of
    257^2 periodic sources; returns (generator blob, per-step records)."""
    from paper_2403_07936_amd import srcnn_train as T
    torch.manual_seed(0)
    pairs = T.make_pairs(torch, 257, range(10000, 10006), dev)
    say(f"{len(pairs)} training pairs")
    groups = {}
    for x, y in pairs:
        groups.setdefault(x.shape[-1], []).append((x, y))
    gen = T.build_model(torch).to(dev)
    gen.load_blob(np.load(W_MSE))
    disc = T.build_discriminator(torch).to(dev)
    og = torch.optim.Adam(gen.parameters(), lr=1e-4)
    od = torch.optim.Adam(disc.parameters(), lr=1e-4)
    rng = np.random.default_rng(0)
    recs = []
    g0 = [p.detach().clone() for p in gen.parameters()]
    for step in range(6):
        N = sorted(groups)[step % len(groups)]
        X = torch.stack([p[0] for p in groups[N]])[:, None]
        Y = torch.stack([p[1] for p in groups[N]])[:, None]
        crops = T.crop_windows(torch, 2 * N, disc.window, 8, rng)
        rec = T.adversarial_step(torch, gen, disc, og, od, X, Y, crops, "mse")
        say(f"  step {step} (coarse side {N}): l_Dis {rec[0]:.4e} l^SR {rec[1]:.4e} "
            f"D(real) - D(fake) {rec[2]:+.4f} -> {rec[3]:+.4f}")
        recs.append(rec)
    moved = any(not torch.equal(a, b) for a, b in zip(g0, gen.parameters()))
    return gen.blob().astype(np.float32), recs, moved


def test_adversarial_steps_on_gpu(trained):
    _, recs, moved = trained
    for ld, lg, before, after in recs:
        assert np.isfinite(ld) and np.isfinite(lg)
        assert after > before
    assert moved


@pytest.mark.parametrize("lvl", [1, 2])
def test_gan_generator_in_the_library_matches_oracle(B, dev, trained, lvl):
    blob, _, _ = trained
    n = 257
    o = B.mg_options_default()
    o.prolong = B.MG_PROLONG_SRCNN
    o.cnn_levels = 0
    o.cnn_weights = blob.ctypes.data
    o.cnn_weights_bytes = blob.nbytes
    ctx = B.mg_setup([(n, 1, 0)], o, torch.cuda.current_stream().cuda_stream)
    try:
        nc = (n - 1) // 2 ** lvl + 1
        rng = np.random.default_rng(30 + lvl)
        k = np.fft.fftfreq(nc - 1)
        a = np.real(np.fft.ifft2(np.fft.fft2(rng.standard_normal((nc - 1, nc - 1)))
                                 * np.exp(-(k[:, None] ** 2 + k[None, :] ** 2) * 60.0)))
        ec = srcnn.with_seam(a - a.mean())
        ct = torch.from_numpy(ec).to(dev)
        ft = torch.full((2 * nc - 1, 2 * nc - 1), float("nan"), dtype=torch.float64, device=dev)
        B.mg_prolong(ctx, 0, lvl, B.MG_PROLONG_SRCNN, ct.data_ptr(), ft.data_ptr(), 0)
        torch.cuda.synchronize()
        got = ft.cpu().numpy()
        want = srcnn.prolong(ec, srcnn.unpack_weights(blob)).astype(np.float64)
        err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        say(f"GAN-trained generator, level {lvl}: rel L2 vs oracle {err:.3e}")
        assert err <= 2e-2
    finally:
        B.mg_destroy(ctx)
