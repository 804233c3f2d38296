"""Plain CPU reference for the adversarial training of the SR model.

TEST INFRASTRUCTURE ONLY (see the package docstring): only the test suite,
the smoke check and the benchmark's CPU baseline leg may use it.

What it computes (Section 2.3, the GAN losses after Ledig et al.; Fig. 2b,
the discriminator and generator structure), in float64 numpy with plain
loops where the operation is small:

  l_Dis   = binary cross-entropy of the discriminator's outputs, real
            samples labelled 1 and generated ones 0;
  l^SR    = l^SR_MSE + 1e-3 l^SR_Gen;
  l^SR_MSE = (1 / (r^2 W H)) sum over the r W x r H fine pixels of
            (I^HR - G(I^LR))^2  (one channel here);
  l^SR_Gen = sum over the N samples of -log D(G(I^LR)).

Readings (listed in the design notes):
  * l_Dis is the mean binary cross-entropy over the real samples plus the
    mean over the generated ones (the paper names only "binary cross
    entropy"; step (ii) of its training trains D on both kinds).
  * The discriminator follows Ledig et al.'s: a 3x3 conv (stride 1) and
    LeakyReLU(0.2), then seven 3x3 convs with strides 2,1,2,1,2,1,2 and
    widths w1..w7, each followed by LeakyReLU(0.2), then a dense layer of
    `dense` units with LeakyReLU(0.2) and a dense layer of one unit with a
    sigmoid.  Convolutions are cross-correlations with zero padding 1 and
    biases; no batch normalisation (the generator has none either, and the
    windows here are normalised by the correction's scale).  The dense
    layer takes the last feature map flattened channel-first (c, y, x).
  * Inputs of D are fine-resolution windows of one channel (the paper's
    n_l x n_l windows, n_l = 24).
"""

from __future__ import annotations

import numpy as np

LEAK = 0.2
ADV_WEIGHT = 1e-3
STRIDES = (1, 2, 1, 2, 1, 2, 1, 2)


def leaky_relu(x: np.ndarray) -> np.ndarray:
    return np.where(x >= 0.0, x, LEAK * x)


def sigmoid(x: np.ndarray) -> np.ndarray:
    return 1.0 / (1.0 + np.exp(-x))


def conv2d(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int) -> np.ndarray:
    """Cross-correlation of x (C_in, H, W) with w (C_out, C_in, 3, 3), zero
    padding 1, the given stride, plus bias b (C_out); loops over the output
    pixels and the nine taps, products summed over the input channels."""
    cin, H, W = x.shape
    cout = w.shape[0]
    xp = np.zeros((cin, H + 2, W + 2))
    xp[:, 1:H + 1, 1:W + 1] = x
    Ho = (H + 2 - 3) // stride + 1
    Wo = (W + 2 - 3) // stride + 1
    out = np.empty((cout, Ho, Wo))
    for oy in range(Ho):
        for ox in range(Wo):
            acc = b.astype(np.float64).copy()
            for ky in range(3):
                for kx in range(3):
                    v = xp[:, oy * stride + ky, ox * stride + kx]
                    acc = acc + w[:, :, ky, kx] @ v
            out[:, oy, ox] = acc
    return out


def param_shapes(widths=(64, 64, 128, 128, 256, 256, 512, 512), window: int = 24,
                 dense: int = 1024):
    """Shapes of the discriminator's parameters, in order: (w, b) per conv,
    then (w, b) of the two dense layers."""
    shapes = []
    cin, side = 1, window
    for cout, s in zip(widths, STRIDES):
        shapes += [(cout, cin, 3, 3), (cout,)]
        cin = cout
        side = (side + 2 - 3) // s + 1
    shapes += [(dense, cin * side * side), (dense,), (1, dense), (1,)]
    return shapes


def discriminator(params: list[np.ndarray], x: np.ndarray) -> np.ndarray:
    """D(x) for windows x (B, 1, n, n): probabilities (B,) that each window
    is a real high-resolution sample."""
    nconv = len(STRIDES)
    out = []
    for sample in np.asarray(x, dtype=np.float64):
        h = sample
        for k in range(nconv):
            h = leaky_relu(conv2d(h, params[2 * k], params[2 * k + 1], STRIDES[k]))
        v = h.reshape(-1)
        w1, b1, w2, b2 = params[2 * nconv:2 * nconv + 4]
        v = leaky_relu(w1 @ v + b1)
        out.append(sigmoid(w2 @ v + b2)[0])
    return np.array(out)


def bce(d: np.ndarray, label: float) -> float:
    """Mean binary cross-entropy of probabilities d against one label."""
    d = np.asarray(d, dtype=np.float64)
    return float(np.mean(-(label * np.log(d) + (1.0 - label) * np.log(1.0 - d))))


def dis_loss(d_real: np.ndarray, d_fake: np.ndarray) -> float:
    """l_Dis: real windows labelled 1, generated ones 0."""
    return bce(d_real, 1.0) + bce(d_fake, 0.0)


def mse_loss(hr: np.ndarray, sr: np.ndarray) -> float:
    """l^SR_MSE: the mean over the fine pixels (and the batch) of the squared
    difference between the high-resolution target and the generator's
    output."""
    d = np.asarray(hr, dtype=np.float64) - np.asarray(sr, dtype=np.float64)
    return float(np.mean(d * d))


def gen_loss(d_fake: np.ndarray) -> float:
    """l^SR_Gen: the sum over the samples of -log D(G(I^LR))."""
    return float(np.sum(-np.log(np.asarray(d_fake, dtype=np.float64))))


def sr_loss(hr: np.ndarray, sr: np.ndarray, d_fake: np.ndarray) -> float:
    """l^SR = l^SR_MSE + 1e-3 l^SR_Gen."""
    return mse_loss(hr, sr) + ADV_WEIGHT * gen_loss(d_fake)
