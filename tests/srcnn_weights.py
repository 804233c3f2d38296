"""Weight sets for the SR-CNN tests: seeded random (He-scaled) weights, and
hand-set weights under which the network is an exactly known linear
interpolation (dyadic values, so every rounding step is exact)."""

import numpy as np

from oracle import srcnn


def random_blob(seed, scale=1.0):
    """Flat float32 blob in the library's weight order."""
    rng = np.random.default_rng(seed)
    out = []
    for s in srcnn.WEIGHT_SHAPES:
        fan_in = s[1] * 9
        out.append(rng.standard_normal(s).astype(np.float32) * np.float32(scale * np.sqrt(2.0 / fan_in)))
    return np.concatenate([w.reshape(-1) for w in out])


def random_layers(seed, scale=1.0):
    return srcnn.unpack_weights(random_blob(seed, scale))


KERNELS = {  # coarse 3x3 stencil per sub-pixel (a, b) of the fine output
    (0, 0): {(1, 1): 1.0},
    (0, 1): {(1, 1): 0.75, (1, 2): 0.25},
    (1, 0): {(1, 1): 0.5, (2, 1): 0.5},
    (1, 1): {(0, 0): 0.125, (1, 1): 0.375, (2, 2): 0.5},
}


def linear_blob():
    """Weights under which the network computes the linear interpolation
    KERNELS exactly: channels 0/1 carry relu(x) and relu(-x); blocks 0-3
    halve them (h + (-1/2) relu(h)), blocks 4-7 are identities only through
    their inner ReLU (h + 7 relu(-h) with h >= 0); channel 2 of the shuffled
    output is -relu-interp(relu(x)), which the ReLU after the shuffle must
    zero; the final conv recombines with weights +16, -16, +1."""
    L = [np.zeros(s, np.float32) for s in srcnn.WEIGHT_SHAPES]
    L[0][0, 0, 1, 1] = 1.0
    L[0][1, 0, 1, 1] = -1.0
    for b in range(srcnn.BLOCKS):
        c1, c2 = L[1 + 2 * b], L[2 + 2 * b]
        for c in (0, 1):
            if b < 4:
                c1[c, c, 1, 1] = 1.0
                c2[c, c, 1, 1] = -0.5
            else:
                c1[c, c, 1, 1] = -1.0
                c2[c, c, 1, 1] = 7.0
    up = L[-2]
    for (a, b), taps in KERNELS.items():
        for (ky, kx), v in taps.items():
            up[0 * 4 + 2 * a + b, 0, ky, kx] = v
            up[1 * 4 + 2 * a + b, 1, ky, kx] = v
            up[2 * 4 + 2 * a + b, 0, ky, kx] = -v
    L[-1][0, 0, 1, 1] = 16.0
    L[-1][0, 1, 1, 1] = -16.0
    L[-1][0, 2, 1, 1] = 1.0
    return np.concatenate([w.reshape(-1) for w in L])


def linear_layers():
    return srcnn.unpack_weights(linear_blob())


def linear_interp(e):
    n = e.shape[0]
    out = np.zeros((2 * n, 2 * n))
    for i in range(n):
        for j in range(n):
            for (a, b), taps in KERNELS.items():
                out[2 * i + a, 2 * j + b] = sum(v * e[(i + ky - 1) % n, (j + kx - 1) % n]
                                                for (ky, kx), v in taps.items())
    return out
