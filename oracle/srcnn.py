"""Plain CPU reference for the super-resolution CNN prolongation.

TEST INFRASTRUCTURE ONLY (see the package docstring): only the test suite,
the smoke check and the benchmark's CPU baseline leg may use it.

What it computes (Section 3.1 and the SR-Prolongation algorithm of the
appendix; generator of Fig. 2b after Ledig et al.): a coarse correction e_c
on the periodic N x N unique nodes is mapped to a fine correction on the
2N x 2N unique nodes by a fully convolutional network, and the V-cycle adds
it in place of the spline interpolant at the finest prolongations.

Readings taken where the paper leaves the network open (each listed in the
design notes):
  * stem: 3x3 conv 1 -> 64, ReLU; 8 residual blocks x + conv(relu(conv(x)))
    with 3x3 convs 64 -> 64; 3x3 conv 64 -> 256 followed by a x2 pixel
    shuffle to 64 channels at twice the resolution and a ReLU; 3x3 conv
    64 -> 1.  No biases, no batch norm, no global skip.  All convolutions
    are cross-correlations with circular padding (periodic domain).
  * scaling: input e_c / s, output times s, with s = max |e_c| (s = 0 gives
    a zero output), in place of the paper's fixed-range symmetric-log
    normalisation, which does not suit corrections that shrink every cycle.
  * arithmetic: weights and every conv's input activations are rounded to
    bfloat16 (round to nearest even); each conv output is the exact sum of
    its bf16 products rounded once to FP32 (here: summed in FP64, then
    rounded), the residual add and ReLU act on FP32 values and the result
    is rounded to bf16 where it is stored.

Weights travel as one flat float32 blob in PyTorch (out, in, ky, kx) order:
stem, then for each block conv1 and conv2, then the 64 -> 256 conv, then
the final conv (WEIGHT_SHAPES).  The conv itself is torch.nn.functional.
conv2d in float64 on the CPU (a library primitive), pinned in the tests
against a brute-force loop and against the closed form of hand-set weights.
"""

from __future__ import annotations

import numpy as np

BLOCKS = 8
WIDTH = 64
WEIGHT_SHAPES = ([(WIDTH, 1, 3, 3)] + [(WIDTH, WIDTH, 3, 3)] * (2 * BLOCKS)
                 + [(4 * WIDTH, WIDTH, 3, 3), (1, WIDTH, 3, 3)])
WEIGHT_COUNT = int(sum(np.prod(s) for s in WEIGHT_SHAPES))
# Receptive-field margin of one output in coarse pixels: 18 coarse convs
# plus one fine conv (half a coarse pixel, rounded up).
MARGIN = 2 + 2 * BLOCKS + 1


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32.  From the definition: keep the top 16 bits of the binary32
    pattern after adding half an ulp of bf16 plus the tie-breaking bit."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = (bits + 0x7FFF + lsb) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).reshape(a.shape)


def unpack_weights(blob: np.ndarray) -> list[np.ndarray]:
    """Split the flat float32 blob into per-layer arrays, rounded to bf16."""
    blob = np.asarray(blob, dtype=np.float32).reshape(-1)
    if blob.size != WEIGHT_COUNT:
        raise ValueError(f"expected {WEIGHT_COUNT} weights, got {blob.size}")
    out, k = [], 0
    for s in WEIGHT_SHAPES:
        m = int(np.prod(s))
        out.append(bf16_round(blob[k:k + m]).reshape(s))
        k += m
    return out


def conv3x3(x: np.ndarray, w: np.ndarray, circular: bool = True) -> np.ndarray:
    """out[o, y, x] = sum over i, ky, kx of w[o, i, ky, kx] * x[i, y+ky-1, x+kx-1].

    x: (C_in, H, W), w: (C_out, C_in, 3, 3).  circular pads periodically
    (same size out); otherwise 'valid' (out is 2 smaller per axis).  Summed
    in FP64, returned rounded to FP32."""
    import torch
    import torch.nn.functional as F

    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))[None]
    if circular:
        t = F.pad(t, (1, 1, 1, 1), mode="circular")
    k = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float64))
    return F.conv2d(t, k)[0].numpy().astype(np.float32)


def pixel_shuffle(y: np.ndarray) -> np.ndarray:
    """(4C, H, W) -> (C, 2H, 2W): z[c, 2i + a, 2j + b] = y[4c + 2a + b, i, j]."""
    c4, h, w = y.shape
    c = c4 // 4
    z = np.empty((c, 2 * h, 2 * w), dtype=y.dtype)
    for a in range(2):
        for b in range(2):
            z[:, a::2, b::2] = y[np.arange(c) * 4 + 2 * a + b]
    return z


def network(x: np.ndarray, layers: list[np.ndarray], circular: bool = True) -> np.ndarray:
    """The generator on a scaled input x (H, W), already bf16-valued.
    Returns the FP32 output (2H, 2W) (circular) or its valid part."""
    stem, body, up, fin = layers[0], layers[1:1 + 2 * BLOCKS], layers[-2], layers[-1]
    h = bf16_round(np.maximum(conv3x3(x[None], stem, circular), 0))
    for b in range(BLOCKS):
        c = 0 if circular else 1
        t = bf16_round(np.maximum(conv3x3(h, body[2 * b], circular), 0))
        y = conv3x3(t, body[2 * b + 1], circular)
        skip = h if circular else h[:, 2 * c:h.shape[1] - 2 * c, 2 * c:h.shape[2] - 2 * c]
        h = bf16_round(skip + y)
    z = bf16_round(np.maximum(pixel_shuffle(conv3x3(h, up, circular)), 0))
    return conv3x3(z, fin, circular)[0]


def scale_of(ec_unique: np.ndarray) -> np.float32:
    """s = max |e_c| over the unique nodes, in FP32."""
    return np.float32(np.max(np.abs(ec_unique.astype(np.float32)))) if ec_unique.size else np.float32(0)


def forward(ec_unique: np.ndarray, layers: list[np.ndarray]) -> np.ndarray:
    """Fine correction (2N, 2N) FP32 from a coarse correction (N, N):
    s * network(bf16(e_c / s))."""
    s = scale_of(ec_unique)
    n = ec_unique.shape[0]
    if s == 0:
        return np.zeros((2 * n, 2 * n), dtype=np.float32)
    x = bf16_round(ec_unique.astype(np.float32) / s)
    return (s * network(x, layers)).astype(np.float32)


def forward_window(ec_unique: np.ndarray, layers: list[np.ndarray], y0: int, x0: int,
                   h: int, w: int) -> np.ndarray:
    """Rows 2*y0 .. 2*(y0+h)-1, columns 2*x0 .. 2*(x0+w)-1 of forward(),
    computed from a periodic crop of the input with valid convolutions (for
    spot checks on grids too large for the whole forward pass)."""
    s = scale_of(ec_unique)
    if s == 0:
        return np.zeros((2 * h, 2 * w), dtype=np.float32)
    n = ec_unique.shape[0]
    m = MARGIN
    rows = np.arange(y0 - m, y0 + h + m) % n
    cols = np.arange(x0 - m, x0 + w + m) % n
    x = bf16_round(ec_unique[np.ix_(rows, cols)].astype(np.float32) / s)
    out = network(x, layers, circular=False)
    # Valid output covers fine rows 2*(y0 - m + 18) + 1 onwards: 18 coarse
    # convs trim 18 coarse pixels (36 fine) per side, the fine conv one more.
    off = 2 * (m - (2 + 2 * BLOCKS)) - 1
    return (s * out[off:off + 2 * h, off:off + 2 * w]).astype(np.float32)


def to_unique(a: np.ndarray) -> np.ndarray:
    """Unique nodes of a periodic grid with seam: (n, n) -> (n-1, n-1)."""
    return a[:-1, :-1]


def with_seam(a: np.ndarray) -> np.ndarray:
    """(N, N) unique nodes -> (N+1, N+1) grid with the seam duplicated."""
    return np.pad(a, ((0, 1), (0, 1)), mode="wrap")


def prolong(ec: np.ndarray, layers: list[np.ndarray]) -> np.ndarray:
    """SR prolongation of a periodic coarse grid (nc, nc) to (2nc-1, 2nc-1),
    FP32 values in the grid's dtype, seam written."""
    return with_seam(forward(to_unique(ec), layers)).astype(ec.dtype)


def vcycle(u: np.ndarray, f: np.ndarray, layers: list[np.ndarray], cnn_levels: int,
           nu1: int = 2, nu2: int = 2) -> np.ndarray:
    """One periodic V(nu1, nu2) cycle in the dtype of u whose `cnn_levels`
    finest prolongations use the network (the appendix's V-CYCLE with the
    SR prolongation selected); coarser levels are the plain cycle."""
    import oracle

    bc = oracle.PERIODIC
    if cnn_levels <= 0:
        return oracle.vcycle(u, f, bc, nu1, nu2)
    u = np.array(u, copy=True)
    for _ in range(nu1):
        u = oracle.relax(oracle.relax(u, f, bc, oracle.RED), f, bc, oracle.BLACK)
    fc = oracle.restrict(oracle.residual(u, f, bc), bc)
    ec = vcycle(np.zeros_like(fc), fc, layers, cnn_levels - 1, nu1, nu2)
    u = u + prolong(ec, layers)
    for _ in range(nu2):
        u = oracle.relax(oracle.relax(u, f, bc, oracle.RED), f, bc, oracle.BLACK)
    return u


def refine_step(u: np.ndarray, f: np.ndarray, layers: list[np.ndarray], cnn_levels: int,
                nu1: int = 2, nu2: int = 2) -> np.ndarray:
    """Mixed path: r = f - A u in FP64, e = FP32 cycle (with the network on
    the finest prolongations) from e = 0 on fl32(r), u + e in FP64."""
    import oracle

    r = oracle.residual(u.astype(np.float64), f.astype(np.float64), oracle.PERIODIC)
    e = vcycle(np.zeros(r.shape, np.float32), r.astype(np.float32), layers, cnn_levels, nu1, nu2)
    return u + e.astype(np.float64)


def prolongation_choice(i: int, n_gan: float, switched: bool) -> bool:
    """Operator of iteration i = 1, 2, ... of the hybrid schedule (appendix
    V-CYCLE with the N_GAN and S_thres parameters of Table 1): True for the
    network, False for the spline.

    N_GAN >= 1 makes the network the first operator and the spline the
    second, N_GAN < 1 the reverse, with N = N_GAN or 1 / N_GAN.  Reading:
    N_GAN counts network prolongations per spline prolongation, so that
    N_GAN = 1 alternates (Section 3), i.e. the first operator runs N times
    and then the second once: the second is taken when i is a multiple of
    N + 1.  (The appendix's modulus is N, which for N_GAN = 1 would never
    alternate.)  Once the switch is set the second operator is used."""
    if n_gan >= 1.0:
        N, first = int(round(n_gan)), True
    else:
        N, first = int(round(1.0 / n_gan)), False
    if i % (N + 1) != 0 and not switched:
        return first
    return not first


def solve_schedule(f: np.ndarray, layers: list[np.ndarray], cnn_levels: int, rtol: float,
                   max_cycles: int, n_gan: float, s_thres: float, mixed: bool = False,
                   nu1: int = 2, nu2: int = 2):
    """Solve a periodic problem from u = 0 with the hybrid schedule: each
    iteration prolongs with prolongation_choice()'s operator (the network on
    the `cnn_levels` finest prolongations, else the spline everywhere); the
    switch of iteration i + 1 is set when iteration i changed the iterate by
    at most s_thres, ||p_i - p_(i-1)||_2 over the unique nodes (Section 4;
    s_thres = 0 never switches).  Stops once ||f - A u|| / ||f|| <= rtol or
    after max_cycles iterations.  mixed: each iteration is refine_step()
    (FP64 residual, FP32 cycle), else vcycle() in FP64.

    Returns (u, ops, diffs, relres): ops[k] True where iteration k + 1 used
    the network, diffs[k] its ||p_(k+1) - p_k||_2."""
    import oracle

    u = np.zeros_like(f)
    rel = oracle.relres(u, f, oracle.PERIODIC)
    ops: list[bool] = []
    diffs: list[float] = []
    switched = False
    while rel > rtol and len(ops) < max_cycles:
        net = prolongation_choice(len(ops) + 1, n_gan, switched)
        lv = cnn_levels if net else 0
        new = (refine_step(u, f, layers, lv, nu1, nu2) if mixed
               else vcycle(u, f, layers, lv, nu1, nu2))
        d = float(np.linalg.norm(to_unique(new - u)))
        switched = s_thres > 0.0 and d <= s_thres
        ops.append(net)
        diffs.append(d)
        u = new
        rel = oracle.relres(u, f, oracle.PERIODIC)
    return u, ops, diffs, rel
