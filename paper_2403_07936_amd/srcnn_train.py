"""Offline training of the SR-CNN prolongation weights (Section 3.2 of the
paper).  Two modes: supervised training with one content loss (below), and
with --adversarial the paper's GAN training (Section 2.3): a discriminator
after Ledig et al. trained with l_Dis (binary cross-entropy, real windows of
the target against generated ones) alternating with the generator trained
with l^SR = l_MSE + 1e-3 l_Gen, l_Gen = sum of -log D(G(I^LR)).

Training pairs come from the solver itself: for each seeded periodic
divergence-of-velocity source (workloads.rhs_divu_periodic), the iterate
after 0, 1 or 2 spline V-cycles is pre-smoothed on the finest level, and
  input  e_c = the coarse correction one V-cycle computes from the restricted
               residual (what the cycle would prolongate),
  target e*  = the exact fine error A^-1 r of the pre-smoothed iterate
               (periodic FFT solve, zero mean),
both divided by s = max |e_c|.  The same is recorded one level down (the
second-finest prolongation).  The loss is the paper's mean square, taken
of the residual that the prolongation error e* - net(e_c) leaves after the
cycle's post-smoothing (two red-black sweeps): a plain MSE on e* rewards
networks that fit the error in L2 while leaving high-frequency residue that
the residual norm, and so the cycle's convergence, punishes.  The forward
pass rounds weights and activations to bf16 as the library's kernels do.  The network (same layers as the library's
kernels: 3x3 circular convs without bias, 8 residual blocks, x2 pixel
shuffle) is trained in FP32 PyTorch and written as the flat float32 blob
that mg_setup takes (include/mg.h, MG_SRCNN_WEIGHT_COUNT).

Usage (on a GPU):  python -m paper_2403_07936_amd.srcnn_train --out W.npy
                   [--adversarial --init W0.npy --content mse|cycle]
"""

from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np


def log(msg: str) -> None:
    print(f"[srcnn_train] {msg}", flush=True)


def build_model(torch):
    """The generator with the library's arithmetic simulated in the forward
    pass: weights, the input and every stored activation rounded to bf16
    (straight-through gradients), FP32 elsewhere."""
    nn = torch.nn
    F = torch.nn.functional

    def q(t):
        return t + (t.to(torch.bfloat16).float() - t).detach()

    def conv(cin, cout):
        return nn.Conv2d(cin, cout, 3, padding=0, bias=False)

    def apply(c, x):
        return F.conv2d(F.pad(x, (1, 1, 1, 1), mode="circular"), q(c.weight))

    class Net(nn.Module):
        def __init__(self):
            super().__init__()
            self.stem = conv(1, 64)
            self.c1 = nn.ModuleList([conv(64, 64) for _ in range(8)])
            self.c2 = nn.ModuleList([conv(64, 64) for _ in range(8)])
            self.up = conv(64, 256)
            self.fin = conv(64, 1)

        def forward(self, x):
            h = q(torch.relu(apply(self.stem, q(x))))
            for c1, c2 in zip(self.c1, self.c2):
                t = q(torch.relu(apply(c1, h)))
                h = q(h + apply(c2, t))
            z = q(torch.relu(F.pixel_shuffle(apply(self.up, h), 2)))
            return apply(self.fin, z)

        def load_blob(self, blob) -> None:
            ws = [self.stem.weight]
            for c1, c2 in zip(self.c1, self.c2):
                ws += [c1.weight, c2.weight]
            ws += [self.up.weight, self.fin.weight]
            flat = np.asarray(blob, dtype=np.float32).reshape(-1)
            k = 0
            with torch.no_grad():
                for w in ws:
                    m = w.numel()
                    w.copy_(torch.from_numpy(flat[k:k + m].reshape(tuple(w.shape))))
                    k += m
            assert k == flat.size, "weight blob of the wrong size"

        def blob(self) -> np.ndarray:
            ws = [self.stem.weight]
            for c1, c2 in zip(self.c1, self.c2):
                ws += [c1.weight, c2.weight]
            ws += [self.up.weight, self.fin.weight]
            return np.concatenate([w.detach().float().cpu().numpy().reshape(-1) for w in ws])

    return Net()


# ---- adversarial training (Section 2.3: l_Dis and l^SR = l_MSE + 1e-3 l_Gen;
# Fig. 2b: the discriminator after Ledig et al.) -----------------------------

DISC_STRIDES = (1, 2, 1, 2, 1, 2, 1, 2)
DISC_WIDTHS = (64, 64, 128, 128, 256, 256, 512, 512)
DISC_LEAK = 0.2
ADV_WEIGHT = 1e-3


def build_discriminator(torch, widths=DISC_WIDTHS, window: int = 24, dense: int = 1024):
    """Ledig et al.'s discriminator on one-channel windows of side `window`:
    a 3x3 conv and LeakyReLU(0.2), seven 3x3 convs with strides 2,1,2,1,2,1,2
    (zero padding 1, biases), each with LeakyReLU(0.2), a dense layer of
    `dense` units with LeakyReLU(0.2), and a one-unit dense layer.  No batch
    normalisation.  `logits(x)` is the last layer's output, `forward(x)` its
    sigmoid (the probability that a window is a real sample)."""
    nn = torch.nn
    F = torch.nn.functional

    class Disc(nn.Module):
        def __init__(self):
            super().__init__()
            self.window = window
            convs, cin, side = [], 1, window
            for cout, st in zip(widths, DISC_STRIDES):
                convs.append(nn.Conv2d(cin, cout, 3, stride=st, padding=1, bias=True))
                cin = cout
                side = (side + 2 - 3) // st + 1
            self.convs = nn.ModuleList(convs)
            self.d1 = nn.Linear(cin * side * side, dense)
            self.d2 = nn.Linear(dense, 1)

        def logits(self, x):
            h = x
            for c in self.convs:
                h = F.leaky_relu(c(h), DISC_LEAK)
            h = F.leaky_relu(self.d1(h.flatten(1)), DISC_LEAK)
            return self.d2(h)[:, 0]

        def forward(self, x):
            return torch.sigmoid(self.logits(x))

    return Disc()


def set_discriminator_params(torch, disc, params) -> None:
    """Load parameters given in order (conv weight, bias per conv, then the
    two dense layers' weight and bias) as numpy arrays."""
    mods = list(disc.convs) + [disc.d1, disc.d2]
    with torch.no_grad():
        for k, m in enumerate(mods):
            m.weight.copy_(torch.from_numpy(np.asarray(params[2 * k])))
            m.bias.copy_(torch.from_numpy(np.asarray(params[2 * k + 1])))


def dis_loss(torch, d_real, d_fake):
    """l_Dis: mean binary cross-entropy of D's probabilities, real windows
    labelled 1 plus generated windows labelled 0."""
    return torch.mean(-torch.log(d_real)) + torch.mean(-torch.log(1.0 - d_fake))


def mse_loss(torch, hr, sr):
    """l^SR_MSE: mean over the fine pixels of (I^HR - G(I^LR))^2."""
    return torch.mean((hr - sr) ** 2)


def gen_loss(torch, d_fake):
    """l^SR_Gen: sum over the samples of -log D(G(I^LR))."""
    return torch.sum(-torch.log(d_fake))


def sr_loss(torch, hr, sr, d_fake):
    """l^SR = l^SR_MSE + 1e-3 l^SR_Gen."""
    return mse_loss(torch, hr, sr) + ADV_WEIGHT * gen_loss(torch, d_fake)


def crop_windows(torch, side: int, window: int, count: int, rng):
    """`count` window origins (y, x) inside a fine grid of the given side."""
    return [(int(rng.integers(0, side - window + 1)), int(rng.integers(0, side - window + 1)))
            for _ in range(count)]


def _windows(torch, a, crops, window):
    return torch.cat([a[:, :, y:y + window, x:x + window] for y, x in crops], 0)


def adversarial_step(torch, gen, disc, og, od, x, y, crops, content: str = "mse"):
    """One step of the paper's alternating training: (i) the generator,
    fixed, makes synthetic fine corrections; (ii) the discriminator is
    trained on real (target) and synthetic windows with l_Dis; (iii) with the
    discriminator fixed, the generator is trained with l^SR = content +
    1e-3 l_Gen, content the paper's l_MSE ("mse") or the post-smoothed
    residual loss of the MSE-only trainer ("cycle").  The cross-entropies are
    taken from D's logits (softplus form, the same values without log(0)).
    Returns (l_Dis, l^SR, and mean D(real) - mean D(fake) on the step's
    windows before and after the D step)."""
    F = torch.nn.functional
    window = disc.window
    with torch.no_grad():
        fake = gen(x)
    real_w, fake_w = _windows(torch, y, crops, window), _windows(torch, fake, crops, window)
    zr, zf = disc.logits(real_w), disc.logits(fake_w)
    gap0 = float(torch.mean(torch.sigmoid(zr)) - torch.mean(torch.sigmoid(zf)))
    ld = torch.mean(F.softplus(-zr)) + torch.mean(F.softplus(zf))
    od.zero_grad(set_to_none=True)
    ld.backward()
    od.step()
    with torch.no_grad():
        gap = float(torch.mean(disc(real_w)) - torch.mean(disc(fake_w)))
    sr = gen(x)
    zg = disc.logits(_windows(torch, sr, crops, window))
    base = mse_loss(torch, y, sr) if content == "mse" else cycle_loss(torch, y, sr)
    lg = base + ADV_WEIGHT * torch.sum(F.softplus(-zg))
    og.zero_grad(set_to_none=True)
    lg.backward()
    og.step()
    return float(ld.detach()), float(lg.detach()), gap0, gap


def exact_error(torch, r: "torch.Tensor") -> "torch.Tensor":
    """A^-1 r on the unique nodes of a periodic grid (zero mean), A the
    5-point -Laplacian with h = 1/N: Fourier symbol (4/h^2)(sin^2(pi kx/N) +
    sin^2(pi ky/N))."""
    N = r.shape[-1]
    k = torch.fft.fftfreq(N, d=1.0 / N, device=r.device, dtype=torch.float64)
    s2 = torch.sin(torch.pi * k / N) ** 2
    lam = 4.0 * N * N * (s2[:, None] + s2[None, :])
    lam[0, 0] = 1.0
    uh = torch.fft.fft2(r) / lam
    uh[0, 0] = 0.0
    return torch.fft.ifft2(uh).real


def post_smooth(torch, d, sweeps: int = 2):
    """Error propagation of `sweeps` red-black Gauss-Seidel sweeps (red =
    (i + j) even first) with zero right-hand side on a periodic grid, applied
    to a batch of errors d (B, 1, M, M): what the cycle's post-smoothing
    leaves of a prolongation error."""
    M = d.shape[-1]
    i = torch.arange(M, device=d.device)
    red = ((i[:, None] + i[None, :]) % 2 == 0).to(d.dtype)
    for _ in range(sweeps):
        for mask in (red, 1 - red):
            nb = (torch.roll(d, 1, -1) + torch.roll(d, -1, -1) + torch.roll(d, 1, -2)
                  + torch.roll(d, -1, -2)) * 0.25
            d = mask * nb + (1 - mask) * d
    return d


def cycle_loss(torch, target, pred):
    """Mean square of the residual A d of what post-smoothing leaves of the
    prolongation error (A: the 5-point stencil without the 1/h^2 factor)."""
    d = post_smooth(torch, target - pred)
    r = 4 * d - (torch.roll(d, 1, -1) + torch.roll(d, -1, -1) + torch.roll(d, 1, -2)
                 + torch.roll(d, -1, -2))
    return torch.mean(r * r)


def make_pairs(torch, n: int, seeds, dev):
    """List of (e_c, e*) pairs, both scaled by max|e_c|, as float32 tensors
    (coarse N x N, fine 2N x 2N), for the two finest prolongations."""
    import workloads
    from . import binding as B

    stream = torch.cuda.current_stream().cuda_stream
    o = B.mg_options_default()
    sizes = [n, (n - 1) // 2 + 1, (n - 1) // 4 + 1]
    ctxs = [B.mg_setup([(m, 1, 0)], o, stream) for m in sizes]
    pairs = []
    try:
        for q, s in enumerate(seeds):
            if q % 250 == 0:
                log(f"pairs from seed {s} ({q} of {len(seeds)})")
            f = torch.from_numpy(workloads.rhs_divu_periodic(n, int(s))).to(dev)
            u = torch.zeros_like(f)
            k = int(s) % 3
            if k:
                B.mg_vcycle(ctxs[0], [u.data_ptr()], [f.data_ptr()], k)
            fl = f
            for lvl in range(2):
                ctx, cc = ctxs[lvl], ctxs[lvl + 1]
                if lvl == 1:
                    u = torch.zeros_like(fl)
                B.mg_relax(ctx, 0, 0, u.data_ptr(), fl.data_ptr(), 0, 4, 0)
                r = torch.empty_like(u)
                B.mg_residual(ctx, 0, 0, u.data_ptr(), fl.data_ptr(), r.data_ptr(), 0)
                mc = sizes[lvl + 1]
                fc = torch.empty((mc, mc), dtype=torch.float64, device=dev)
                B.mg_restrict(ctx, 0, 0, r.data_ptr(), fc.data_ptr(), 0)
                ec = torch.zeros_like(fc)
                B.mg_vcycle(cc, [ec.data_ptr()], [fc.data_ptr()], 1)
                torch.cuda.synchronize()
                target = exact_error(torch, r[:-1, :-1])
                inp = ec[:-1, :-1]
                sc = inp.abs().max()
                if sc > 0:
                    pairs.append(((inp / sc).float(), (target / sc).float()))
                fl = fc
    finally:
        for c in ctxs:
            B.mg_destroy(c)
    return pairs


def spline_loss(torch, pairs, n: int, dev):
    """Training loss of the spline interpolant (the baseline the network has
    to beat)."""
    from . import binding as B

    stream = torch.cuda.current_stream().cuda_stream
    ctx = B.mg_setup([(n, 1, 0)], B.mg_options_default(), stream)
    tot, cnt = 0.0, 0
    try:
        for x, y in pairs:
            N = x.shape[-1]
            lvl = {(n - 1) // 2: 1, (n - 1) // 4: 2}[N]
            c = torch.nn.functional.pad(x.double()[None, None], (0, 1, 0, 1), mode="circular")[0, 0]
            c = c.contiguous()
            fine = torch.empty((2 * N + 1, 2 * N + 1), dtype=torch.float64, device=dev)
            B.mg_prolong(ctx, 0, lvl, 0, c.data_ptr(), fine.data_ptr(), 0)
            torch.cuda.synchronize()
            tot += float(cycle_loss(torch, y[None, None], fine[:-1, :-1].float()[None, None]))
            cnt += 1
    finally:
        B.mg_destroy(ctx)
    return tot / max(cnt, 1)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--n", type=int, default=1025)
    ap.add_argument("--train-seeds", type=int, nargs=2, default=(10000, 12000))
    ap.add_argument("--val-seeds", type=int, nargs=2, default=(0, 10))
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--adversarial", action="store_true",
                    help="train with the paper's GAN losses (l_Dis; l^SR = content + 1e-3 l_Gen)")
    ap.add_argument("--content", choices=["mse", "cycle"], default="mse",
                    help="content term of l^SR: the paper's l_MSE, or the post-smoothed residual")
    ap.add_argument("--init", default=None, help="generator weights to start from (.npy blob)")
    ap.add_argument("--window", type=int, default=24, help="discriminator window side (n_l)")
    ap.add_argument("--crops", type=int, default=8, help="windows per sample and step")
    ap.add_argument("--d-lr", type=float, default=1e-4)
    args = ap.parse_args(argv)

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch

    if not torch.cuda.is_available():
        log("needs a GPU")
        return 1
    dev = torch.device("cuda:0")
    torch.manual_seed(args.seed)
    t0 = time.time()
    train = make_pairs(torch, args.n, range(*args.train_seeds), dev)
    val = make_pairs(torch, args.n, range(*args.val_seeds), dev)
    log(f"{len(train)} training pairs, {len(val)} validation pairs ({time.time() - t0:.1f} s)")
    base = spline_loss(torch, val, args.n, dev)
    log(f"validation loss of the spline interpolant: {base:.4e}")

    by_size = {}
    for x, y in train:
        by_size.setdefault(x.shape[-1], []).append((x, y))
    groups = {N: (torch.stack([p[0] for p in v])[:, None], torch.stack([p[1] for p in v])[:, None])
              for N, v in by_size.items()}
    net = build_model(torch).to(dev)
    if args.init:
        net.load_blob(np.load(args.init))
        log(f"generator initialised from {args.init}")
    opt = torch.optim.Adam(net.parameters(), lr=args.lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, args.steps)
    rng = np.random.default_rng(args.seed)
    sizes = sorted(groups)
    if args.adversarial:
        disc = build_discriminator(torch, DISC_WIDTHS, args.window).to(dev)
        od = torch.optim.Adam(disc.parameters(), lr=args.d_lr)
        for step in range(args.steps):
            N = sizes[step % len(sizes)]
            X, Y = groups[N]
            idx = torch.from_numpy(rng.integers(0, X.shape[0], args.batch)).to(dev)
            crops = crop_windows(torch, 2 * N, args.window, args.crops, rng)
            ld, lg, g0, g1 = adversarial_step(torch, net, disc, opt, od, X[idx], Y[idx], crops,
                                              args.content)
            sched.step()
            if step % 100 == 0 or step == args.steps - 1:
                log(f"step {step}: l_Dis {ld:.4e}, l^SR {lg:.4e}, D(real) - D(fake) {g0:+.3f} -> "
                    f"{g1:+.3f} ({time.time() - t0:.1f} s)")
        args.steps = 0
    for step in range(args.steps):
        N = sizes[step % len(sizes)]
        X, Y = groups[N]
        idx = torch.from_numpy(rng.integers(0, X.shape[0], args.batch)).to(dev)
        loss = cycle_loss(torch, Y[idx], net(X[idx]))
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        sched.step()
        if step % 100 == 0 or step == args.steps - 1:
            log(f"step {step}: loss {float(loss.detach()):.4e} ({time.time() - t0:.1f} s)")
    with torch.no_grad():
        v = float(np.mean([float(cycle_loss(torch, y[None, None], net(x[None, None]))) for x, y in val]))
        m = float(np.mean([float(mse_loss(torch, y[None, None], net(x[None, None]))) for x, y in val]))
    log(f"validation loss of the network: {v:.4e} (spline {base:.4e}); its l_MSE {m:.4e}")
    blob = net.blob().astype(np.float32)
    np.save(args.out, blob)
    log(f"wrote {blob.size} weights to {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
