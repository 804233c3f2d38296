"""Offline training of the SR-CNN prolongation weights (Section 3.2 of the
paper: supervised super-resolution with the MSE loss, here without the
adversarial term).

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

        def blob(self) -> np.ndarray:
            ws = [self.stem.weight]
            for c1, c2 in zip(self.c1, self.c2):
                ws += [c1.weight, c2.weight]
            ws += [self.up.weight, self.fin.weight]
            return np.concatenate([w.detach().float().cpu().numpy().reshape(-1) for w in ws])

    return Net()


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
    opt = torch.optim.Adam(net.parameters(), lr=args.lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, args.steps)
    rng = np.random.default_rng(args.seed)
    sizes = sorted(groups)
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
    log(f"validation loss of the network: {v:.4e} (spline {base:.4e})")
    blob = net.blob().astype(np.float32)
    np.save(args.out, blob)
    log(f"wrote {blob.size} weights to {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
