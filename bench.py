"""Benchmark: grid-points/s per V-cycle and time to 1e-10 relative residual.

Default workload: 2-D Poisson on a 4097 x 4097 zero-Dirichlet grid (11
levels), sine-basis divergence-of-velocity source with a k^(-5/3) spectrum,
V(2,2) cycles with red-black Gauss-Seidel, full weighting, cubic-spline
prolongation and a direct 5 x 5 solve.  Both the plain FP64 path and the
mixed path (FP64 refinement around FP32 cycles) are timed; the faster one is
the headline.  A step is one cycle of the headline path (one V-cycle, or one
refinement step with its FP32 V-cycle) on the resident grid.

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic(kind_name: str, precision: str, bc: int):
    """HBM bytes per launch of the level-0 kernel from the committed counter
    summary (profiles/hbm_traffic.json: FETCH_SIZE and WRITE_SIZE scaled by a
    known-size copy), or None when that kernel's source has changed since the
    counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    names = {"down": "k_down_s", "up": "k_up_s"}
    if kind_name not in names or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if "sources" not in rec:
        return None
    hh = hashlib.sha256()
    for src in rec["sources"]:
        hh.update(open(os.path.join(ROOT, src), "rb").read())
    if hh.hexdigest() != rec["sources_sha256"]:
        return None
    t = "float" if precision == "mixed" else "double"
    if precision == "mixed":
        # The mixed level-0 passes: the down pass that makes the FP64
        # residual itself (and stores no pre-smoothed iterate), the up pass
        # that re-makes that iterate and adds into the FP64 one.
        head = {"down": f"k_down_res_s<{bc}, false, false>", "up": f"k_up_pre_s<{bc}>"}[kind_name]
        ents = [v for k, v in rec["per_launch"].items() if k == head]
    else:
        # Template variants of the kernel (input/accumulation flags); the
        # level-0 launch is the one with the most traffic.
        head = f"{names[kind_name]}<{t}, {bc}"
        ents = [v for k, v in rec["per_launch"].items()
                if k == head + ">" or k.startswith(head + ",")]
    return round(max(e["bytes"] for e in ents), 0) if ents else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dirichlet4097",
                    choices=["dirichlet4097", "periodic1025", "dirichlet65", "batch256",
                             "periodic1025_srcnn", "periodic4097_projection", "twolevel192"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-extra", action="store_true",
                    help="default workload only: skip the periodic1025, batch256 and "
                         "periodic1025_srcnn sub-objects")
    ap.add_argument("--weights", default=None,
                    help="periodic1025_srcnn: SR-CNN weight blob (.npy) instead of the committed "
                         "supervised one")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file (read, and appended with new choices), so that "
                         "several runs (e.g. one per profiler counter) use the same launch shapes")
    return ap.parse_args()


BF16_PEAK_TFLOPS = 2500.0
WEIGHTS = os.path.join(ROOT, "paper_2403_07936_amd", "weights", "srcnn_divu_periodic.npy")


def measure_srcnn(args, dev, W, steps, warmup):
    """SR-CNN cycles on the 1025 x 1025 periodic source (FP64 cycle, the
    network on the two finest prolongations) next to the spline cycle and the
    hybrid schedule at N_GAN = 1: seconds per cycle and the best of three
    solves to 1e-8 each; then the level-0 kernels of the network cycle timed
    by HIP events.  Returns ((n, bc, f), per-mode results, roofline,
    per-kernel times); the solvers are closed."""
    import torch

    import workloads
    from paper_2403_07936_amd import binding as B
    from paper_2403_07936_amd.solver import Solver

    n, bc, f = workloads.workload("periodic1025", args.seed)
    ft = torch.from_numpy(f).to(dev)
    ut = torch.zeros_like(ft)
    res = {}
    for mode in ("srcnn", "spline", "hybrid"):
        kw = dict(cnn_weights=W, cnn_levels=2) if mode != "spline" else {}
        if mode == "hybrid":
            kw.update(n_gan=1.0)
        s = Solver([(n, bc)], precision="fp64", use_graph=True, **kw)
        ut.zero_()
        s.vcycle([ut], [ft], warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.vcycle([ut], [ft], steps)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        best = None
        for _ in range(3):
            ut.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, cyc, rel = s.solve([ut], [ft], rtol=1e-8, max_cycles=60)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best[0]:
                best = (dt, st, cyc[0], rel[0])
        ops = "".join("N" if o == B.MG_PROLONG_SRCNN else "s" for o in s.history()[0])
        res[mode] = {"solver": s, "sec": sec, "ttt": best, "ops": ops}
        log(f"{mode}: {sec * 1e3:.3f} ms/cycle; to 1e-8: {best[0] * 1e3:.2f} ms, {best[2]} cycles, "
            f"relres {best[3]:.2e}")
    hs = res["srcnn"]["solver"]
    B.mg_timing_enable(hs.ctx, True)
    ut.zero_()
    torch.cuda.synchronize()
    for _ in range(steps):
        hs.vcycle([ut], [ft], 1)
    torch.cuda.synchronize()
    kern = {}
    for kind in range(B.MG_K_COUNT):
        for lvl in range(2):
            cnt, ms, by = B.mg_timing_read(hs.ctx, kind, lvl)
            if cnt:
                kern[f"{B.mg_kernel_name(kind)}@{lvl}"] = (cnt, ms, by)
    B.mg_timing_enable(hs.ctx, False)
    cnt, ms, flops = kern["cnn_conv@0"]
    achieved = flops / (ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "kernel": "cnn_conv (level 0, 512^2 coarse, 64->64 and 64->256)",
                "achieved": round(achieved, 1), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / BF16_PEAK_TFLOPS, 4), "traffic": None,
                "avg_launch_us": round(ms / cnt * 1e3, 2), "flops_per_launch": flops / cnt}
    per_kernel = {k: {"launches": c, "avg_us": round(m / c * 1e3, 2)} for k, (c, m, b) in kern.items()}
    for v in res.values():
        v["solver"].close()
        del v["solver"]
    return (n, bc, f), res, roofline, per_kernel


def srcnn_summary(res, unknowns):
    """Compact record of measure_srcnn's modes."""
    out = {}
    for mode, r in res.items():
        out[mode] = {"ms_per_cycle": round(r["sec"] * 1e3, 4),
                     "grid_points_per_s": round(unknowns / r["sec"], 1),
                     "time_to_1e-8_s": round(r["ttt"][0], 6), "cycles_to_1e-8": r["ttt"][2],
                     "final_relres": r["ttt"][3], "status": r["ttt"][1]}
    out["hybrid"]["prolongations"] = res["hybrid"]["ops"]
    return out


def bench_srcnn(args) -> int:
    """1025 x 1025 periodic div-u source, V(2,2) cycles whose two finest
    prolongations use the SR-CNN (bf16 matrix cores), FP64 cycle.  A step is
    one such cycle.  Also reported: time to 1e-8 with the network-then-spline
    schedule, with the hybrid schedule at N_GAN = 1 (network and spline
    cycles alternating), and the spline cycle for comparison."""
    import numpy as np
    import torch

    import workloads
    from paper_2403_07936_amd import binding as B

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    B.lib()
    wpath = args.weights or WEIGHTS
    W = np.load(wpath)
    (n, bc, f), res, roofline, per_kernel = measure_srcnn(args, dev, W, args.steps, args.warmup)
    unknowns = workloads.grid_unknowns(n, bc)
    cpu = None
    if not args.no_cpu:
        from oracle import srcnn

        layers = srcnn.unpack_weights(W)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        u = np.zeros_like(f)
        count, t0 = 0, time.perf_counter()
        while True:
            u = srcnn.vcycle(u, f, layers, 2)
            count += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds or count >= 3:
                break
        cpu = {"value": round(unknowns * count / el, 1), "unit": "grid-points/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{count} SR-CNN cycles of periodic1025 ({el:.1f} s, oracle: C V-cycle "
                         f"steps and float64 torch CPU convolutions)"}
    r = res["srcnn"]
    out = {
        "metric": "grid-points/s per V-cycle + time to 1e-10 rel. residual, 4097² Poisson",
        "value": round(unknowns / r["sec"], 1), "unit": "grid-points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["sec"] * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 network, f64 cycle", "data": "synthetic",
        "config": {"workload": "periodic1025_srcnn", "n": n, "bc": "periodic",
                   "unknowns": unknowns, "cnn_levels": 2, "seed": args.seed,
                   "weights": os.path.relpath(wpath, ROOT)},
        "time_to_1e-8_s": round(r["ttt"][0], 6), "cycles_to_1e-8": r["ttt"][2],
        "final_relres": r["ttt"][3],
        "spline": {"ms_per_cycle": round(res["spline"]["sec"] * 1e3, 4),
                   "time_to_1e-8_s": round(res["spline"]["ttt"][0], 6),
                   "cycles_to_1e-8": res["spline"]["ttt"][2]},
        "hybrid_n_gan_1": {"time_to_1e-8_s": round(res["hybrid"]["ttt"][0], 6),
                           "cycles_to_1e-8": res["hybrid"]["ttt"][2],
                           "final_relres": res["hybrid"]["ttt"][3],
                           "prolongations": res["hybrid"]["ops"]},
        "roofline": roofline, "kernels": per_kernel, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


def projection_traffic(kernel: str):
    """HBM bytes per launch of a projection kernel from the committed counter
    summary (profiles/hbm_traffic_projection.json), or None when its source
    has changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "hbm_traffic_projection.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    hh = hashlib.sha256()
    for src in rec["sources"]:
        hh.update(open(os.path.join(ROOT, src), "rb").read())
    if hh.hexdigest() != rec["sources_sha256"] or kernel not in rec["per_launch"]:
        return None
    return round(rec["per_launch"][kernel]["bytes"], 0)


def bench_projection(args) -> int:
    """4097 x 4097 periodic pressure-projection time step: the source
    f = -div((u . grad) u) (mg_ns_rhs), the pressure solve to 1e-10 (mixed
    precision, from the previous step's pressure) and the explicit Euler
    velocity step (mg_ns_update), ping-ponging two velocity buffers.  A step
    is those three.  Each projection kernel is also timed on its own with HIP
    events on the stream it runs on."""
    import numpy as np
    import torch

    import workloads
    from paper_2403_07936_amd import binding as B
    from paper_2403_07936_amd.solver import Solver

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    B.lib()
    # The known-size device copy that scales HBM counters under a profiler
    # (as in the default workload).
    calib = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device=dev)
    calib_dst = torch.empty_like(calib)
    calib.fill_(1.0)
    calib_dst.copy_(calib)
    torch.cuda.synchronize()
    del calib, calib_dst
    n, N = 4097, 4096
    log(f"generating velocity n={n} seed {args.seed}")
    ux, uy = workloads.velocity_periodic(n, args.seed)
    # The explicit velocity step with central differences grows the shortest
    # waves by sqrt(1 + CFL^2) per step: at CFL 0.25 the timed steps stay
    # bounded (at dt = 1e-4, CFL 1.1, the field blew up within 17 steps).
    cfl = 0.25
    dt = cfl / (N * float(max(np.abs(ux).max(), np.abs(uy).max())))
    vel = [[torch.from_numpy(ux).to(dev), torch.from_numpy(uy).to(dev)]]
    vel.append([torch.empty_like(vel[0][0]), torch.empty_like(vel[0][0])])
    f = torch.zeros_like(vel[0][0])
    q = torch.zeros_like(f)  # the solver's output, -p: handed to mg_ns_update unchanged
    stream = torch.cuda.current_stream().cuda_stream
    s = Solver([(n, "periodic")], precision="mixed")
    F64 = B.MG_DT_F64
    cyc_log = []

    def step(k):
        a, b = vel[k % 2], vel[(k + 1) % 2]
        B.mg_ns_rhs(n, a[0].data_ptr(), a[1].data_ptr(), f.data_ptr(), n, F64, stream)
        st, cyc, rel = s.solve([q], [f], rtol=1e-10, max_cycles=30)
        if st != 0:
            raise RuntimeError(f"pressure solve failed: status {st}, relres {rel[0]:.2e}")
        cyc_log.append(cyc[0])
        B.mg_ns_update(n, a[0].data_ptr(), a[1].data_ptr(), q.data_ptr(), dt, b[0].data_ptr(),
                       b[1].data_ptr(), n, F64, stream)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    cyc_log.clear()
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        step(k)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    log(f"projection step: {sec * 1e3:.3f} ms, solve cycles {cyc_log}")

    def kernel_avg(fn, reps=20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    a, b = vel[0], vel[1]
    t_rhs = kernel_avg(lambda: B.mg_ns_rhs(n, a[0].data_ptr(), a[1].data_ptr(), f.data_ptr(), n,
                                           F64, stream))
    t_upd = kernel_avg(lambda: B.mg_ns_update(n, a[0].data_ptr(), a[1].data_ptr(), q.data_ptr(),
                                              dt, b[0].data_ptr(), b[1].data_ptr(), n, F64,
                                              stream))
    by_rhs, by_upd = 3 * 8 * N * N, 5 * 8 * N * N
    kernels = {"ns_rhs": {"avg_us": round(t_rhs * 1e6, 2), "bytes": by_rhs,
                          "GBps": round(by_rhs / t_rhs / 1e9, 1)},
               "ns_update": {"avg_us": round(t_upd * 1e6, 2), "bytes": by_upd,
                             "GBps": round(by_upd / t_upd / 1e9, 1)}}
    log(f"kernels: {kernels}")
    ach = by_upd / t_upd / 1e9
    roofline = {"bound": "hbm", "kernel": "ns_update", "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": projection_traffic("k_ns_update<double>"),
                "avg_launch_us": round(t_upd * 1e6, 2), "bytes_per_launch": by_upd}
    cpu = None
    if not args.no_cpu:
        import oracle
        from oracle import projection as pj

        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        pj.time_step(ux, uy, dt,
                     lambda fo: oracle.solve(fo, oracle.PERIODIC, rtol=1e-10, max_cycles=30)[0])
        el = time.perf_counter() - t0
        cpu = {"value": round(N * N / el, 1), "unit": "grid-points/s", "cores": threads,
               "kind": "oracle",
               "sample": f"one projection step of periodic4097 from p = 0 ({el:.1f} s: numpy "
                         f"source and update, plain C FP64 V-cycles to 1e-10)"}
    out = {
        "metric": "grid-points/s per pressure-projection time step (source, solve to 1e-10, "
                  "velocity step)",
        "value": round(N * N / sec, 1), "unit": "grid-points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "periodic4097_projection", "n": n, "bc": "periodic",
                   "unknowns": N * N, "dt": dt, "cfl": cfl,
                   "solve": "mixed, rtol 1e-10, warm start",
                   "seed": args.seed},
        "solve_cycles": cyc_log, "roofline": roofline, "kernels": kernels, "cpu_baseline": cpu,
    }
    s.close()
    print(json.dumps(out), flush=True)
    return 0


# FP64 vector arithmetic of MI355X for single adds and multiplies (the
# two-level kernel has no fused multiply-adds): 256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz = 39.3 T operations/s (the published 78.6 TFLOP/s counts an FMA
# as two).
FP64_ADDMUL_PEAK_TFLOPS = 39.3


def twolevel_flops(N, F, n_smooth, coarse_sweeps):
    """Algorithmic FP64 operations of one two-level iteration of one problem:
    5 per node and sweep (three adds for the neighbour sum, one add, one
    multiply), 7 per node for the residual, 2 per weight for the two
    restriction passes, 5 per coarse node and sweep, 2 Nc per coefficient for
    the two prefilter products, 8 per x-interpolated value, 10 per node for
    the evaluation along y, the correction and the change."""
    Nc = N // F
    return (5 * n_smooth * N * N + 7 * N * N + 2 * (2 * F - 1) * (N * Nc + Nc * Nc)
            + 5 * coarse_sweeps * Nc * Nc + 2 * 2 * Nc * Nc * Nc + 8 * Nc * N + 10 * N * N)


def bench_twolevel(args) -> int:
    """The paper's controlled two-level experiment (Section 4.1, Table 1):
    the 100-problem test set of 192 x 192 periodic grids coarsened directly to
    12 x 12 (N_step = 4), 20 sweeps per iteration, the coarse level relaxed 10
    times, N_smooth,pre = 10 on the random initial grid, stop once the change
    between iterates is <= 1e-10.  A step is one iteration of the whole test
    set (every problem active).  Also reported: time to tolerance of the
    whole set (device-side stopping per problem)."""
    import numpy as np
    import torch

    import workloads
    from paper_2403_07936_amd import binding as B

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    B.lib()
    N, F, ns, cs, npre, tol = workloads.TWOLEVEL_N, 16, 20, 10, 10, 1e-10
    count = workloads.TWOLEVEL_BATCH
    log(f"generating the two-level test set ({count} problems of {N}^2) seed {args.seed}")
    f, p0 = workloads.twolevel_batch(args.seed)
    ft = torch.from_numpy(f).to(dev)
    pt = torch.from_numpy(p0).to(dev)
    stream = torch.cuda.current_stream().cuda_stream
    ctx = B.mg_twolevel_setup(N, F, count, ns, cs, stream)
    try:
        B.mg_twolevel_cycle(ctx, pt.data_ptr(), ft.data_ptr(), args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.mg_twolevel_cycle(ctx, pt.data_ptr(), ft.data_ptr(), args.steps)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / args.steps

        # The iteration kernel alone, with HIP events on the stream it runs on:
        # a call of K iterations packs h^2 f once, so the difference between
        # K and 1 iterations over K - 1 is one launch of the iteration kernel.
        def timed(k, reps=3):
            best = None
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                B.mg_twolevel_cycle(ctx, pt.data_ptr(), ft.data_ptr(), k)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                best = ms if best is None else min(best, ms)
            return best * 1e-3

        k = max(args.steps, 2)
        t_launch = (timed(k) - timed(1)) / (k - 1)
        best = None
        for _ in range(3):
            pt.copy_(torch.from_numpy(p0))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, it, ch = B.mg_twolevel_solve(ctx, pt.data_ptr(), ft.data_ptr(), count, npre, tol,
                                             300)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best[0]:
                best = (dt, st, it, ch)
        log(f"two-level: {sec * 1e3:.3f} ms per iteration of the test set "
            f"(kernel {t_launch * 1e6:.1f} us); all to change <= {tol:g}: "
            f"{best[0] * 1e3:.2f} ms, iterations {min(best[2])}..{max(best[2])}, status {best[1]}")
    finally:
        B.mg_twolevel_destroy(ctx)
    flops = count * twolevel_flops(N, F, ns, cs)
    ach = flops / t_launch / 1e12
    roofline = {"bound": "alu", "kernel": "k_twolevel", "achieved": round(ach, 3),
                "peak": FP64_ADDMUL_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / FP64_ADDMUL_PEAK_TFLOPS, 4), "traffic": None,
                "avg_launch_us": round(t_launch * 1e6, 2), "flops_per_launch": flops,
                "note": f"{count} workgroups (one per problem) on 256 compute units"}
    cpu = None
    if not args.no_cpu:
        import oracle

        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds:
            b = done % count
            oracle.twolevel(p0[b], f[b], F, ns, cs)
            done += 1
        el = time.perf_counter() - t0
        cpu = {"value": round(done * N * N / el, 1), "unit": "grid-points/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{done} two-level iterations of test-set problems ({el:.1f} s, plain "
                         f"C oracle, OpenMP over independent grid lines)"}
    out = {
        "metric": "grid-points/s per two-level iteration of the 100-problem 192^2 test set, "
                  "and time to a change <= 1e-10",
        "value": round(count * N * N / sec, 1), "unit": "grid-points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "twolevel192", "problems": count, "n_unique": N, "factor": F,
                   "coarse": N // F, "n_smooth": ns, "coarse_sweeps": cs, "n_smooth_pre": npre,
                   "tol_change": tol, "bc": "periodic", "seed": args.seed},
        "time_to_tol_s": round(best[0], 6), "status": best[1],
        "iterations": {"min": min(best[2]), "max": max(best[2]),
                       "mean": round(float(np.mean(best[2])), 2)},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


def measure_single(n, bc, f, steps, warmup, tune_cache, dev, reps=3):
    """FP64 and mixed paths on one resident grid: seconds per step (K steps
    after W warm-up steps, each one mg_vcycle call), and the best of `reps`
    solves to 1e-10 from u = 0.  Returns {precision: {...}} with the solvers
    left open."""
    import torch

    from paper_2403_07936_amd.solver import Solver

    ft = torch.from_numpy(f).to(dev)
    ut = torch.zeros_like(ft)
    res = {}
    for prec in ("fp64", "mixed"):
        s = Solver([(n, bc)], precision=prec, use_graph=True, tune_cache_path=tune_cache)
        ut.zero_()
        s.vcycle([ut], [ft], warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.vcycle([ut], [ft], 1)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        best = None
        for _ in range(reps):
            ut.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, cyc, rel = s.solve([ut], [ft], rtol=1e-10, max_cycles=50)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best[0]:
                best = (dt, st, cyc[0], rel[0])
        res[prec] = {"solver": s, "sec_per_step": sec, "ttt": best, "u": ut.clone()}
        log(f"n={n} {prec}: {sec * 1e3:.3f} ms/cycle; to 1e-10: {best[0] * 1e3:.2f} ms, "
            f"{best[2]} cycles, relres {best[3]:.2e}, status {best[1]}")
    return res, ft, ut


def measure_batch(probs, steps, warmup, tune_cache, dev, reps=2):
    """FP64 and mixed paths on the 256-problem batch (schedule autotuned:
    the persistent launch or per-problem graphs): seconds per step (one
    mg_vcycle call steps every problem), and the best of `reps` solves of
    all problems to 1e-10 from u = 0 (problems stop independently)."""
    import torch

    from paper_2403_07936_amd.solver import Solver

    fts = [torch.from_numpy(f).to(dev) for _, _, f in probs]
    uts = [torch.zeros_like(t) for t in fts]
    grids = [(n, bc) for n, bc, _ in probs]
    res = {}
    for prec in ("fp64", "mixed"):
        t0 = time.perf_counter()
        s = Solver(grids, precision=prec, use_graph=True, tune_cache_path=tune_cache)
        t_setup = time.perf_counter() - t0
        for t in uts:
            t.zero_()
        s.vcycle(uts, fts, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.vcycle(uts, fts, 1)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        best = None
        for _ in range(reps):
            for t in uts:
                t.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, cyc, rel = s.solve(uts, fts, rtol=1e-10, max_cycles=50)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best[0]:
                best = (dt, st, max(cyc), max(rel), [u.clone() for u in uts])
        res[prec] = {"solver": s, "sec_per_step": sec, "ttt": best, "setup_s": t_setup}
        log(f"batch {prec}: {sec * 1e3:.3f} ms/step; all to 1e-10: {best[0] * 1e3:.2f} ms, "
            f"max {best[2]} cycles, max relres {best[3]:.2e}, status {best[1]} "
            f"(setup with tuning {t_setup:.1f} s)")
    return res, fts


def kernel_events(B, solver, run, level=0):
    """Kernel classes of one context from HIP events around every launch
    (on the context's stream) while `run()` queues steps: list of
    (total_ms, kind, launches, algorithmic_bytes), largest time first."""
    import torch

    B.mg_timing_enable(solver.ctx, True)
    torch.cuda.synchronize()
    run()
    torch.cuda.synchronize()
    kern = []
    for kind in range(B.MG_K_COUNT):
        cnt, ms, by = B.mg_timing_read(solver.ctx, kind, level)
        if cnt:
            kern.append((ms, kind, cnt, by))
    B.mg_timing_enable(solver.ctx, False)
    kern.sort(reverse=True)
    return kern


def path_summary(res, unknowns):
    return {p: {"ms_per_step": round(r["sec_per_step"] * 1e3, 4),
                "grid_points_per_s": round(unknowns / r["sec_per_step"], 1),
                "time_to_tol_s": round(r["ttt"][0], 6), "cycles_to_tol": r["ttt"][2],
                "final_relres": r["ttt"][3], "status": r["ttt"][1]}
            for p, r in res.items()}


def batch_errors(probs, res, sample):
    """Relative 2-norm error of the batch solves against the oracle's FP64
    solutions on the problems in `sample` (mean removed: periodic)."""
    import numpy as np

    import oracle

    err = {p: 0.0 for p in res}
    for b in sample:
        n, bc, f = probs[b]
        uo = oracle.solve(f, bc, rtol=1e-10, max_cycles=50)[0]
        uo = uo[:-1, :-1] - uo[:-1, :-1].mean()
        for p, r in res.items():
            g = r["ttt"][4][b].cpu().numpy()
            g = g[:-1, :-1] - g[:-1, :-1].mean()
            err[p] = max(err[p], float(np.linalg.norm(g - uo) / np.linalg.norm(uo)))
    return err


def bench_batch(args, B, dev, probs, full: bool):
    """The 256-problem periodic batch (sides 129..1025, one persistent launch
    per step when the tuner picks it).  full=False: the compact sub-object of
    the default line; full=True: the workload's own JSON line."""
    import numpy as np

    import workloads

    unknowns = sum(workloads.grid_unknowns(n, bc) for n, bc, _ in probs)
    steps, warmup = (args.steps, args.warmup) if full else (min(args.steps, 10), 2)
    res, fts = measure_batch(probs, steps, warmup, args.tune_cache, dev)
    head = min(res, key=lambda p: res[p]["sec_per_step"])
    hs = res[head]["solver"]
    uts = res[head]["ttt"][4]

    def run():
        for _ in range(steps):
            hs.vcycle(uts, fts, 1)

    kern = kernel_events(B, hs, run)
    ms, kind, cnt, by = kern[0]
    avg = ms / cnt
    ach = (by / cnt) / (avg * 1e-3) / 1e9 if by > 0 else None
    roofline = {"bound": "hbm", "kernel": B.mg_kernel_name(kind),
                "achieved": round(ach, 1) if ach else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4) if ach else None, "traffic": None,
                "avg_launch_us": round(avg * 1e3, 2), "bytes_per_launch": by / cnt}
    sample = list(range(0, len(probs), 16)) if not args.no_cpu else []
    errs = batch_errors(probs, res, sample) if sample else {}
    sub = {
        "problems": len(probs), "unknowns": unknowns,
        "sizes": {str(m): sum(1 for n, _, _ in probs if n == m) for m in workloads.SIZES_BATCHED},
        "head": head, "paths": path_summary(res, unknowns),
        "speedup_mixed_vs_fp64": round(res["fp64"]["sec_per_step"] / res["mixed"]["sec_per_step"], 3),
        "schedule": {B.MG_K_PERSISTENT: "persistent", B.MG_K_PHASED: "one launch per phase"}.get(
            kind, "per-problem graphs"),
        "roofline": roofline,
        "setup_s": {p: round(r["setup_s"], 2) for p, r in res.items()},
    }
    if errs:
        sub["err_vs_oracle_fp64"] = {p: errs[p] for p in errs}
        sub["err_sample"] = f"problems {sample[0]}, {sample[1]}, ... (every 16th), oracle FP64 " \
                            f"solve to 1e-10"
    cpu = None
    if full and not args.no_cpu:
        import oracle

        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log(f"CPU baseline: oracle {head} steps over the batch for ~{args.cpu_seconds:.0f} s")
        done, t0, b = 0, time.perf_counter(), 0
        while True:
            n, bc, f = probs[b % len(probs)]
            u = np.zeros_like(f)
            u = oracle.vcycle(u, f, bc) if head == "fp64" else oracle.refine_step(u, f, bc)
            done += workloads.grid_unknowns(n, bc)
            b += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds:
                break
        cpu = {"value": round(done / el, 1), "unit": "grid-points/s", "cores": threads,
               "kind": "oracle",
               "sample": f"one {head} step of each of the first {b} problems of batch256 "
                         f"({done} unknowns, {el:.1f} s, plain C oracle)"}
    for r in res.values():
        r["solver"].close()
    if not full:
        return sub
    r = res[head]
    out = {
        "metric": "grid-points/s per V-cycle + time to 1e-10 rel. residual, 256-problem batch",
        "value": round(unknowns / r["sec_per_step"], 1), "unit": "grid-points/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(r["sec_per_step"] * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": "batch256", "bc": "periodic", "problems": len(probs),
                   "unknowns": unknowns, "precision": head, "seed": args.seed},
        "time_to_tol_s": round(r["ttt"][0], 6), "cycles_to_tol_max": r["ttt"][2],
        "final_relres_max": r["ttt"][3],
        "roofline": roofline, "cpu_baseline": cpu,
    }
    out.update({k: v for k, v in sub.items() if k not in ("roofline",)})
    return out


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (this build has no multi-GPU path); "
              f"got --gpus {args.gpus}", file=sys.stderr)
        return 2
    if args.workload == "periodic1025_srcnn":
        return bench_srcnn(args)
    if args.workload == "periodic4097_projection":
        return bench_projection(args)
    if args.workload == "twolevel192":
        return bench_twolevel(args)

    import numpy as np
    import torch

    import workloads
    from paper_2403_07936_amd import binding as B

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    B.lib()

    # A plain device copy of known size (256 MiB read + 256 MiB written): the
    # reference dispatch for scaling HBM traffic counters (FETCH_SIZE,
    # WRITE_SIZE) when this script runs under a counter-collecting profiler.
    calib = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device=dev)
    calib_dst = torch.empty_like(calib)
    calib.fill_(1.0)
    calib_dst.copy_(calib)
    torch.cuda.synchronize()
    del calib, calib_dst

    if args.workload == "batch256":
        log(f"generating batch256 seed {args.seed}")
        probs = workloads.workload("batch256", args.seed)
        out = bench_batch(args, B, dev, probs, full=True)
        print(json.dumps(out), flush=True)
        return 0

    log(f"generating {args.workload} seed {args.seed}")
    n, bc, f = workloads.workload(args.workload, args.seed)
    unknowns = workloads.grid_unknowns(n, bc)
    results, ft, ut = measure_single(n, bc, f, args.steps, args.warmup, args.tune_cache, dev)

    head = min(results, key=lambda p: results[p]["sec_per_step"])
    hs = results[head]["solver"]

    # Per-kernel timing: the same number of steps again with every launch
    # bracketed by HIP events on the solver's stream (no graph capture).
    def run():
        ut.zero_()
        for _ in range(args.steps):
            hs.vcycle([ut], [ft], 1)

    kern = kernel_events(B, hs, run)
    ms, kind, cnt, by = kern[0]
    avg_ms = ms / cnt
    achieved = (by / cnt) / (avg_ms * 1e-3) / 1e9
    per_kernel = {B.mg_kernel_name(k): {"launches": c, "avg_us": 1e3 * m / c,
                                        "GBps": (b / c) / (m / c * 1e-3) / 1e9}
                  for m, k, c, b in kern}
    log(f"level-0 kernels (events): {json.dumps(per_kernel)}")
    roofline = {"bound": "hbm", "kernel": B.mg_kernel_name(kind), "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(B.mg_kernel_name(kind), head, bc),
                "avg_launch_us": round(avg_ms * 1e3, 2), "bytes_per_launch": by / cnt}

    extra = {}
    cpu = None
    if not args.no_cpu:
        import oracle

        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log(f"oracle FP64 solve for the error check ({threads} threads)")
        t0 = time.perf_counter()
        uo, co, ho = oracle.solve(f, bc, rtol=1e-10, max_cycles=50)
        t_orc = time.perf_counter() - t0
        for prec in results:
            got = results[prec]["u"].cpu().numpy()
            a, b = got, uo
            if bc == workloads.rhs.PERIODIC:
                a = a[:-1, :-1] - a[:-1, :-1].mean()
                b = b[:-1, :-1] - b[:-1, :-1].mean()
            extra[f"err_vs_oracle_fp64_{prec}"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        extra["oracle_fp64_cycles_to_tol"] = int(co)
        extra["oracle_fp64_time_to_tol_s"] = round(t_orc, 3)

        log(f"CPU baseline: oracle {head} cycles for ~{args.cpu_seconds:.0f} s")
        u = np.zeros_like(f)
        step = (lambda u: oracle.vcycle(u, f, bc)) if head == "fp64" else \
            (lambda u: oracle.refine_step(u, f, bc))
        count, t0 = 0, time.perf_counter()
        while True:
            u = step(u)
            count += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds and count >= 2:
                break
        cpu = {"value": round(unknowns * count / el, 1), "unit": "grid-points/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{count} {head} cycles of {args.workload} ({el:.1f} s, plain C oracle, "
                         f"OpenMP over independent grid lines)"}

    hr = results[head]
    sec = hr["sec_per_step"]
    out = {
        "metric": "grid-points/s per V-cycle + time to 1e-10 rel. residual, 4097² Poisson",
        "value": round(unknowns / sec, 1),
        "unit": "grid-points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n,
                   "bc": "dirichlet" if bc == 0 else "periodic", "unknowns": unknowns,
                   "levels": hs.num_levels(), "cycle": "V(2,2) red-black GS, full weighting, "
                   "cubic-spline prolongation, direct 5x5 solve", "precision": head,
                   "seed": args.seed},
        "time_to_tol_s": round(hr["ttt"][0], 6),
        "cycles_to_tol": hr["ttt"][2],
        "final_relres": hr["ttt"][3],
        "paths": {p: {"ms_per_cycle": round(r["sec_per_step"] * 1e3, 4),
                      "grid_points_per_s": round(unknowns / r["sec_per_step"], 1),
                      "time_to_tol_s": round(r["ttt"][0], 6), "cycles_to_tol": r["ttt"][2],
                      "final_relres": r["ttt"][3], "status": r["ttt"][1]}
                  for p, r in results.items()},
        "roofline": roofline,
        "kernels_level0": per_kernel,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    for r in results.values():
        r["solver"].close()
    del ft, ut
    torch.cuda.empty_cache()

    if args.workload == "dirichlet4097" and not args.no_extra:
        # The other configurations, measured by the same run: the periodic
        # 1025^2 grid (FP64 against mixed) and the 256-problem batch.
        subs = {}
        n2, bc2, f2 = workloads.workload("periodic1025", args.seed)
        r2, ft2, ut2 = measure_single(n2, bc2, f2, args.steps, args.warmup, args.tune_cache, dev)
        u2 = workloads.grid_unknowns(n2, bc2)
        subs["periodic1025"] = {"unknowns": u2, "paths": path_summary(r2, u2),
                                "speedup_mixed_vs_fp64": round(
                                    r2["fp64"]["sec_per_step"] / r2["mixed"]["sec_per_step"], 3)}
        for r in r2.values():
            r["solver"].close()
        del ft2, ut2
        log(f"generating batch256 seed {args.seed}")
        probs = workloads.workload("batch256", args.seed)
        subs["batch256"] = bench_batch(args, B, dev, probs, full=False)
        # The learned prolongation on the periodic 1025^2 source: network
        # cycles (bf16 matrix cores) against the spline and the hybrid
        # schedule, and the level-0 convolutions against the bf16 peak.
        import numpy as np
        W = np.load(args.weights or WEIGHTS)
        (n5, bc5, _), r5, roof5, _ = measure_srcnn(args, dev, W, args.steps, args.warmup)
        u5 = workloads.grid_unknowns(n5, bc5)
        subs["periodic1025_srcnn"] = {"unknowns": u5, "cnn_levels": 2,
                                      "weights": os.path.relpath(args.weights or WEIGHTS, ROOT),
                                      "paths": srcnn_summary(r5, u5), "roofline": roof5}
        out["other_workloads"] = subs
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
