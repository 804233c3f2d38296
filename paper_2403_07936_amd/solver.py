"""torch-tensor front end of the C ABI (argument marshalling only).

``Solver`` owns one ``mg_ctx`` for a batch of problems.  Tensors must be
float64 CUDA (HIP) tensors of shape ``(n, n)`` whose rows may be strided
(``stride(1) == 1``); the row stride is passed as the pitch.
"""

from __future__ import annotations

import torch

from . import binding as B

PRECISIONS = {"fp64": B.MG_FP64, "mixed": B.MG_MIXED}
BCS = {"dirichlet": B.MG_BC_DIRICHLET0, "periodic": B.MG_BC_PERIODIC}


class Solver:
    def __init__(self, grids, precision: str = "fp64", nu_pre: int = 2, nu_post: int = 2,
                 inner_cycles: int = 1, use_graph: bool = True, check_every: int = 0,
                 pitch=None, stream: torch.cuda.Stream | None = None, schedule: int = 0,
                 kernel_path: int = 0, tune_cache_path: str | None = None,
                 cnn_weights=None, cnn_levels: int = 2, cnn_max_ratio: float = 0.5,
                 cnn_min_relres: float = 1e-7, n_gan: float = 0.0, s_thres: float = 0.0):
        """grids: sequence of (n, bc) with bc 0/1 or "dirichlet"/"periodic".
        pitch: optional sequence of row pitches (elements) of the level-0 arrays.
        schedule: 0 autotuned, 1 per-problem graphs, 2 one persistent launch per step,
            3 one launch per phase of the step for the whole batch.
        tune_cache_path: optional text file the autotuner reads and appends to.
        cnn_weights: optional flat float32 array of SR-CNN weights (MG_SRCNN_WEIGHT_COUNT
        values, see include/mg.h); selects the network prolongation on the
        cnn_levels finest levels.
        n_gan, s_thres: the hybrid prolongation schedule of mg_solve (N_GAN
        network prolongations per spline one, switch once a cycle changes u by
        at most s_thres); n_gan = 0 keeps the network-then-spline rule."""
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        opt = B.mg_options_default()
        opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        opt.nu_pre, opt.nu_post = nu_pre, nu_post
        opt.inner_cycles = inner_cycles
        opt.use_graph = int(bool(use_graph))
        opt.check_every = check_every
        opt.schedule = schedule
        opt.kernel_path = kernel_path
        self._cache_path = tune_cache_path.encode() if tune_cache_path else None
        opt.tune_cache_path = self._cache_path
        self._weights = None
        if cnn_weights is not None:
            import numpy as np

            self._weights = np.ascontiguousarray(cnn_weights, dtype=np.float32).reshape(-1)
            opt.prolong = B.MG_PROLONG_SRCNN
            opt.cnn_levels = cnn_levels
            opt.cnn_weights = self._weights.ctypes.data
            opt.cnn_weights_bytes = self._weights.nbytes
            opt.cnn_max_ratio = cnn_max_ratio
            opt.cnn_min_relres = cnn_min_relres
            opt.n_gan = n_gan
            opt.s_thres = s_thres
        self.grids = [(int(n), BCS[bc] if isinstance(bc, str) else int(bc)) for n, bc in grids]
        pitches = list(pitch) if pitch is not None else [0] * len(self.grids)
        self.pitch = [p if p else n for (n, _), p in zip(self.grids, pitches)]
        self.ctx = B.mg_setup([(n, bc, p) for (n, bc), p in zip(self.grids, self.pitch)], opt,
                              self.stream.cuda_stream)

    def _addr(self, ts, write: bool):
        if len(ts) != len(self.grids):
            raise ValueError(f"expected {len(self.grids)} arrays, got {len(ts)}")
        out = []
        for t, (n, _), p in zip(ts, self.grids, self.pitch):
            if t.dtype != torch.float64 or not t.is_cuda:
                raise TypeError("arrays must be float64 device tensors")
            if t.dim() != 2 or tuple(t.shape) != (n, n) or t.stride(1) != 1 or t.stride(0) != p:
                raise ValueError(f"array must be ({n}, {n}) with row stride {p}")
            out.append(t.data_ptr())
        return out

    def vcycle(self, u, f, ncycles: int = 1, relres: bool = False):
        return B.mg_vcycle(self.ctx, self._addr(u, True), self._addr(f, False), ncycles, relres)

    def solve(self, u, f, rtol: float = 1e-10, max_cycles: int = 50):
        return B.mg_solve(self.ctx, self._addr(u, True), self._addr(f, False), rtol, max_cycles)

    def history(self, problem: int = 0):
        """(prolongations, changes) per cycle of the last solve."""
        return B.mg_solve_history(self.ctx, problem)

    def num_levels(self, problem: int = 0) -> int:
        return B.mg_num_levels(self.ctx, problem)

    def close(self) -> None:
        if self.ctx:
            B.mg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
