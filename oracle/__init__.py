"""Plain CPU reference ("oracle") for the 2-D Poisson multigrid V-cycle.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It is built from the
C sources in this directory (``gcc -O2 -ffp-contract=off``), shares no code
with the HIP library and never imports it.

Every function takes and returns ``numpy`` arrays laid out as in
``workloads`` (square ``(n, n)`` row-major, i = y, j = x).

Pins: each function is checked in ``tests/test_oracle_pins.py`` against
something other than itself (closed forms, scipy/numpy library routines,
dense linear algebra on tiny grids, invariants).  No function is "parity
unpinned".  The SR-CNN prolongation and the hybrid schedule live in
``srcnn.py`` (pins in ``tests/test_srcnn_pins.py``), the pressure-projection
steps around the solve in ``projection.py`` (``tests/test_projection_pins.py``).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

DIRICHLET = 0
PERIODIC = 1
RED = 0
BLACK = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ("mg_oracle_core.c", "mg_oracle_drivers.c")


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` and return its path."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    core = os.path.join(_HERE, "mg_oracle_core.c")
    drv = os.path.join(_HERE, "mg_oracle_drivers.c")
    flags = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-std=c11", "-Wall", "-fopenmp"]
    # The core is compiled twice (FP64, and FP32 emulation of the inner
    # cycle of the mixed path) into separate objects, then linked with the
    # FP64 drivers.
    objs = []
    for real, sfx in (("double", "f64"), ("float", "f32")):
        obj = os.path.join(_HERE, f"_core_{sfx}.o")
        subprocess.check_call(["gcc"] + flags + ["-c", f"-DREAL={real}", f"-DSFX={sfx}",
                                                 "-o", obj, core])
        objs.append(obj)
    obj = os.path.join(_HERE, "_drivers.o")
    subprocess.check_call(["gcc"] + flags + ["-c", "-o", obj, drv])
    objs.append(obj)
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-shared", "-fopenmp", "-o", tmp] + objs + ["-lm"])
    os.replace(tmp, _LIB_PATH)
    for o in objs:
        os.remove(o)
    return _LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        pd = ctypes.POINTER(ctypes.c_double)
        pf = ctypes.POINTER(ctypes.c_float)
        i = ctypes.c_int
        for sfx, p in (("f64", pd), ("f32", pf)):
            getattr(L, f"orc_relax_{sfx}").argtypes = [i, i, p, p, i]
            getattr(L, f"orc_residual_{sfx}").argtypes = [i, i, p, p, p]
            getattr(L, f"orc_restrict_{sfx}").argtypes = [i, i, p, p]
            getattr(L, f"orc_prolong_{sfx}").argtypes = [i, i, p, p]
            getattr(L, f"orc_coarse_{sfx}").argtypes = [i, p, p]
            getattr(L, f"orc_vcycle_{sfx}").argtypes = [i, i, i, i, p, p]
            getattr(L, f"orc_restrict_factor_{sfx}").argtypes = [i, i, p, p]
            getattr(L, f"orc_prolong_factor_{sfx}").argtypes = [i, i, p, p]
            getattr(L, f"orc_twolevel_{sfx}").argtypes = [i, i, i, i, p, p]
            for name in ("relax", "residual", "restrict", "prolong", "coarse", "vcycle",
                         "restrict_factor", "prolong_factor", "twolevel"):
                getattr(L, f"orc_{name}_{sfx}").restype = None
        L.orc_coarse_direct.argtypes = [i, pd, pd]
        L.orc_coarse_direct.restype = None
        L.orc_norm2.argtypes = [i, i, pd]
        L.orc_norm2.restype = ctypes.c_double
        L.orc_relres.argtypes = [i, i, pd, pd]
        L.orc_relres.restype = ctypes.c_double
        L.orc_solve_f64.argtypes = [i, i, i, i, pd, pd, ctypes.c_double, i, pd]
        L.orc_solve_f64.restype = i
        L.orc_refine_step.argtypes = [i, i, i, i, i, pd, pd]
        L.orc_refine_step.restype = None
        L.orc_solve_mixed.argtypes = [i, i, i, i, i, pd, pd, ctypes.c_double, i, pd]
        L.orc_solve_mixed.restype = i
        L.orc_twolevel_solve.argtypes = [i, i, i, i, i, pd, pd, ctypes.c_double, i, pd]
        L.orc_twolevel_solve.restype = i
        _lib = L
    return _lib


def _dt(dtype) -> tuple[str, type]:
    dtype = np.dtype(dtype)
    if dtype == np.float64:
        return "f64", ctypes.c_double
    if dtype == np.float32:
        return "f32", ctypes.c_float
    raise TypeError(dtype)


def _ptr(a: np.ndarray, ctype):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _sq(a: np.ndarray, dtype=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=dtype)
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("expected a square 2-D array")
    return a


def levels(n: int) -> list[int]:
    """Grid sides of the hierarchy from n down to 5."""
    out = [n]
    while out[-1] > 5:
        out.append((out[-1] - 1) // 2 + 1)
    return out


def relax(u: np.ndarray, f: np.ndarray, bc: int, colour: int) -> np.ndarray:
    """One red (colour 0) or black (colour 1) Gauss-Seidel half-sweep; returns new u."""
    u = _sq(u).copy()
    sfx, ct = _dt(u.dtype)
    f = _sq(f, u.dtype)
    getattr(lib(), f"orc_relax_{sfx}")(u.shape[0], bc, _ptr(u, ct), _ptr(f, ct), colour)
    return u


def residual(u: np.ndarray, f: np.ndarray, bc: int) -> np.ndarray:
    u = _sq(u)
    sfx, ct = _dt(u.dtype)
    f = _sq(f, u.dtype)
    r = np.empty_like(u)
    getattr(lib(), f"orc_residual_{sfx}")(u.shape[0], bc, _ptr(u, ct), _ptr(f, ct), _ptr(r, ct))
    return r


def restrict(r: np.ndarray, bc: int) -> np.ndarray:
    r = _sq(r)
    sfx, ct = _dt(r.dtype)
    n = r.shape[0]
    nc = (n - 1) // 2 + 1
    fc = np.empty((nc, nc), dtype=r.dtype)
    getattr(lib(), f"orc_restrict_{sfx}")(n, bc, _ptr(r, ct), _ptr(fc, ct))
    return fc


def prolong(ec: np.ndarray, bc: int) -> np.ndarray:
    """Cubic-spline interpolation of a coarse grid function to the next finer grid."""
    ec = _sq(ec)
    sfx, ct = _dt(ec.dtype)
    nc = ec.shape[0]
    n = 2 * (nc - 1) + 1
    ef = np.empty((n, n), dtype=ec.dtype)
    getattr(lib(), f"orc_prolong_{sfx}")(nc, bc, _ptr(ec, ct), _ptr(ef, ct))
    return ef


def coarse_solve(f: np.ndarray, bc: int) -> np.ndarray:
    """Direct solve on the 5 x 5 grid (FP64)."""
    f = _sq(f, np.float64)
    assert f.shape == (5, 5)
    u = np.empty_like(f)
    lib().orc_coarse_direct(bc, _ptr(f, ctypes.c_double), _ptr(u, ctypes.c_double))
    return u


def vcycle(u: np.ndarray, f: np.ndarray, bc: int, nu1: int = 2, nu2: int = 2) -> np.ndarray:
    """One V(nu1, nu2) cycle; returns the new u (input untouched)."""
    u = _sq(u).copy()
    sfx, ct = _dt(u.dtype)
    f = _sq(f, u.dtype)
    getattr(lib(), f"orc_vcycle_{sfx}")(u.shape[0], bc, nu1, nu2, _ptr(u, ct), _ptr(f, ct))
    return u


def norm2(a: np.ndarray, bc: int) -> float:
    a = _sq(a, np.float64)
    return lib().orc_norm2(a.shape[0], bc, _ptr(a, ctypes.c_double))


def relres(u: np.ndarray, f: np.ndarray, bc: int) -> float:
    u = _sq(u, np.float64)
    f = _sq(f, np.float64)
    return lib().orc_relres(u.shape[0], bc, _ptr(u, ctypes.c_double), _ptr(f, ctypes.c_double))


def solve(f: np.ndarray, bc: int, rtol: float = 1e-10, max_cycles: int = 50,
          u0: np.ndarray | None = None, nu1: int = 2, nu2: int = 2):
    """Plain FP64 V-cycles from u0 (default 0).  Returns (u, cycles, history)."""
    f = _sq(f, np.float64)
    u = np.zeros_like(f) if u0 is None else _sq(u0, np.float64).copy()
    hist = np.full(max_cycles + 1, np.nan)
    c = lib().orc_solve_f64(f.shape[0], bc, nu1, nu2, _ptr(u, ctypes.c_double),
                            _ptr(f, ctypes.c_double), rtol, max_cycles,
                            _ptr(hist, ctypes.c_double))
    return u, c, hist[: c + 1]


def refine_step(u: np.ndarray, f: np.ndarray, bc: int, inner: int = 1,
                nu1: int = 2, nu2: int = 2) -> np.ndarray:
    """One mixed-precision refinement step; returns the new FP64 u."""
    u = _sq(u, np.float64).copy()
    f = _sq(f, np.float64)
    lib().orc_refine_step(u.shape[0], bc, nu1, nu2, inner, _ptr(u, ctypes.c_double),
                          _ptr(f, ctypes.c_double))
    return u


def solve_mixed(f: np.ndarray, bc: int, rtol: float = 1e-10, max_steps: int = 50,
                inner: int = 1, u0: np.ndarray | None = None, nu1: int = 2, nu2: int = 2):
    """FP64 refinement around FP32 V-cycles.  Returns (u, steps, history)."""
    f = _sq(f, np.float64)
    u = np.zeros_like(f) if u0 is None else _sq(u0, np.float64).copy()
    hist = np.full(max_steps + 1, np.nan)
    c = lib().orc_solve_mixed(f.shape[0], bc, nu1, nu2, inner, _ptr(u, ctypes.c_double),
                              _ptr(f, ctypes.c_double), rtol, max_steps,
                              _ptr(hist, ctypes.c_double))
    return u, c, hist[: c + 1]


# ---- the paper's controlled two-level experiment (periodic grids only) -----

def _check_factor(n: int, F: int) -> None:
    """The two-level grids: N = n - 1 unique nodes, N / F of them on the
    coarse grid, both even (red-black colouring must agree across the wrap)."""
    N = n - 1
    if F < 2 or N % F or N % 2 or (N // F) % 2 or N // F < 2:
        raise ValueError(f"unique side {N} and factor {F}: need N and N/F even, N/F >= 2")


def restrict_factor(r: np.ndarray, F: int) -> np.ndarray:
    """Restriction of a periodic grid function by the factor F (full weighting
    widened to the step: 1-D weights (F - |a|)/F^2, x then y)."""
    r = _sq(r)
    sfx, ct = _dt(r.dtype)
    n = r.shape[0]
    _check_factor(n, F)
    nc = (n - 1) // F + 1
    fc = np.empty((nc, nc), dtype=r.dtype)
    getattr(lib(), f"orc_restrict_factor_{sfx}")(n, F, _ptr(r, ct), _ptr(fc, ct))
    return fc


def prolong_factor(ec: np.ndarray, F: int) -> np.ndarray:
    """Periodic tensor cubic-spline interpolation by the factor F."""
    ec = _sq(ec)
    sfx, ct = _dt(ec.dtype)
    nc = ec.shape[0]
    n = F * (nc - 1) + 1
    _check_factor(n, F)
    ef = np.empty((n, n), dtype=ec.dtype)
    getattr(lib(), f"orc_prolong_factor_{sfx}")(nc, F, _ptr(ec, ct), _ptr(ef, ct))
    return ef


def twolevel(p: np.ndarray, f: np.ndarray, F: int, n_smooth: int = 20,
             coarse_sweeps: int = 10) -> np.ndarray:
    """One iteration of the two-level method; returns the new p."""
    p = _sq(p).copy()
    _check_factor(p.shape[0], F)
    sfx, ct = _dt(p.dtype)
    f = _sq(f, p.dtype)
    getattr(lib(), f"orc_twolevel_{sfx}")(p.shape[0], F, n_smooth, coarse_sweeps, _ptr(p, ct),
                                          _ptr(f, ct))
    return p


def twolevel_solve(f: np.ndarray, p0: np.ndarray, F: int, n_smooth: int = 20,
                   coarse_sweeps: int = 10, n_pre: int = 10, tol: float = 1e-10,
                   max_iter: int = 300):
    """n_pre sweeps on p0, then two-level iterations until the change between
    iterates is <= tol.  Returns (p, iterations, changes)."""
    f = _sq(f, np.float64)
    p = _sq(p0, np.float64).copy()
    _check_factor(p.shape[0], F)
    hist = np.full(max_iter, np.nan)
    it = lib().orc_twolevel_solve(f.shape[0], F, n_smooth, coarse_sweeps, n_pre,
                                  _ptr(p, ctypes.c_double), _ptr(f, ctypes.c_double), tol,
                                  max_iter, _ptr(hist, ctypes.c_double))
    return p, it, hist[:it]

