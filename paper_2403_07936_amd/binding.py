"""ctypes binding of the C ABI in ``include/mg.h`` (argument marshalling only).

Functions keep the C names.  Device arrays are passed as integer device
addresses (e.g. ``tensor.data_ptr()``); every step of the solver runs in the
HIP library ``libmg355.so``.  There is no fallback: if the library is not
built or cannot be loaded, ``lib()`` raises.

torch is imported before the library is loaded so that the process uses a
single HIP runtime (torch's), which the library then shares.
"""

from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmg355.so")

MG_OK = 0
MG_ERR_INVALID_ARG = -1
MG_ERR_UNSUPPORTED = -2
MG_ERR_OOM = -3
MG_ERR_HIP = -4
MG_ERR_INCOMPATIBLE_RHS = -5
MG_ERR_NOT_CONVERGED = -6
MG_ERR_STAGNATED = -7
MG_ERR_NONFINITE = -8

MG_BC_DIRICHLET0 = 0
MG_BC_PERIODIC = 1
MG_FP64 = 0
MG_MIXED = 1
MG_PROLONG_SPLINE = 0
MG_PROLONG_SRCNN = 1
MG_DT_F64 = 0
MG_DT_F32 = 1

i32 = ctypes.c_int32
vp = ctypes.c_void_p


class mg_grid(ctypes.Structure):
    _fields_ = [("n", i32), ("bc", i32), ("pitch", i32)]


class mg_options(ctypes.Structure):
    _fields_ = [
        ("precision", i32),
        ("nu_pre", i32),
        ("nu_post", i32),
        ("inner_cycles", i32),
        ("prolong", i32),
        ("cnn_levels", i32),
        ("cnn_weights", vp),
        ("cnn_weights_bytes", ctypes.c_size_t),
        ("check_every", i32),
        ("use_graph", i32),
        ("tune_cache_path", ctypes.c_char_p),
        ("kernel_path", i32),
        ("schedule", i32),
        ("cnn_max_ratio", ctypes.c_double),
        ("cnn_min_relres", ctypes.c_double),
        ("n_gan", ctypes.c_double),
        ("s_thres", ctypes.c_double),
    ]


class MGError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{mg_status_string(status)} ({status}): {detail}")
        self.status = status
        self.detail = detail


_lib = None


def lib() -> ctypes.CDLL:
    """Load ``libmg355.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2403_07936_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    pp = ctypes.POINTER(vp)
    pd = ctypes.POINTER(ctypes.c_double)
    pi = ctypes.POINTER(i32)
    sig = {
        "mg_options_default": (None, [ctypes.POINTER(mg_options)]),
        "mg_setup": (i32, [ctypes.POINTER(mg_grid), i32, ctypes.POINTER(mg_options), vp,
                           ctypes.POINTER(vp)]),
        "mg_vcycle": (i32, [vp, pp, pp, i32, pd]),
        "mg_solve": (i32, [vp, pp, pp, ctypes.c_double, i32, pi, pd]),
        "mg_solve_history": (i32, [vp, i32, i32, pi, pd, pi]),
        "mg_ns_rhs": (i32, [i32, vp, vp, vp, i32, i32, vp]),
        "mg_ns_update": (i32, [i32, vp, vp, vp, ctypes.c_double, vp, vp, i32, i32, vp]),
        "mg_prolong": (i32, [vp, i32, i32, i32, vp, vp, i32]),
        "mg_prolong_noalloc": (i32, [i32, i32, vp, vp, i32, vp]),
        "mg_twolevel_setup": (i32, [i32, i32, i32, i32, i32, vp, ctypes.POINTER(vp)]),
        "mg_twolevel_smooth": (i32, [vp, vp, vp, i32]),
        "mg_twolevel_cycle": (i32, [vp, vp, vp, i32, pd]),
        "mg_twolevel_solve": (i32, [vp, vp, vp, i32, ctypes.c_double, i32, pi, pd]),
        "mg_twolevel_destroy": (i32, [vp]),
        "mg_relax": (i32, [vp, i32, i32, vp, vp, i32, i32, i32]),
        "mg_residual": (i32, [vp, i32, i32, vp, vp, vp, i32]),
        "mg_restrict": (i32, [vp, i32, i32, vp, vp, i32]),
        "mg_coarse_solve": (i32, [vp, i32, vp, vp, i32]),
        "mg_num_levels": (i32, [vp, i32]),
        "mg_persistent_mark_timeout": (i32, [vp]),
        "mg_timing_enable": (i32, [vp, i32]),
        "mg_timing_read": (i32, [vp, i32, i32, ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        "mg_kernel_name": (ctypes.c_char_p, [i32]),
        "mg_graph_stats": (i32, [vp, ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int64)]),
        "mg_destroy": (i32, [vp]),
        "mg_status_string": (ctypes.c_char_p, [i32]),
        "mg_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def mg_status_string(status: int) -> str:
    return lib().mg_status_string(status).decode()


def mg_last_error() -> str:
    return lib().mg_last_error().decode()


def _check(status: int) -> int:
    if status != MG_OK:
        raise MGError(status, mg_last_error())
    return status


def _ptrs(addrs) -> ctypes.Array:
    arr = (vp * len(addrs))()
    for k, a in enumerate(addrs):
        arr[k] = int(a) if a else None
    return arr


def mg_options_default() -> mg_options:
    opt = mg_options()
    lib().mg_options_default(ctypes.byref(opt))
    return opt


def mg_setup(grids, opt: mg_options, stream: int = 0) -> int:
    """grids: sequence of (n, bc, pitch).  Returns the context handle."""
    arr = (mg_grid * len(grids))(*[mg_grid(int(n), int(bc), int(p)) for n, bc, p in grids])
    out = vp()
    _check(lib().mg_setup(arr, len(grids), ctypes.byref(opt), vp(stream or None),
                          ctypes.byref(out)))
    return out.value


def mg_vcycle(ctx: int, u, f, ncycles: int = 1, want_relres: bool = False):
    relres = (ctypes.c_double * len(u))() if want_relres else None
    _check(lib().mg_vcycle(vp(ctx), _ptrs(u), _ptrs(f), ncycles, relres))
    return list(relres) if want_relres else None


def mg_solve(ctx: int, u, f, rtol: float, max_cycles: int):
    """Returns (status, cycles, relres); raises only on argument/HIP errors."""
    cyc = (i32 * len(u))()
    rel = (ctypes.c_double * len(u))()
    st = lib().mg_solve(vp(ctx), _ptrs(u), _ptrs(f), float(rtol), int(max_cycles), cyc, rel)
    if st in (MG_ERR_INVALID_ARG, MG_ERR_UNSUPPORTED, MG_ERR_OOM, MG_ERR_HIP):
        raise MGError(st, mg_last_error())
    return st, list(cyc), list(rel)


def mg_solve_history(ctx: int, problem: int):
    """Per-cycle record of the last mg_solve: (prolongations, changes), the
    change NaN where the schedule does not measure it."""
    n = i32()
    _check(lib().mg_solve_history(vp(ctx), problem, 0, None, None, ctypes.byref(n)))
    ops = (i32 * max(n.value, 1))()
    dif = (ctypes.c_double * max(n.value, 1))()
    _check(lib().mg_solve_history(vp(ctx), problem, n.value, ops, dif, ctypes.byref(n)))
    return list(ops)[:n.value], list(dif)[:n.value]


def mg_ns_rhs(n: int, ux: int, uy: int, f: int, pitch: int, dtype: int, stream: int = 0) -> None:
    _check(lib().mg_ns_rhs(n, vp(ux), vp(uy), vp(f), pitch, dtype, vp(stream or None)))


def mg_ns_update(n: int, ux: int, uy: int, q: int, dt: float, ux_out: int, uy_out: int,
                 pitch: int, dtype: int, stream: int = 0) -> None:
    """q is mg_solve's solution for mg_ns_rhs's source (q = -p)."""
    _check(lib().mg_ns_update(n, vp(ux), vp(uy), vp(q), float(dt), vp(ux_out), vp(uy_out), pitch,
                              dtype, vp(stream or None)))


def mg_prolong(ctx: int, problem: int, coarse_level: int, kind: int, coarse: int, fine: int,
               dtype: int) -> None:
    _check(lib().mg_prolong(vp(ctx), problem, coarse_level, kind, vp(coarse), vp(fine), dtype))


def mg_prolong_noalloc(nc: int, bc: int, coarse: int, fine: int, dtype: int,
                       stream: int = 0) -> None:
    _check(lib().mg_prolong_noalloc(nc, bc, vp(coarse), vp(fine), dtype, vp(stream or None)))


def mg_twolevel_setup(n_unique: int, factor: int, batch: int, n_smooth: int = 20,
                      coarse_sweeps: int = 10, stream: int = 0) -> int:
    out = vp()
    _check(lib().mg_twolevel_setup(n_unique, factor, batch, n_smooth, coarse_sweeps,
                                   vp(stream or None), ctypes.byref(out)))
    return out.value


def mg_twolevel_smooth(ctx: int, p: int, f: int, sweeps: int) -> None:
    _check(lib().mg_twolevel_smooth(vp(ctx), vp(p), vp(f), sweeps))


def mg_twolevel_cycle(ctx: int, p: int, f: int, ncycles: int, batch: int | None = None):
    """Returns the last iteration's change per problem when batch is given."""
    ch = (ctypes.c_double * batch)() if batch else None
    _check(lib().mg_twolevel_cycle(vp(ctx), vp(p), vp(f), ncycles, ch))
    return list(ch) if batch else None


def mg_twolevel_solve(ctx: int, p: int, f: int, batch: int, n_pre: int, tol: float,
                      max_iter: int):
    """Returns (status, iterations, changes); raises only on argument/HIP errors."""
    it = (i32 * batch)()
    ch = (ctypes.c_double * batch)()
    st = lib().mg_twolevel_solve(vp(ctx), vp(p), vp(f), n_pre, float(tol), max_iter, it, ch)
    if st in (MG_ERR_INVALID_ARG, MG_ERR_UNSUPPORTED, MG_ERR_OOM, MG_ERR_HIP):
        raise MGError(st, mg_last_error())
    return st, list(it), list(ch)


def mg_twolevel_destroy(ctx: int) -> None:
    _check(lib().mg_twolevel_destroy(vp(ctx)))


def mg_relax(ctx: int, problem: int, level: int, u: int, f: int, colour: int, count: int,
             dtype: int) -> None:
    _check(lib().mg_relax(vp(ctx), problem, level, vp(u), vp(f), colour, count, dtype))


def mg_residual(ctx: int, problem: int, level: int, u: int, f: int, r: int, dtype: int) -> None:
    _check(lib().mg_residual(vp(ctx), problem, level, vp(u), vp(f), vp(r), dtype))


def mg_restrict(ctx: int, problem: int, level: int, r: int, fc: int, dtype: int) -> None:
    _check(lib().mg_restrict(vp(ctx), problem, level, vp(r), vp(fc), dtype))


def mg_coarse_solve(ctx: int, problem: int, f: int, u: int, dtype: int) -> None:
    _check(lib().mg_coarse_solve(vp(ctx), problem, vp(f), vp(u), dtype))


def mg_persistent_mark_timeout(ctx: int) -> None:
    _check(lib().mg_persistent_mark_timeout(vp(ctx)))


def mg_num_levels(ctx: int, problem: int) -> int:
    v = lib().mg_num_levels(vp(ctx), problem)
    if v < 0:
        raise MGError(v, mg_last_error())
    return v


MG_K_DOWN = 10
MG_K_UP = 11
MG_K_TAIL = 12
MG_K_PERSISTENT = 13
MG_K_CNN = 14
MG_K_CNN_AUX = 15
MG_K_PHASED = 16
MG_K_COUNT = 17
MG_SRCNN_WEIGHT_COUNT = 738432


def mg_timing_enable(ctx: int, enable: bool) -> None:
    _check(lib().mg_timing_enable(vp(ctx), int(bool(enable))))


def mg_timing_read(ctx: int, kind: int, level: int = -1):
    """Returns (launches, total_ms, algorithmic_bytes) for a kernel class."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(lib().mg_timing_read(vp(ctx), kind, level, ctypes.byref(n), ctypes.byref(ms),
                                ctypes.byref(by)))
    return n.value, ms.value, by.value


def mg_graph_stats(ctx: int):
    """Returns (captures, instantiations) of step graphs since setup."""
    c = ctypes.c_int64()
    i = ctypes.c_int64()
    _check(lib().mg_graph_stats(vp(ctx), ctypes.byref(c), ctypes.byref(i)))
    return c.value, i.value


def mg_kernel_name(kind: int) -> str:
    return lib().mg_kernel_name(kind).decode()


def mg_destroy(ctx: int) -> None:
    _check(lib().mg_destroy(vp(ctx)))
