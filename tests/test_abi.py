"""C-ABI checks that need no GPU: the library loads, exports every function
that include/mg.h declares, and rejects bad arguments before touching a
device."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mg.h")


def declared_functions():
    text = open(HEADER).read()
    return re.findall(r"^MG_API\s+[\w\s\*]*?\b(mg_\w+)\s*\(", text, re.M)


@pytest.fixture(scope="module")
def B():
    from paper_2403_07936_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libmg355.so not built (run __graft_entry__.build())")
    binding.lib()
    return binding


def test_header_declares_the_boundary():
    names = set(declared_functions())
    for required in ("mg_setup", "mg_vcycle", "mg_solve", "mg_prolong", "mg_destroy",
                     "mg_status_string", "mg_relax", "mg_residual", "mg_restrict",
                     "mg_coarse_solve", "mg_options_default", "mg_last_error",
                     "mg_num_levels"):
        assert required in names


def test_library_exports_every_declared_symbol(B):
    import ctypes
    L = ctypes.CDLL(B.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings(B):
    for st in range(0, -9, -1):
        s = B.mg_status_string(st)
        assert s and s != "unknown status"
    assert B.mg_status_string(-99) == "unknown status"


def test_options_default(B):
    o = B.mg_options_default()
    assert (o.precision, o.nu_pre, o.nu_post, o.inner_cycles, o.use_graph) == (0, 2, 2, 1, 1)


@pytest.mark.parametrize("grids,field,value", [
    ([(6, 0, 0)], None, None),          # n - 1 not 4 * 2^k
    ([(3, 0, 0)], None, None),          # too small
    ([(65, 2, 0)], None, None),         # bad boundary condition
    ([(65, 0, 10)], None, None),        # pitch < n
    ([(65, 0, 0)], "nu_pre", 9),
    ([(65, 0, 0)], "inner_cycles", 0),
    ([(65, 0, 0)], "precision", 7),
    ([(65, 0, 0)], "n_gan", -1.0),      # negative schedule ratio
    ([(65, 0, 0)], "s_thres", -1.0),    # negative switch threshold
    ([(65, 1, 0)], "n_gan", 1.0),       # schedule without the network prolongation
])
def test_setup_rejects_bad_arguments_before_device_use(B, grids, field, value):
    o = B.mg_options_default()
    if field:
        setattr(o, field, value)
    with pytest.raises(B.MGError) as ei:
        B.mg_setup(grids, o, 0)
    assert ei.value.status == B.MG_ERR_INVALID_ARG
    assert B.mg_last_error()


def test_setup_srcnn_on_dirichlet_is_unsupported(B):
    o = B.mg_options_default()
    o.prolong = B.MG_PROLONG_SRCNN
    with pytest.raises(B.MGError) as ei:
        B.mg_setup([(65, 0, 0)], o, 0)
    assert ei.value.status == B.MG_ERR_UNSUPPORTED


def test_null_context_calls(B):
    B.mg_destroy(0)
    with pytest.raises(B.MGError) as ei:
        B.mg_vcycle(0, [1], [1], 1)
    assert ei.value.status == B.MG_ERR_INVALID_ARG
    with pytest.raises(B.MGError):
        B.mg_num_levels(0, 0)
    with pytest.raises(B.MGError) as ei:
        B.mg_solve_history(0, 0)
    assert ei.value.status == B.MG_ERR_INVALID_ARG
    with pytest.raises(B.MGError) as ei:
        B.mg_graph_stats(0)
    assert ei.value.status == B.MG_ERR_INVALID_ARG


def test_options_default_schedule_is_off(B):
    o = B.mg_options_default()
    assert (o.n_gan, o.s_thres, o.cnn_max_ratio, o.cnn_min_relres) == (0.0, 0.0, 0.5, 1e-7)


@pytest.mark.parametrize("nc,bc,dtype,status", [
    (2049, 0, 0, -2),   # above the static scratch's 1025
    (6, 0, 0, -1),      # not 4 * 2^k + 1
    (129, 2, 0, -1),    # bad boundary condition
    (129, 0, 5, -1),    # bad dtype
])
def test_prolong_noalloc_rejects_before_any_device_call(B, nc, bc, dtype, status):
    """Argument checks of mg_prolong_noalloc run on the host, before any HIP
    call (the device pointers below are never touched)."""
    st = B.lib().mg_prolong_noalloc(nc, bc, 0x1000, 0x2000, dtype, None)
    assert st == status
    assert B.mg_last_error()


def test_prolong_noalloc_rejects_null_arrays(B):
    assert B.lib().mg_prolong_noalloc(129, 0, None, 0x2000, 0, None) == -1
    assert B.lib().mg_prolong_noalloc(129, 0, 0x1000, 0x1000, 0, None) == -1


@pytest.mark.parametrize("N,F,batch,ns,cs,status", [
    (96, 8, 1, 20, 10, -2),     # unique side not 64, 128 or 192
    (192, 3, 1, 20, 10, -1),    # factor not a power of two
    (192, 64, 1, 20, 10, -1),   # factor above 32
    (192, 16, 0, 20, 10, -1),   # empty batch
    (192, 16, 1, -1, 10, -1),   # negative sweep count
])
def test_twolevel_setup_rejects_before_any_device_call(B, N, F, batch, ns, cs, status):
    import ctypes
    out = ctypes.c_void_p()
    st = B.lib().mg_twolevel_setup(N, F, batch, ns, cs, None, ctypes.byref(out))
    assert st == status and not out.value
    assert B.mg_last_error()


def test_twolevel_calls_reject_a_null_context(B):
    assert B.lib().mg_twolevel_smooth(None, 0x1000, 0x2000, 1) == -1
    assert B.lib().mg_twolevel_cycle(None, 0x1000, 0x2000, 1, None) == -1
    assert B.lib().mg_twolevel_destroy(None) == 0
