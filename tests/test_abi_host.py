"""C-ABI checks that need no GPU: the library loads, exports every function
the header declares, and rejects bad arguments on the host before touching a
device (include/xbar.h)."""
import ctypes
import math

import pytest

from paper_2410_19993_amd import _lib

EXPECTED = ["xbar_assemble", "xbar_create", "xbar_create_ordered", "xbar_currents",
            "xbar_debug_shift_pivots", "xbar_destroy", "xbar_factor", "xbar_get_info", "xbar_get_timing",
            "xbar_set_diagnostics", "xbar_set_factor_method", "xbar_set_timing", "xbar_sg_adam",
            "xbar_sg_calib_ratios", "xbar_sg_conv_backward_data", "xbar_sg_conv_backward_data_bf16",
            "xbar_sg_conv_backward_weight", "xbar_sg_conv_backward_weight_bf16",
            "xbar_sg_conv_backward_weight_noalloc", "xbar_sg_conv_forward", "xbar_sg_conv_forward_bf16",
            "xbar_sg_features", "xbar_sg_predict", "xbar_sg_readout_loss", "xbar_sg_route",
            "xbar_sg_targets", "xbar_sg_workspace_floats", "xbar_solve_batch", "xbar_status_string",
            "xbar_tiles_create", "xbar_tiles_currents", "xbar_tiles_destroy", "xbar_tiles_run",
            "xbar_tiles_workspace_bytes", "xbar_transfer", "xbar_transfer_apply"]


def _gpu_visible():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_header_declares_the_boundary():
    assert _lib.header_functions() == EXPECTED


def test_library_exports_every_header_symbol():
    L = _lib.lib()
    for name in _lib.header_functions():
        assert hasattr(L, name), name


def test_status_strings():
    names = {0: "XBAR_OK", 1: "XBAR_ERR_ARG", 2: "XBAR_ERR_ALLOC", 3: "XBAR_ERR_STATE",
             4: "XBAR_ERR_NOT_SPD", 5: "XBAR_ERR_NO_CONVERGENCE", 6: "XBAR_ERR_DEVICE",
             7: "XBAR_ERR_INPUT"}
    for k, v in names.items():
        assert _lib.status_string(k) == v
    assert _lib.status_string(99) == "XBAR_UNKNOWN_STATUS"


def _create(geom, prec=0, max_batch=8, tol=0.0, iters=0):
    plan = ctypes.c_void_p()
    st = _lib.lib().xbar_create(ctypes.byref(geom), prec, max_batch, tol, iters, None,
                                ctypes.byref(plan))
    return st, plan


GOOD = dict(m=4, n=4, r_wl=1.0, r_bl=1.0, r_src=50.0, r_sense=50.0)


@pytest.mark.parametrize("field,value", [
    ("m", 0), ("n", 0), ("m", -3), ("r_wl", 0.0), ("r_bl", -1.0),
    ("r_src", math.inf), ("r_sense", math.nan), ("r_wl", math.nan)])
def test_create_rejects_bad_geometry(field, value):
    kw = dict(GOOD)
    kw[field] = value
    st, plan = _create(_lib.Geometry(**kw))
    assert st == _lib.XBAR_ERR_ARG and not plan.value


@pytest.mark.parametrize("m,n,ordering", [(4, 4, 3), (4, 4, -1), (4, 600, 1)])
def test_create_ordered_rejects_bad_orderings(m, n, ordering):
    """Unknown orderings, and row blocks along the word lines when n > XBAR_MAX_N."""
    geom = _lib.Geometry(**dict(GOOD, m=m, n=n))
    plan = ctypes.c_void_p()
    st = _lib.lib().xbar_create_ordered(ctypes.byref(geom), 0, 8, 0.0, 0, None, ordering, ctypes.byref(plan))
    assert st == _lib.XBAR_ERR_ARG and not plan.value


@pytest.mark.parametrize("m,n", [(513, 513), (600, 1000), (1000, 600)])
def test_create_rejects_both_sides_above_the_block_limit(m, n):
    """Row blocks take the smaller side, which must be <= XBAR_MAX_N (512); one side
    alone may be longer (reciprocal ordering when the columns are)."""
    kw = dict(GOOD, m=m, n=n)
    st, plan = _create(_lib.Geometry(**kw))
    assert st == _lib.XBAR_ERR_ARG and not plan.value


@pytest.mark.parametrize("prec,max_batch,tol,iters", [
    (7, 8, 0.0, 0), (-1, 8, 0.0, 0), (4, 8, 0.0, 0), (0, 0, 0.0, 0), (0, -5, 0.0, 0),
    (0, 8, -1.0, 0), (0, 8, math.nan, 0), (0, 8, 1.5, 0), (0, 8, 0.0, -1), (0, 8, 0.0, 1000)])
def test_create_rejects_bad_options(prec, max_batch, tol, iters):
    st, plan = _create(_lib.Geometry(**GOOD), prec, max_batch, tol, iters)
    assert st == _lib.XBAR_ERR_ARG and not plan.value


def test_create_null_pointers():
    L = _lib.lib()
    plan = ctypes.c_void_p()
    assert L.xbar_create(None, 0, 8, 0.0, 0, None, ctypes.byref(plan)) == _lib.XBAR_ERR_ARG
    g = _lib.Geometry(**GOOD)
    assert L.xbar_create(ctypes.byref(g), 0, 8, 0.0, 0, None, None) == _lib.XBAR_ERR_ARG


def test_null_plan_calls():
    L = _lib.lib()
    assert L.xbar_assemble(None, None) == _lib.XBAR_ERR_ARG
    assert L.xbar_factor(None) == _lib.XBAR_ERR_ARG
    assert L.xbar_solve_batch(None, None, 1, None) == _lib.XBAR_ERR_ARG
    assert L.xbar_currents(None, None) == _lib.XBAR_ERR_ARG
    assert L.xbar_transfer(None, None) == _lib.XBAR_ERR_ARG
    assert L.xbar_transfer_apply(None, None, None, 1, None) == _lib.XBAR_ERR_ARG
    info = _lib.Info()
    assert L.xbar_get_info(None, ctypes.byref(info)) == _lib.XBAR_ERR_ARG
    assert L.xbar_destroy(None) == _lib.XBAR_OK
    assert L.xbar_set_timing(None, 1) == _lib.XBAR_ERR_ARG
    assert L.xbar_set_factor_method(None, 0) == _lib.XBAR_ERR_ARG
    assert L.xbar_get_timing(None, ctypes.byref(_lib.Timing()), 0) == _lib.XBAR_ERR_ARG
    assert L.xbar_set_diagnostics(None, 1) == _lib.XBAR_ERR_ARG
    assert L.xbar_debug_shift_pivots(None, 1.0) == _lib.XBAR_ERR_ARG


def test_info_struct_matches_the_header():
    """The binding's xbar_info mirrors the header's field order and types."""
    import re
    text = open(_lib.HEADER).read()
    body = text[text.index("typedef struct {\n    int32_t state;"):]
    body = body[:body.index("} xbar_info;")]
    fields = re.findall(r"^\s*(int32_t|int64_t|double)\s+(\w+);", body, re.M)
    ctype = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "double": ctypes.c_double}
    assert [(n, ctype[t]) for t, n in fields] == list(_lib.Info._fields_)


@pytest.mark.skipif(_gpu_visible(), reason="checks the GPU-less path")
def test_create_without_device_reports_device_error():
    st, plan = _create(_lib.Geometry(**GOOD))
    assert st == _lib.XBAR_ERR_DEVICE and not plan.value


@pytest.mark.parametrize("field,value,T,B", [
    ("n", 65, 2, 4), ("n", 0, 2, 4), ("m", 0, 2, 4), ("r_wl", 0.0, 2, 4), ("r_sense", math.inf, 2, 4),
    ("n", 8, 0, 4), ("n", 8, 2, 0), ("n", 8, 2, 257)])
def test_tiles_rejects_bad_arguments(field, value, T, B):
    """Host checks of xbar_tiles_currents come before any device call (no GPU needed)."""
    kw = dict(GOOD)
    kw[field] = value
    g = _lib.Geometry(**kw)
    buf = (ctypes.c_double * 4096)()
    L = _lib.lib()
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert L.xbar_tiles_currents(ctypes.byref(g), T, B, p, p, None, None) == _lib.XBAR_ERR_ARG
    assert L.xbar_tiles_currents(None, 1, 1, p, p, p, None) == _lib.XBAR_ERR_ARG


def test_tiles_rejects_overlapping_output():
    g = _lib.Geometry(**GOOD)                      # 4 x 4
    buf = (ctypes.c_double * 4096)()
    base = ctypes.addressof(buf)
    G, V = ctypes.c_void_p(base), ctypes.c_void_p(base + 8 * 1024)
    L = _lib.lib()
    # I over G, then over V: rejected before any device call
    assert L.xbar_tiles_currents(ctypes.byref(g), 2, 3, G, V, ctypes.c_void_p(base + 8 * 16), None) == _lib.XBAR_ERR_ARG
    assert L.xbar_tiles_currents(ctypes.byref(g), 2, 3, G, V, ctypes.c_void_p(base + 8 * 1030), None) == _lib.XBAR_ERR_ARG


def test_surrogate_calls_reject_bad_arguments():
    """Host checks of the surrogate calls come before any device call (no GPU needed)."""
    L = _lib.lib()
    buf = (ctypes.c_float * 65536)()
    base = ctypes.addressof(buf)
    a, b, c, d = (ctypes.c_void_p(base + k * 65536) for k in range(4))
    E = _lib.XBAR_ERR_ARG
    assert L.xbar_sg_workspace_floats(32, 32) == 512 * (32 * 32 * 9 + 32)
    assert L.xbar_sg_workspace_floats(33, 1) == -1 and L.xbar_sg_workspace_floats(1, 0) == -1
    # channels out of range, empty shapes, NULL pointers
    assert L.xbar_sg_conv_forward(1, 4, 4, 33, 2, 1, a, b, c, d, None) == E
    assert L.xbar_sg_conv_forward(1, 4, 4, 2, 0, 1, a, b, c, d, None) == E
    assert L.xbar_sg_conv_forward(0, 4, 4, 2, 2, 1, a, b, c, d, None) == E
    assert L.xbar_sg_conv_forward(1, 4, 0, 2, 2, 1, a, b, c, d, None) == E
    assert L.xbar_sg_conv_forward(1, 4, 4, 2, 2, 1, None, b, c, d, None) == E
    assert L.xbar_sg_conv_backward_data(1, 4, 4, 2, 2, a, None, b, None, None, None) == E
    assert L.xbar_sg_features(1, 0, 4, a, b, c, d, None) == E
    assert L.xbar_sg_features(1, 4, 2049, a, b, c, d, None) == E
    assert L.xbar_sg_readout_loss(1, 4, 4, a, b, 0.1, None, d, None) == E
    assert L.xbar_sg_readout_loss(1, 4, 4, a, b, -1.0, c, d, None) == E        # lam < 0
    assert L.xbar_sg_predict(1, 4, 4, a, b, c, None, None, None) == E
    # outputs overlapping inputs: y over x, gx over gy, I over Y
    assert L.xbar_sg_conv_forward(1, 4, 4, 2, 2, 1, a, b, c, ctypes.c_void_p(base + 16), None) == E
    assert L.xbar_sg_conv_backward_data(1, 4, 4, 2, 2, a, None, b, None, ctypes.c_void_p(base + 64), None) == E
    assert L.xbar_sg_conv_backward_data(1, 4, 4, 2, 2, a, None, b, ctypes.c_void_p(base + 3 * 65536 + 8), d,
                                        None) == E                                # gx over xmask
    assert L.xbar_sg_predict(1, 4, 4, a, b, c, ctypes.c_void_p(base + 8), None, None) == E
    assert L.xbar_sg_predict(1, 4, 4, a, b, c, d, ctypes.c_void_p(base + 3 * 65536 + 8), None) == E  # est over I
    # weight gradient: workspace too small, gw over gb
    ws = L.xbar_sg_workspace_floats(2, 2)
    assert L.xbar_sg_conv_backward_weight(1, 4, 4, 2, 2, a, b, None, c, d, ctypes.c_void_p(base + 4 * 65536 * 8),
                                          1, None) == E
    assert L.xbar_sg_conv_backward_weight(1, 4, 4, 2, 2, a, b, None, c, ctypes.c_void_p(base + 2 * 65536 + 8),
                                          ctypes.c_void_p(base + 4 * 65536 * 8), ws, None) == E
    # allocation-free weight gradient: the same host checks, and gw over gb
    assert L.xbar_sg_conv_backward_weight_noalloc(1, 4, 4, 33, 2, a, b, None, c, d, None) == E
    assert L.xbar_sg_conv_backward_weight_noalloc(0, 4, 4, 2, 2, a, b, None, c, d, None) == E
    assert L.xbar_sg_conv_backward_weight_noalloc(1, 4, 4, 2, 2, None, b, None, c, d, None) == E
    assert L.xbar_sg_conv_backward_weight_noalloc(1, 4, 4, 2, 2, a, b, None, c, ctypes.c_void_p(base + 2 * 65536 + 8),
                                                  None) == E
    # Adam: step 0, lr <= 0, beta outside [0, 1)
    assert L.xbar_sg_adam(4, a, b, c, d, 1e-3, 0.9, 0.999, 1e-8, 0, None) == E
    assert L.xbar_sg_adam(4, a, b, c, d, 0.0, 0.9, 0.999, 1e-8, 1, None) == E
    assert L.xbar_sg_adam(4, a, b, c, d, 1e-3, 1.0, 0.999, 1e-8, 1, None) == E
