"""ctypes binding of libxbar.so (include/xbar.h): argument marshalling only.

Every step of the solve runs in the library's HIP kernels; this module
only converts Python values and torch device tensors into the C ABI's
plain pointers and sizes.  It raises if the library is missing: there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxbar.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "xbar.h")

XBAR_OK = 0
XBAR_ERR_ARG = 1
XBAR_ERR_ALLOC = 2
XBAR_ERR_STATE = 3
XBAR_ERR_NOT_SPD = 4
XBAR_ERR_NO_CONVERGENCE = 5
XBAR_ERR_DEVICE = 6
XBAR_ERR_INPUT = 7

XBAR_FP64 = 0
XBAR_FP32_IR = 1
XBAR_BF16_IR = 2
XBAR_BF16_GMRES_IR = 3
PRECISIONS = {"fp64": XBAR_FP64, "fp32_ir": XBAR_FP32_IR, "bf16_ir": XBAR_BF16_IR, "bf16_gmres": XBAR_BF16_GMRES_IR}

XBAR_FACTOR_AUTO = 0
XBAR_FACTOR_GJ = 1
XBAR_FACTOR_NS = 2
XBAR_FACTOR_CHECKED = 3
FACTOR_METHODS = {"auto": XBAR_FACTOR_AUTO, "gj": XBAR_FACTOR_GJ, "ns": XBAR_FACTOR_NS,
                  "checked": XBAR_FACTOR_CHECKED}


class Geometry(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32),
                ("r_wl", ctypes.c_double), ("r_bl", ctypes.c_double),
                ("r_src", ctypes.c_double), ("r_sense", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("last_batch", ctypes.c_int32),
                ("ir_iters", ctypes.c_int32), ("device_error", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_int64), ("block", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("min_pivot", ctypes.c_double),
                ("max_backward_err", ctypes.c_double), ("factor_slots_used", ctypes.c_int32),
                ("factor_slots_launched", ctypes.c_int32)]


class TileClass(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("count", ctypes.c_int32), ("B", ctypes.c_int32),
                ("method", ctypes.c_int32), ("block", ctypes.c_int32), ("split", ctypes.c_int32),
                ("transpose", ctypes.c_int32)]


XBAR_TILE_ONE_WG = 0
XBAR_TILE_PIPELINE = 1


class Timing(ctypes.Structure):
    _fields_ = [("condense_ms", ctypes.c_double), ("condense_launches", ctypes.c_int64),
                ("factor_ms", ctypes.c_double), ("factor_launches", ctypes.c_int64),
                ("sweep_ms", ctypes.c_double), ("sweep_launches", ctypes.c_int64),
                ("recover_ms", ctypes.c_double), ("recover_launches", ctypes.c_int64),
                ("ir_sweep_ms", ctypes.c_double), ("ir_sweep_launches", ctypes.c_int64),
                ("residual_ms", ctypes.c_double), ("residual_launches", ctypes.c_int64)]


class XbarError(RuntimeError):
    def __init__(self, call: str, status: int):
        self.status = status
        super().__init__(f"{call} -> {status_string(status)}")


_lib = None


def lib() -> ctypes.CDLL:
    """Load libxbar.so (build it first with paper_2410_19993_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2410_19993_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.xbar_create.argtypes = [ctypes.POINTER(Geometry), ctypes.c_int, ctypes.c_int32,
                                  ctypes.c_double, ctypes.c_int32, vp, ctypes.POINTER(vp)]
        L.xbar_create_ordered.argtypes = [ctypes.POINTER(Geometry), ctypes.c_int, ctypes.c_int32,
                                          ctypes.c_double, ctypes.c_int32, vp, ctypes.c_int32, ctypes.POINTER(vp)]
        L.xbar_assemble.argtypes = [vp, vp]
        L.xbar_factor.argtypes = [vp]
        L.xbar_solve_batch.argtypes = [vp, vp, ctypes.c_int32, vp]
        L.xbar_currents.argtypes = [vp, vp]
        L.xbar_transfer.argtypes = [vp, vp]
        L.xbar_transfer_apply.argtypes = [vp, vp, vp, ctypes.c_int32, vp]
        L.xbar_tiles_currents.argtypes = [ctypes.POINTER(Geometry), ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp]
        L.xbar_get_info.argtypes = [vp, ctypes.POINTER(Info)]
        L.xbar_tiles_create.argtypes = [ctypes.POINTER(TileClass), ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int32, vp, ctypes.POINTER(vp)]
        L.xbar_tiles_run.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp)]
        L.xbar_tiles_workspace_bytes.argtypes = [vp]
        L.xbar_tiles_workspace_bytes.restype = ctypes.c_int64
        L.xbar_tiles_destroy.argtypes = [vp]
        L.xbar_destroy.argtypes = [vp]
        L.xbar_set_timing.argtypes = [vp, ctypes.c_int32]
        L.xbar_set_factor_method.argtypes = [vp, ctypes.c_int]
        L.xbar_set_diagnostics.argtypes = [vp, ctypes.c_int32]
        L.xbar_debug_shift_pivots.argtypes = [vp, ctypes.c_double]
        L.xbar_get_timing.argtypes = [vp, ctypes.POINTER(Timing), ctypes.c_int32]
        L.xbar_status_string.argtypes = [ctypes.c_int]
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.xbar_sg_features.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp]
        L.xbar_sg_conv_forward.argtypes = [i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp]
        L.xbar_sg_conv_backward_data.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp]
        L.xbar_sg_conv_backward_weight.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, i64, vp]
        L.xbar_sg_conv_backward_weight_noalloc.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp]
        L.xbar_sg_conv_forward_bf16.argtypes = [i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp]
        L.xbar_sg_conv_backward_data_bf16.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp]
        L.xbar_sg_conv_backward_weight_bf16.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, i64, vp]
        L.xbar_sg_workspace_floats.argtypes = [i32, i32]
        L.xbar_sg_workspace_floats.restype = i64
        L.xbar_sg_readout_loss.argtypes = [i32, i32, i32, vp, vp, f64, vp, vp, vp]
        L.xbar_sg_adam.argtypes = [i64, vp, vp, vp, vp, f64, f64, f64, f64, i32, vp]
        L.xbar_sg_predict.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp]
        L.xbar_sg_targets.argtypes = [i32, i32, vp, vp, vp, vp]
        L.xbar_sg_calib_ratios.argtypes = [i32, i32, vp, vp, vp, vp, vp]
        L.xbar_sg_route.argtypes = [i32, i32, i32, vp, vp, vp, vp, f64, f64, vp, vp]
        L.xbar_status_string.restype = ctypes.c_char_p
        for f in ("xbar_create", "xbar_create_ordered", "xbar_assemble", "xbar_factor", "xbar_solve_batch",
                  "xbar_currents", "xbar_get_info", "xbar_destroy", "xbar_set_timing",
                  "xbar_get_timing", "xbar_set_factor_method", "xbar_set_diagnostics",
                  "xbar_debug_shift_pivots", "xbar_transfer",
                  "xbar_transfer_apply", "xbar_tiles_currents", "xbar_tiles_create", "xbar_tiles_run",
                  "xbar_tiles_destroy", "xbar_sg_features", "xbar_sg_conv_forward",
                  "xbar_sg_conv_backward_data", "xbar_sg_conv_backward_weight",
                  "xbar_sg_conv_backward_weight_noalloc", "xbar_sg_conv_forward_bf16",
                  "xbar_sg_conv_backward_data_bf16", "xbar_sg_conv_backward_weight_bf16", "xbar_sg_readout_loss",
                  "xbar_sg_adam", "xbar_sg_predict", "xbar_sg_targets", "xbar_sg_calib_ratios", "xbar_sg_route"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of every function the public header declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(xbar_\w+)\s*\(", text, re.M)))


def status_string(s: int) -> str:
    return lib().xbar_status_string(int(s)).decode()


def _ptr(t):
    """Device pointer of a torch tensor (or None -> NULL)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _check(call, st):
    if st != XBAR_OK:
        raise XbarError(call, st)


ORDERINGS = {"auto": 0, "rows": 1, "smaller": 2}


def xbar_create(geom: Geometry, precision: int, max_batch: int, ir_tol: float = 0.0,
                ir_max_iter: int = 0, stream: int | None = None, ordering: int = 0) -> ctypes.c_void_p:
    plan = ctypes.c_void_p()
    st = lib().xbar_create_ordered(ctypes.byref(geom), int(precision), int(max_batch), float(ir_tol),
                                   int(ir_max_iter), ctypes.c_void_p(stream or 0), int(ordering),
                                   ctypes.byref(plan))
    _check("xbar_create_ordered", st)
    return plan


def xbar_assemble(plan, G) -> None:
    _check("xbar_assemble", lib().xbar_assemble(plan, _ptr(G)))


def xbar_factor(plan) -> None:
    _check("xbar_factor", lib().xbar_factor(plan))


def xbar_solve_batch(plan, V, B: int, node_v=None) -> None:
    _check("xbar_solve_batch", lib().xbar_solve_batch(plan, _ptr(V), int(B), _ptr(node_v)))


def xbar_currents(plan, I) -> None:
    _check("xbar_currents", lib().xbar_currents(plan, _ptr(I)))


def xbar_transfer(plan, T) -> None:
    _check("xbar_transfer", lib().xbar_transfer(plan, _ptr(T)))


def xbar_transfer_apply(plan, T, V, B: int, I) -> None:
    _check("xbar_transfer_apply", lib().xbar_transfer_apply(plan, _ptr(T), _ptr(V), int(B), _ptr(I)))


def xbar_tiles_currents(geom: Geometry, T: int, B: int, G, V, I, stream: int | None = None) -> None:
    _check("xbar_tiles_currents", lib().xbar_tiles_currents(ctypes.byref(geom), int(T), int(B), _ptr(G), _ptr(V),
                                                            _ptr(I), ctypes.c_void_p(stream or 0)))


def xbar_tiles_create(classes, r_wl, r_bl, r_src, r_sense, streams: int, stream: int | None = None):
    arr = (TileClass * len(classes))(*classes)
    t = ctypes.c_void_p()
    _check("xbar_tiles_create", lib().xbar_tiles_create(arr, len(classes), float(r_wl), float(r_bl), float(r_src),
                                                        float(r_sense), int(streams), ctypes.c_void_p(stream or 0),
                                                        ctypes.byref(t)))
    return t


def xbar_tiles_run(t, Gs, Vs, Is) -> None:
    k = len(Gs)
    G = (ctypes.c_void_p * k)(*[g.data_ptr() for g in Gs])
    V = (ctypes.c_void_p * k)(*[v.data_ptr() for v in Vs])
    I = (ctypes.c_void_p * k)(*[i.data_ptr() for i in Is])
    _check("xbar_tiles_run", lib().xbar_tiles_run(t, G, V, I))


def xbar_tiles_workspace_bytes(t) -> int:
    return int(lib().xbar_tiles_workspace_bytes(t))


def xbar_tiles_destroy(t) -> None:
    _check("xbar_tiles_destroy", lib().xbar_tiles_destroy(t))


def xbar_get_info(plan) -> tuple[int, Info]:
    info = Info()
    st = lib().xbar_get_info(plan, ctypes.byref(info))
    return st, info


def xbar_set_factor_method(plan, method: int) -> None:
    _check("xbar_set_factor_method", lib().xbar_set_factor_method(plan, int(method)))


def xbar_set_diagnostics(plan, enable: bool) -> None:
    _check("xbar_set_diagnostics", lib().xbar_set_diagnostics(plan, 1 if enable else 0))


def xbar_debug_shift_pivots(plan, shift: float) -> None:
    _check("xbar_debug_shift_pivots", lib().xbar_debug_shift_pivots(plan, float(shift)))


def xbar_set_timing(plan, enable: bool) -> None:
    _check("xbar_set_timing", lib().xbar_set_timing(plan, 1 if enable else 0))


def xbar_get_timing(plan, reset: bool = False) -> Timing:
    t = Timing()
    _check("xbar_get_timing", lib().xbar_get_timing(plan, ctypes.byref(t), 1 if reset else 0))
    return t


def xbar_destroy(plan) -> None:
    _check("xbar_destroy", lib().xbar_destroy(plan))


# ---- learned current surrogate (argument marshalling only) -------------------------

def _s(stream):
    return ctypes.c_void_p(stream or 0)


def xbar_sg_features(B, m, n, G, V, r, X, stream=None) -> None:
    _check("xbar_sg_features", lib().xbar_sg_features(B, m, n, _ptr(G), _ptr(V), _ptr(r), _ptr(X), _s(stream)))


def _sfx(bf16: bool) -> str:
    return "_bf16" if bf16 else ""


def xbar_sg_conv_forward(B, H, W, C, O, relu, x, w, b, y, stream=None, bf16=False) -> None:
    name = "xbar_sg_conv_forward" + _sfx(bf16)
    _check(name, getattr(lib(), name)(B, H, W, C, O, int(bool(relu)), _ptr(x), _ptr(w), _ptr(b), _ptr(y), _s(stream)))


def xbar_sg_conv_backward_data(B, H, W, C, O, gy, ymask, w, gx, xmask=None, stream=None, bf16=False) -> None:
    name = "xbar_sg_conv_backward_data" + _sfx(bf16)
    _check(name, getattr(lib(), name)(B, H, W, C, O, _ptr(gy), _ptr(ymask), _ptr(w), _ptr(xmask), _ptr(gx),
                                      _s(stream)))


def xbar_sg_conv_backward_weight(B, H, W, C, O, x, gy, ymask, gw, gb, work, stream=None, bf16=False) -> None:
    name = "xbar_sg_conv_backward_weight" + _sfx(bf16)
    _check(name, getattr(lib(), name)(B, H, W, C, O, _ptr(x), _ptr(gy), _ptr(ymask), _ptr(gw), _ptr(gb),
                                      _ptr(work), int(work.numel()), _s(stream)))


def xbar_sg_conv_backward_weight_noalloc(B, H, W, C, O, x, gy, ymask, gw, gb, stream=None) -> None:
    _check("xbar_sg_conv_backward_weight_noalloc",
           lib().xbar_sg_conv_backward_weight_noalloc(B, H, W, C, O, _ptr(x), _ptr(gy), _ptr(ymask), _ptr(gw),
                                                      _ptr(gb), _s(stream)))


def xbar_sg_workspace_floats(C, O) -> int:
    return int(lib().xbar_sg_workspace_floats(C, O))


def xbar_sg_readout_loss(B, m, n, Y, delta, lam, gY, err2, stream=None) -> None:
    _check("xbar_sg_readout_loss", lib().xbar_sg_readout_loss(B, m, n, _ptr(Y), _ptr(delta), float(lam), _ptr(gY),
                                                              _ptr(err2), _s(stream)))


def xbar_sg_adam(p, g, m1, m2, lr, b1, b2, eps, t, stream=None) -> None:
    _check("xbar_sg_adam", lib().xbar_sg_adam(int(p.numel()), _ptr(p), _ptr(g), _ptr(m1), _ptr(m2), float(lr),
                                              float(b1), float(b2), float(eps), int(t), _s(stream)))


def xbar_sg_predict(B, m, n, Y, G, V, I, est=None, stream=None) -> None:
    _check("xbar_sg_predict", lib().xbar_sg_predict(B, m, n, _ptr(Y), _ptr(G), _ptr(V), _ptr(I), _ptr(est),
                                                    _s(stream)))


def xbar_sg_targets(S, n, I, I0, delta, stream=None) -> None:
    _check("xbar_sg_targets", lib().xbar_sg_targets(S, n, _ptr(I), _ptr(I0), _ptr(delta), _s(stream)))


def xbar_sg_calib_ratios(B, n, Ip, I, est, ratio, stream=None) -> None:
    _check("xbar_sg_calib_ratios", lib().xbar_sg_calib_ratios(B, n, _ptr(Ip), _ptr(I), _ptr(est), _ptr(ratio),
                                                              _s(stream)))


def xbar_sg_route(B, m, n, G, V, I, est, kappa, tol, flag, stream=None) -> None:
    _check("xbar_sg_route", lib().xbar_sg_route(B, m, n, _ptr(G), _ptr(V), _ptr(I), _ptr(est), float(kappa),
                                                float(tol), _ptr(flag), _s(stream)))
