"""MI355X (gfx950) crossbar nodal solver: Python front end of libxbar.so.

The names mirror the C ABI of include/xbar.h; torch supplies device memory
and the HIP stream.  All arithmetic runs in the library's HIP kernels.
"""
from __future__ import annotations

from . import _lib
from ._lib import (FACTOR_METHODS, PRECISIONS, XBAR_BF16_GMRES_IR, XBAR_BF16_IR, XBAR_FP32_IR, XBAR_FP64,  # noqa: F401
                   Geometry, XbarError, status_string)

__all__ = ["Plan", "PlanLanes", "TileBatch", "TileConfig", "solve", "tiles_currents", "Geometry", "XbarError",
           "PRECISIONS", "status_string"]


def _torch():
    import torch
    return torch


def _check_tensor(name, t, shape):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA/HIP tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Plan:
    """One crossbar geometry: xbar_create ... xbar_destroy."""

    def __init__(self, m: int, n: int, r_wl: float, r_bl: float, r_src: float = 50.0,
                 r_sense: float = 50.0, precision: str = "fp64", max_batch: int = 1024,
                 ir_tol: float = 0.0, ir_max_iter: int = 0, stream=None, factor_method: str = "auto",
                 ordering: str = "auto"):
        torch = _torch()
        self.m, self.n = int(m), int(n)
        self.max_batch = int(max_batch)
        self.geom = Geometry(self.m, self.n, float(r_wl), float(r_bl), float(r_src), float(r_sense))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.precision = precision
        self._plan = _lib.xbar_create(self.geom, PRECISIONS[precision], self.max_batch, ir_tol,
                                      ir_max_iter, self.stream.cuda_stream, _lib.ORDERINGS[ordering])
        self._B = 0
        _lib.xbar_set_factor_method(self._plan, FACTOR_METHODS[factor_method])

    def assemble(self, G) -> None:
        _check_tensor("G", G, (self.m, self.n))
        _lib.xbar_assemble(self._plan, G)

    def factor(self) -> None:
        _lib.xbar_factor(self._plan)

    def solve_batch(self, V, node_v=None) -> None:
        B = int(V.shape[0])
        _check_tensor("V", V, (B, self.m))
        if node_v is not None:
            _check_tensor("node_v", node_v, (B, 2 * self.m * self.n))
        _lib.xbar_solve_batch(self._plan, V, B, node_v)
        self._B = B

    def currents(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty((self._B, self.n), dtype=torch.float64, device="cuda")
        _check_tensor("I", out, (self._B, self.n))
        _lib.xbar_currents(self._plan, out)
        return out

    def transfer(self, out=None):
        """T [m][n]: output currents per unit volt on each word line (xbar_transfer)."""
        torch = _torch()
        if out is None:
            out = torch.empty((self.m, self.n), dtype=torch.float64, device="cuda")
        _check_tensor("T", out, (self.m, self.n))
        _lib.xbar_transfer(self._plan, out)
        self._B = 0
        return out

    def transfer_apply(self, T, V, out=None):
        """I = V T for any batch V [B][m] (xbar_transfer_apply)."""
        torch = _torch()
        B = int(V.shape[0])
        _check_tensor("T", T, (self.m, self.n))
        _check_tensor("V", V, (B, self.m))
        if out is None:
            out = torch.empty((B, self.n), dtype=torch.float64, device="cuda")
        _check_tensor("I", out, (B, self.n))
        _lib.xbar_transfer_apply(self._plan, T, V, B, out)
        return out

    def set_diagnostics(self, enable: bool = True) -> None:
        """Measure the backward error of every batch solved with node voltages
        (xbar_set_diagnostics); read it from info()[1].max_backward_err."""
        _lib.xbar_set_diagnostics(self._plan, enable)

    def debug_shift_pivots(self, shift: float) -> None:
        """Test hook (xbar_debug_shift_pivots): subtract `shift` S from the diagonal of
        every condensed block at the next assemble."""
        _lib.xbar_debug_shift_pivots(self._plan, shift)

    def set_timing(self, enable: bool = True) -> None:
        _lib.xbar_set_timing(self._plan, enable)

    def timing(self, reset: bool = False):
        return _lib.xbar_get_timing(self._plan, reset)

    def info(self):
        return _lib.xbar_get_info(self._plan)

    def check(self) -> None:
        st, _ = self.info()
        if st != _lib.XBAR_OK:
            raise XbarError("xbar_get_info", st)

    def close(self) -> None:
        if getattr(self, "_plan", None) is not None:
            _lib.xbar_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def tiles_currents(G, V, r_wl, r_bl, r_src=50.0, r_sense=50.0, out=None, stream=None):
    """Output currents of T crossbars of one shape in one launch (xbar_tiles_currents):
    G [T][m][n], V [T][B][m] float64 CUDA/HIP tensors; returns I [T][B][n]."""
    torch = _torch()
    T, m, n = (int(x) for x in G.shape)
    B = int(V.shape[1])
    _check_tensor("G", G, (T, m, n))
    _check_tensor("V", V, (T, B, m))
    if out is None:
        out = torch.empty((T, B, n), dtype=torch.float64, device="cuda")
    _check_tensor("I", out, (T, B, n))
    s = stream if stream is not None else torch.cuda.current_stream()
    geom = Geometry(m, n, float(r_wl), float(r_bl), float(r_src), float(r_sense))
    _lib.xbar_tiles_currents(geom, T, B, G, V, out, s.cuda_stream)
    return out


def solve(G, V, r_wl, r_bl, r_src=50.0, r_sense=50.0, precision="fp64", node_voltages=True,
          factor_method="auto"):
    """One-shot solve: returns (currents [B][n], node voltages [B][2mn] or None)."""
    torch = _torch()
    m, n = G.shape
    B = V.shape[0]
    with Plan(m, n, r_wl, r_bl, r_src, r_sense, precision, max_batch=B,
              factor_method=factor_method) as p:
        p.assemble(G)
        p.factor()
        nv = torch.empty((B, 2 * m * n), dtype=torch.float64, device="cuda") if node_voltages else None
        p.solve_batch(V, nv)
        I = p.currents()
        p.check()
    return I, nv


from .lanes import PlanLanes  # noqa: E402  (needs Plan above)
from .tiles import TileBatch, TileConfig  # noqa: E402
