"""Oracle solve: nodal matrix in band form, LU, substitution, refinement, readout.

Steps, in the paper's order (Sec. II.A-II.C):

1. Stamp the conductance matrix G and the injection vector I of the nodal
   equations G v = I (Eqs. 1-7) from the netlist, in the interleaved node
   order of Sec. II.B.  Row order = node order, so the matrix is symmetric
   (Sec. II.A) and banded with half-bandwidth 2n when m >= 2 (Sec. II.B and
   the bandwidth discussion of Sec. III.B).
2. LU decomposition G = LU with L unit lower (Sec. II.C), once per
   conductance map, without row exchanges (the matrix is symmetric and
   diagonally dominant, so Gaussian elimination never needs them).
3. For every input vector: L y = I, then U v = y (Sec. II.C); a batch of
   input vectors shares the one decomposition (Sec. III.A).
4. Classical iterative refinement with the KCL residual evaluated in long
   double from the resistor list, so that the reference is accurate well
   below the tolerances the GPU path is held to.
5. Output currents I_j = v(BL(m-1, j)) / r_sense: the current through the
   termination of each bit line (Sec. II).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _clib
from .netlist import GROUND, Netlist, build_netlist, sense_nodes


def half_bandwidth(net: Netlist) -> int:
    both = net.b != GROUND
    if not np.any(both):
        return 0
    return int(np.max(np.abs(net.a[both] - net.b[both])))


def assemble_band(net: Netlist, w: int | None = None):
    """Band storage of the nodal conductance matrix: ab[r][c - r + w]."""
    if w is None:
        w = half_bandwidth(net)
    N = net.num_nodes
    ab = np.zeros((N, 2 * w + 1), dtype=np.float64)
    a, b, g = net.a, net.b, net.g
    np.add.at(ab, (a, np.full(a.shape, w)), g)
    both = b != GROUND
    np.add.at(ab, (b[both], np.full(int(both.sum()), w)), g[both])
    np.add.at(ab, (a[both], b[both] - a[both] + w), -g[both])
    np.add.at(ab, (b[both], a[both] - b[both] + w), -g[both])
    np.add.at(ab, (net.src_node, np.full(net.src_node.shape, w)), net.src_g)
    return ab, w


def injections(net: Netlist, V: np.ndarray) -> np.ndarray:
    """Right-hand side I [N][B]: each source drives its node through src_g."""
    V = np.asarray(V, dtype=np.float64)
    Bn = V.shape[0]
    rhs = np.zeros((net.num_nodes, Bn), dtype=np.float64)
    np.add.at(rhs, net.src_node, net.src_g[:, None] * V[:, net.src_row].T)
    return rhs


def band_to_dense(ab: np.ndarray, w: int) -> np.ndarray:
    N = ab.shape[0]
    A = np.zeros((N, N))
    for r in range(N):
        lo, hi = max(0, r - w), min(N - 1, r + w)
        A[r, lo:hi + 1] = ab[r, lo - r + w:hi - r + w + 1]
    return A


def lu_factor(ab: np.ndarray, w: int):
    """In-place band LU; returns (lu, min_pivot)."""
    lu = np.ascontiguousarray(ab.copy())
    mp = ctypes.c_double(0.0)
    rc = _clib.lib().band_lu(lu.shape[0], w, _clib.dptr(lu), ctypes.pointer(mp))
    if rc != 0:
        raise FloatingPointError(f"non-positive or non-finite pivot at row {rc - 1}")
    return lu, float(mp.value)


def lu_solve(lu: np.ndarray, w: int, rhs: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(rhs.astype(np.float64, copy=True))
    _clib.lib().band_solve(lu.shape[0], w, _clib.dptr(lu), x.shape[1], _clib.dptr(x))
    return x


def kcl_residual_ld(net: Netlist, V: np.ndarray, x: np.ndarray, chunk: int = 64) -> np.ndarray:
    """I - G x from the resistor list in long double, rounded to float64 [N][B]."""
    V = np.ascontiguousarray(np.asarray(V, dtype=np.float64))
    N, Bn = x.shape
    out = np.empty_like(x)
    L = _clib.lib()
    for s in range(0, Bn, chunk):
        e = min(Bn, s + chunk)
        xs = np.ascontiguousarray(x[:, s:e])
        Vs = np.ascontiguousarray(V[s:e])
        acc = np.empty(N * (e - s), dtype=np.longdouble)
        o = np.empty((N, e - s), dtype=np.float64)
        L.netlist_residual_ld(N, net.g.size, _clib.iptr(net.a), _clib.iptr(net.b),
                              _clib.dptr(net.g), net.src_g.size, _clib.iptr(net.src_node),
                              _clib.iptr(net.src_row), _clib.dptr(net.src_g), net.m,
                              _clib.dptr(Vs), e - s, _clib.dptr(xs),
                              acc.ctypes.data_as(ctypes.c_void_p), _clib.dptr(o))
        out[:, s:e] = o
    return out


@dataclass
class OracleResult:
    currents: np.ndarray      # [B][n] amperes, + into the sense resistor
    node_v: np.ndarray        # [B][2mn] volts, paper order
    min_pivot: float
    correction_norms: list    # max |dx| of each refinement step
    residual_inf: float       # max |I - G v| after refinement (A)


def solve(G, V, r_wl, r_bl, r_src, r_sense, refine: int = 2) -> OracleResult:
    G = np.asarray(G, dtype=np.float64)
    V = np.atleast_2d(np.asarray(V, dtype=np.float64))
    net = build_netlist(G, r_wl, r_bl, r_src, r_sense)
    ab, w = assemble_band(net)
    lu, mp = lu_factor(ab, w)
    rhs = injections(net, V)
    x = lu_solve(lu, w, rhs)
    norms = []
    for _ in range(refine):
        r = kcl_residual_ld(net, V, x)
        d = lu_solve(lu, w, r)
        x = x + d
        norms.append(float(np.max(np.abs(d))) if d.size else 0.0)
    res = kcl_residual_ld(net, V, x)
    g_sense = 1.0 / r_sense
    cur = (x[sense_nodes(net.m, net.n), :] * g_sense).T.copy()
    return OracleResult(currents=cur, node_v=np.ascontiguousarray(x.T), min_pivot=mp,
                        correction_norms=norms,
                        residual_inf=float(np.max(np.abs(res))) if res.size else 0.0)


def solve_workload(wl, refine: int = 2, rows=None) -> OracleResult:
    """Solve a ``workloads.Workload`` (optionally only the input vectors ``rows``)."""
    V = wl.V if rows is None else wl.V[np.asarray(rows)]
    g = wl.geom
    return solve(wl.G, V, g.r_wl, g.r_bl, g.r_src, g.r_sense, refine=refine)
