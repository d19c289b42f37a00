"""Physical diagnostics of a node-voltage solution (branch currents, KCL, energy).

These evaluate a solution against the circuit itself rather than against the
matrix: every quantity is a sum of branch currents g * (v_a - v_b) over the
resistor list of ``oracle.netlist`` (Kirchhoff's current law, Eqs. 1-4).
"""
from __future__ import annotations

import numpy as np

from .netlist import GROUND, Netlist


def branch_currents(net: Netlist, node_v: np.ndarray) -> np.ndarray:
    """Current a -> b through every two-terminal resistor, [R][B]."""
    x = np.asarray(node_v, dtype=np.float64).T          # [N][B]
    xb = np.where((net.b == GROUND)[:, None], 0.0, x[np.maximum(net.b, 0)])
    return net.g[:, None] * (x[net.a] - xb)


def source_currents(net: Netlist, V: np.ndarray, node_v: np.ndarray) -> np.ndarray:
    """Current delivered by each input source into its word line, [B][m]."""
    x = np.asarray(node_v, dtype=np.float64).T
    V = np.atleast_2d(V)
    return (net.src_g[:, None] * (V[:, net.src_row].T - x[net.src_node])).T


def kcl_imbalance(net: Netlist, V: np.ndarray, node_v: np.ndarray) -> np.ndarray:
    """Net current into every node, [B][N] (zero for an exact solution)."""
    x = np.asarray(node_v, dtype=np.float64).T
    cur = branch_currents(net, node_v)
    acc = np.zeros_like(x)
    np.add.at(acc, net.a, -cur)
    both = net.b != GROUND
    np.add.at(acc, net.b[both], cur[both])
    np.add.at(acc, net.src_node, source_currents(net, V, node_v).T)
    return acc.T


def sense_currents_from_branches(net: Netlist, node_v: np.ndarray) -> np.ndarray:
    cur = branch_currents(net, node_v)
    sel = net.b == GROUND
    order = np.argsort(net.a[sel])
    return cur[sel][order].T                            # [B][n], column order


def power_balance(net: Netlist, V: np.ndarray, node_v: np.ndarray):
    """(power delivered by the sources, power dissipated in all resistors), [B] each."""
    x = np.asarray(node_v, dtype=np.float64).T
    V = np.atleast_2d(V)
    isrc = source_currents(net, V, node_v)              # [B][m]
    p_in = np.sum(isrc * V[:, net.src_row], axis=1)
    cur = branch_currents(net, node_v)
    p_res = np.sum(cur * cur / net.g[:, None], axis=0)
    drop_src = V[:, net.src_row].T - x[net.src_node]
    p_src = np.sum(net.src_g[:, None] * drop_src * drop_src, axis=0)
    return p_in, p_res + p_src


def relative_error(I: np.ndarray, I_ref: np.ndarray, abs_floor: float = 1e-18) -> np.ndarray:
    """Per input vector ||I - I_ref||_inf / ||I_ref||_inf over the columns ([B]).

    For an input vector whose reference currents are all zero the comparison is
    absolute: the error is 0 when every |I_j| <= abs_floor (amperes) and inf
    otherwise, so any relative tolerance then demands currents within abs_floor.
    """
    I = np.atleast_2d(np.asarray(I, dtype=np.float64))
    I_ref = np.atleast_2d(np.asarray(I_ref, dtype=np.float64))
    if I.shape != I_ref.shape:
        raise ValueError(f"shape mismatch {I.shape} vs {I_ref.shape}")
    num = np.max(np.abs(I - I_ref), axis=1)
    den = np.max(np.abs(I_ref), axis=1)
    zero_ref = np.where(num <= abs_floor, 0.0, np.inf)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), zero_ref)
