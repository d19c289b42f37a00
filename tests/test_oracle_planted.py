"""Sensitivity of the pins: plant plausible mistakes in the oracle, expect a pin to fail.

Each mutation rewires the oracle's netlist (or its refinement residual) the
way a slip in the code would, and the test asserts that at least one of the
independent checks below rejects the mutated oracle while all of them accept
the real one.
"""
import importlib

import numpy as np
import pytest

import oracle
from oracle import netlist as nl
from tests import closed_forms as cf

solve_mod = importlib.import_module("oracle.solve")


_TRUE_BUILD = nl.build_netlist


def _pins_pass() -> dict:
    """Run a compact set of independent pins on the (possibly mutated) oracle."""
    out = {}
    rng = np.random.default_rng(123)
    # single cell
    I = oracle.solve(np.array([[4e-5]]), np.array([[0.3]]), 2.0, 3.0, 50.0, 40.0).currents[0, 0]
    out["cell"] = abs(I - cf.single_cell(4e-5, 0.3, 50.0, 40.0)) <= 1e-15 * abs(I)
    # one row (m = 1)
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (1, 9)))
    r = oracle.solve(G, np.array([[0.4]]), 2.0, 3.0, 50.0, 40.0)
    _, Iref = cf.one_row(G[0], 0.4, 2.0, 50.0, 40.0)
    out["row"] = np.allclose(r.currents[0], Iref, rtol=1e-12, atol=0)
    # one column (n = 1)
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (9, 1)))
    V = rng.uniform(0, 0.5, (1, 9))
    r = oracle.solve(G, V, 2.0, 3.0, 50.0, 40.0)
    out["col"] = np.isclose(r.currents[0, 0], cf.one_column(G[:, 0], V[0], 3.0, 50.0, 40.0),
                            rtol=1e-12, atol=0)
    # shorted-wire limit on a non-square crossbar
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (5, 4)))
    V = rng.uniform(0, 0.5, (2, 5))
    r = oracle.solve(G, V, 1e-4, 1e-4, 50.0, 40.0)
    ref = cf.shorted_wires(G, V, 50.0, 40.0)
    out["shorted"] = np.allclose(r.currents, ref, rtol=1e-5, atol=0)
    # exact rational solve, 2x3, distinct resistances
    G = rng.uniform(1e-6, 1e-4, (2, 3))
    V = rng.uniform(0, 0.5, (1, 2))
    r = oracle.solve(G, V, 1.5, 2.5, 50.0, 40.0)
    net = _TRUE_BUILD(G, 1.5, 2.5, 50.0, 40.0)            # the real circuit, never the mutated one
    res = [(int(a), int(b), float(g)) for a, b, g in zip(net.a, net.b, net.g)]
    src = [(int(nd), float(g), float(V[0, rr])) for nd, rr, g in zip(net.src_node, net.src_row, net.src_g)]
    A, rhs = cf.mna_fraction_system(res, src, net.num_nodes)
    x = np.array([float(v) for v in cf.fraction_solve(A, rhs)])
    out["exact"] = np.allclose(r.node_v[0], x, rtol=1e-14, atol=0)
    return out


def _mutated(kind):
    def build(G, r_wl, r_bl, r_src, r_sense):
        net = _TRUE_BUILD(G, r_wl, r_bl, r_src, r_sense)
        m, n = net.m, net.n
        if kind == "source_far_end":
            net.src_node = nl.wl_node(np.arange(m), n - 1, n).astype(np.int64)
        elif kind == "sense_top_row":
            s = net.kind == nl.KIND_SENSE
            net.a[s] = nl.bl_node(0, np.arange(n), n)
        elif kind == "wl_uses_bl_conductance":
            net.g[net.kind == nl.KIND_WL] = 1.0 / r_bl
        elif kind == "sense_uses_r_bl":
            net.g[net.kind == nl.KIND_SENSE] = 1.0 / r_bl
        elif kind == "device_G_transposed_index":
            d = net.kind == nl.KIND_DEVICE
            net.g[d] = np.asarray(G, dtype=np.float64)[:, ::-1].ravel()
        elif kind == "bl_coupling_off_by_one":
            s = net.kind == nl.KIND_BL
            net.b[s] = net.b[s] - 1
        elif kind == "source_conductance_dropped_row0":
            net.src_g = net.src_g.copy()
            net.src_g[0] = 0.5 * net.src_g[0]
        return net
    return build


MUTATIONS = ["source_far_end", "sense_top_row", "wl_uses_bl_conductance", "sense_uses_r_bl",
             "device_G_transposed_index", "bl_coupling_off_by_one",
             "source_conductance_dropped_row0"]


def test_pins_accept_true_oracle():
    res = _pins_pass()
    assert all(res.values()), res


@pytest.mark.parametrize("kind", MUTATIONS)
def test_pins_reject_mutated_netlist(kind, monkeypatch):
    monkeypatch.setattr(solve_mod, "build_netlist", _mutated(kind))
    res = _pins_pass()
    assert not all(res.values()), f"mutation {kind} went unnoticed: {res}"


def test_pins_reject_flipped_residual_sign(monkeypatch):
    true_res = solve_mod.kcl_residual_ld
    monkeypatch.setattr(solve_mod, "kcl_residual_ld", lambda *a, **k: -true_res(*a, **k))
    res = _pins_pass()
    assert not all(res.values()), res
