"""Pins on the oracle from circuit laws that hold for any crossbar.

KCL at every node (Eqs. 1-4) is evaluated from branch currents over the
resistor list in float64 (oracle.diagnostics), a separate implementation
from the long-double residual the oracle refines with.
"""
import numpy as np
import pytest

import oracle
from oracle import diagnostics as dg

CASES = [(5, 4, 1.0), (8, 13, 2.5), (13, 8, 5.0), (24, 24, 2.5)]


def _case(m, n, r, seed=0, B=4):
    rng = np.random.default_rng(seed + 31 * m + n)
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (m, n)))
    V = rng.uniform(0, 0.5, (B, m))
    net = oracle.build_netlist(G, r, r, 50.0, 50.0)
    return G, V, net, oracle.solve(G, V, r, r, 50.0, 50.0)


@pytest.mark.parametrize("m,n,r", CASES)
def test_kcl_every_node(m, n, r):
    G, V, net, res = _case(m, n, r)
    imb = dg.kcl_imbalance(net, V, res.node_v)
    scale = np.max(np.abs(dg.source_currents(net, V, res.node_v)))
    assert np.max(np.abs(imb)) < 1e-12 * scale


@pytest.mark.parametrize("m,n,r", CASES)
def test_charge_conservation(m, n, r):
    """Current delivered by the sources equals current collected by the sense resistors."""
    G, V, net, res = _case(m, n, r)
    src = dg.source_currents(net, V, res.node_v).sum(axis=1)
    out = res.currents.sum(axis=1)
    np.testing.assert_allclose(src, out, rtol=1e-12)
    np.testing.assert_allclose(dg.sense_currents_from_branches(net, res.node_v), res.currents,
                               rtol=1e-14)


@pytest.mark.parametrize("m,n,r", CASES)
def test_power_balance(m, n, r):
    G, V, net, res = _case(m, n, r)
    p_in, p_diss = dg.power_balance(net, V, res.node_v)
    np.testing.assert_allclose(p_in, p_diss, rtol=1e-10)


@pytest.mark.parametrize("m,n,r", CASES)
def test_superposition(m, n, r):
    G, V, net, res = _case(m, n, r, B=2)
    V3 = np.vstack([V, V[0] + V[1], 2.5 * V[0]])
    out = oracle.solve(G, V3, r, r, 50.0, 50.0).currents
    np.testing.assert_allclose(out[2], out[0] + out[1], rtol=1e-13)
    np.testing.assert_allclose(out[3], 2.5 * out[0], rtol=1e-13)


@pytest.mark.parametrize("m,n,r", CASES)
def test_maximum_principle(m, n, r):
    """With non-negative inputs every node voltage lies in [0, max V_i]."""
    G, V, net, res = _case(m, n, r)
    assert np.all(res.node_v >= 0)
    assert np.all(res.node_v <= V.max(axis=1, keepdims=True) * (1 + 1e-14))


@pytest.mark.parametrize("m,n,r", CASES)
def test_parasitics_only_reduce_uniform_reads(m, n, r):
    """Equal inputs: wire and terminal resistance can only lower each column current below G^T V."""
    G, V, net, res = _case(m, n, r)
    Vu = np.full((1, m), 0.3)
    I = oracle.solve(G, Vu, r, r, 50.0, 50.0).currents[0]
    assert np.all(I > 0) and np.all(I <= (Vu @ G)[0])


def test_zero_input_zero_output():
    G, V, net, res = _case(6, 6, 2.5)
    out = oracle.solve(G, np.zeros((1, 6)), 2.5, 2.5, 50, 50)
    assert np.all(out.currents == 0) and np.all(out.node_v == 0)


def test_reciprocity():
    """Symmetric nodal matrix: the transfer from injection at node a to node b equals b to a."""
    m, n = 5, 6
    G = np.random.default_rng(9).uniform(1e-6, 1e-4, (m, n))
    net = oracle.build_netlist(G, 2.0, 3.0, 50, 40)
    ab, w = oracle.assemble_band(net)
    lu, _ = oracle.lu_factor(ab, w)
    N = net.num_nodes
    E = oracle.lu_solve(lu, w, np.eye(N))
    np.testing.assert_allclose(E, E.T, rtol=1e-10, atol=0)


@pytest.mark.parametrize("m,n", [(4, 7), (1, 5), (3, 3), (6, 2)])
def test_turned_crossbar_is_the_reciprocal_two_port(m, n):
    """The crossbar turned by 180 degrees and transposed (G'[i][j] = G[m-1-j][n-1-i], word
    and bit lines exchanged, so r_wl' = r_bl, r_bl' = r_wl, and the source and sense
    resistors exchanged) carries, by reciprocity of the passive network, the transfer
    T'[n-1-j][m-1-i] = T[i][j] between the same pair of terminals.  This is the relabelling
    that lets a wide crossbar be solved with row blocks of its smaller side."""
    rng = np.random.default_rng(100 + 10 * m + n)
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (m, n)))
    r_wl, r_bl, r_src, r_sense = 2.0, 3.5, 40.0, 60.0
    T = oracle.solve(G, np.eye(m), r_wl, r_bl, r_src, r_sense).currents
    Gt = np.empty((n, m))
    for i in range(n):
        for j in range(m):
            Gt[i, j] = G[m - 1 - j, n - 1 - i]
    Tt = oracle.solve(Gt, np.eye(n), r_bl, r_wl, r_sense, r_src).currents
    for i in range(m):
        for j in range(n):
            assert abs(Tt[n - 1 - j, m - 1 - i] - T[i, j]) <= 1e-12 * abs(T[i, j])
    # a wrong relabelling (resistances not exchanged) breaks it
    Tw = oracle.solve(Gt, np.eye(n), r_wl, r_bl, r_src, r_sense).currents
    assert max(abs(Tw[n - 1 - j, m - 1 - i] - T[i, j]) / T[i, j] for i in range(m) for j in range(n)) > 1e-6


@pytest.mark.parametrize("m,n,r", CASES)
def test_transfer_matrix_superposition(m, n, r):
    """Linear network: each vector's currents are its voltages times the currents per unit
    volt on each word line (I = V T), and every entry of T is positive (passive network with
    every conductance > 0)."""
    G, V, net, res = _case(m, n, r, B=6)
    T = oracle.solve(G, np.eye(m), r, r, 50.0, 50.0).currents      # row i: 1 V on word line i
    assert T.shape == (m, n) and np.all(T > 0)
    np.testing.assert_allclose(V @ T, res.currents, rtol=1e-12)
