"""Pins on the oracle against closed-form and limiting circuits.

Every expected value comes from tests/closed_forms.py, which derives it by
elementary circuit analysis without any oracle code.
"""
import numpy as np
import pytest

import oracle
from oracle import diagnostics as dg
from tests import closed_forms as cf


@pytest.mark.parametrize("G,V,r_src,r_sense", [(1e-4, 0.5, 50, 50), (3.3e-6, 0.17, 1.0, 7.0),
                                                (2e-5, 0.0, 10, 20)])
def test_single_cell(G, V, r_src, r_sense):
    res = oracle.solve(np.array([[G]]), np.array([[V]]), 5.0, 5.0, r_src, r_sense)
    assert res.currents[0, 0] == pytest.approx(cf.single_cell(G, V, r_src, r_sense), rel=4e-16, abs=0)


@pytest.mark.parametrize("n,r_wl", [(1, 1.0), (2, 2.5), (17, 1.0), (64, 5.0), (200, 2.5)])
def test_one_row_general(n, r_wl):
    rng = np.random.default_rng(n)
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (1, n)))
    V = 0.4
    res = oracle.solve(G, np.array([[V]]), r_wl, 3.0, 50.0, 50.0)
    v, I = cf.one_row(G[0], V, r_wl, 50.0, 50.0)
    np.testing.assert_allclose(res.currents[0], I, rtol=1e-13)
    np.testing.assert_allclose(res.node_v[0, 0::2], v, rtol=1e-13)


@pytest.mark.parametrize("n,G,r_wl", [(1, 5e-5, 1.0), (8, 1e-4, 5.0), (128, 3e-5, 2.5), (512, 1e-4, 1.0)])
def test_one_row_uniform_cosh(n, G, r_wl):
    Gm = np.full((1, n), G)
    res = oracle.solve(Gm, np.array([[0.5]]), r_wl, 1.0, 50.0, 50.0)
    v, I = cf.one_row_uniform_cosh(G, n, 0.5, r_wl, 50.0, 50.0)
    np.testing.assert_allclose(res.node_v[0, 0::2], v, rtol=1e-12)
    np.testing.assert_allclose(res.currents[0], I, rtol=1e-12)


@pytest.mark.parametrize("m,r_bl", [(1, 1.0), (2, 2.5), (33, 1.0), (256, 5.0)])
def test_one_column(m, r_bl):
    rng = np.random.default_rng(m + 1000)
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (m, 1)))
    V = rng.uniform(0, 0.5, (3, m))
    res = oracle.solve(G, V, 4.0, r_bl, 50.0, 50.0)
    for k in range(3):
        assert res.currents[k, 0] == pytest.approx(cf.one_column(G[:, 0], V[k], r_bl, 50.0, 50.0),
                                                   rel=1e-13)


def _dev(res_I, ref_I):
    return float(np.max(dg.relative_error(res_I, ref_I)))


def test_shorted_wire_limit():
    """Segment resistance -> 0 with finite source/sense: the bipartite network; deviation ~ r."""
    rng = np.random.default_rng(3)
    m, n = 7, 6
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (m, n)))
    V = rng.uniform(0, 0.5, (3, m))
    ref = cf.shorted_wires(G, V, 50.0, 50.0)
    devs = [_dev(oracle.solve(G, V, r, r, 50.0, 50.0).currents, ref) for r in (1e-2, 1e-3, 1e-4)]
    assert devs[0] < 1e-4
    assert 8.0 < devs[0] / devs[1] < 12.0 and 8.0 < devs[1] / devs[2] < 12.0


def test_ideal_limit_GtV():
    """All parasitic resistances -> 0: I = G^T V, with a deviation proportional to r."""
    rng = np.random.default_rng(4)
    m, n = 6, 5
    G = rng.uniform(1e-6, 1e-4, (m, n))
    V = rng.uniform(0, 0.5, (4, m))
    ref = cf.ideal_currents(G, V)
    devs = [_dev(oracle.solve(G, V, r, r, r, r).currents, ref) for r in (1e-1, 1e-2, 1e-3)]
    assert devs[2] < 5e-6
    assert 8.0 < devs[0] / devs[1] < 12.0 and 8.0 < devs[1] / devs[2] < 12.0
