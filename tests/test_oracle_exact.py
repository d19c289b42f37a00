"""Pins on the oracle's solve against exact and library solutions.

* Exact rational solves (brute force over Fractions) for crossbars up to 3x3,
  with the conductance sums formed exactly from the resistor list.
* LAPACK's dense partial-pivoting solve (numpy.linalg.solve) up to 12x12.
* SciPy's banded Cholesky (a different factorization of the same SPD
  matrix) up to 48x40.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import diagnostics as dg
from tests.closed_forms import fraction_solve, mna_fraction_system


@pytest.mark.parametrize("m,n", [(1, 1), (1, 3), (2, 2), (3, 1), (2, 3), (3, 3)])
def test_exact_rational(m, n):
    rng = np.random.default_rng(10 * m + n)
    G = rng.uniform(1e-6, 1e-4, (m, n))
    V = rng.uniform(0, 0.5, (2, m))
    r_wl, r_bl, r_src, r_sense = 1.5, 2.5, 50.0, 40.0
    res = oracle.solve(G, V, r_wl, r_bl, r_src, r_sense)
    net = oracle.build_netlist(G, r_wl, r_bl, r_src, r_sense)
    resistors = [(int(a), int(b), float(g)) for a, b, g in zip(net.a, net.b, net.g)]
    for k in range(V.shape[0]):
        sources = [(int(nd), float(g), float(V[k, r]))
                   for nd, r, g in zip(net.src_node, net.src_row, net.src_g)]
        A, rhs = mna_fraction_system(resistors, sources, net.num_nodes)
        x = np.array([float(v) for v in fraction_solve(A, rhs)])
        np.testing.assert_allclose(res.node_v[k], x, rtol=2e-15, atol=0)
        I_exact = x[oracle.sense_nodes(m, n)] / r_sense
        np.testing.assert_allclose(res.currents[k], I_exact, rtol=2e-15, atol=0)


@pytest.mark.parametrize("m,n", [(4, 4), (5, 9), (9, 5), (12, 12), (1, 12), (12, 1)])
def test_lapack_dense(m, n):
    rng = np.random.default_rng(m * 100 + n)
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (m, n)))
    V = rng.uniform(0, 0.5, (5, m))
    res = oracle.solve(G, V, 2.5, 2.5, 50, 50)
    net = oracle.build_netlist(G, 2.5, 2.5, 50, 50)
    ab, w = oracle.assemble_band(net)
    x = np.linalg.solve(oracle.band_to_dense(ab, w), oracle.injections(net, V))
    I = x[oracle.sense_nodes(m, n)].T / 50.0
    assert np.max(dg.relative_error(res.currents, I)) < 1e-12
    np.testing.assert_allclose(res.node_v, x.T, rtol=1e-12, atol=1e-16)


@pytest.mark.parametrize("m,n,r", [(32, 32, 1.0), (48, 40, 5.0), (40, 48, 2.5)])
def test_scipy_banded_cholesky(m, n, r):
    rng = np.random.default_rng(m + n)
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (m, n)))
    V = rng.uniform(0, 0.5, (4, m))
    res = oracle.solve(G, V, r, r, 50, 50)
    net = oracle.build_netlist(G, r, r, 50, 50)
    ab, w = oracle.assemble_band(net)
    N = ab.shape[0]
    upper = np.zeros((w + 1, N))             # LAPACK upper band: upper[w + r - c, c] = A[r, c]
    for d in range(w + 1):
        upper[w - d, d:] = ab[:N - d, w + d]
    cb = sla.cholesky_banded(upper, lower=False)
    x = sla.cho_solve_banded((cb, False), oracle.injections(net, V))
    I = x[oracle.sense_nodes(m, n)].T / 50.0
    assert np.max(dg.relative_error(res.currents, I)) < 1e-11


def test_refinement_converges():
    """Refinement corrections shrink; the final KCL residual is at rounding level."""
    rng = np.random.default_rng(7)
    m, n = 40, 40
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (m, n)))
    V = rng.uniform(0, 0.5, (3, m))
    res = oracle.solve(G, V, 2.5, 2.5, 50, 50, refine=3)
    c = res.correction_norms
    assert c[1] < 1e-2 * c[0] and c[2] <= c[1] * 10
    assert res.residual_inf < 1e-15


def test_batch_columns_independent():
    """Each input vector's arithmetic is independent: batch and single solves agree bitwise."""
    rng = np.random.default_rng(8)
    G = rng.uniform(1e-6, 1e-4, (6, 7))
    V = rng.uniform(0, 0.5, (5, 6))
    full = oracle.solve(G, V, 1, 1, 50, 50)
    for k in range(5):
        one = oracle.solve(G, V[k:k + 1], 1, 1, 50, 50)
        assert np.array_equal(one.currents[0], full.currents[k])
