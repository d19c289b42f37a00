"""Pins on the oracle's nodal matrix: sizes, structure and the paper's stamps.

Sources: Sec. II (2mn unknowns, nonzero count), Sec. II.A (3mn resistors,
symmetric matrix, Eqs. 5-7), Sec. II.B (interleaved unknown order, banded
form) and Sec. III.B (bandwidth grows with the number of columns n).
"""
import numpy as np
import pytest

import oracle
from oracle.netlist import GROUND

SHAPES = [(1, 1), (1, 2), (2, 1), (2, 2), (3, 7), (4, 3), (7, 3), (16, 16)]


def dense(G, r_wl=2.0, r_bl=3.0, r_src=50.0, r_sense=40.0):
    net = oracle.build_netlist(G, r_wl, r_bl, r_src, r_sense)
    ab, w = oracle.assemble_band(net)
    return net, oracle.band_to_dense(ab, w)


def rand_G(m, n, seed=0):
    return np.random.default_rng(seed).uniform(1e-6, 1e-4, (m, n))


@pytest.mark.parametrize("m,n", SHAPES)
def test_counts(m, n):
    """2mn nodes, 3mn resistors (Sec. II.A) and 8mn-2m-2n nonzeros (Sec. II, read as a sum)."""
    net, A = dense(rand_G(m, n))
    assert A.shape == (2 * m * n, 2 * m * n)
    assert net.num_resistors == 3 * m * n
    assert np.count_nonzero(A) == 8 * m * n - 2 * m - 2 * n


@pytest.mark.parametrize("m,n", SHAPES)
def test_symmetric_m_matrix(m, n):
    """Symmetric (Sec. II.A), positive diagonal, non-positive off-diagonal."""
    _, A = dense(rand_G(m, n, 1))
    assert np.array_equal(A, A.T)
    assert np.all(np.diag(A) > 0)
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0)


@pytest.mark.parametrize("m,n", SHAPES)
def test_row_sums_are_grounded_conductance(m, n):
    r_src, r_sense = 50.0, 40.0
    G = rand_G(m, n, 2)
    _, A = dense(G, r_src=r_src, r_sense=r_sense)
    expect = np.zeros(2 * m * n)
    for i in range(m):
        expect[oracle.wl_node(i, 0, n)] += 1 / r_src
    for j in range(n):
        expect[oracle.bl_node(m - 1, j, n)] += 1 / r_sense
    np.testing.assert_allclose(A.sum(axis=1), expect, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("m,n", SHAPES)
def test_half_bandwidth(m, n):
    """Bit-line coupling BL(i,j)-BL(i+1,j) sits 2n off the diagonal (Sec. II.B, III.B)."""
    net, A = dense(rand_G(m, n, 3))
    rows, cols = np.nonzero(A)
    w = int(np.max(np.abs(rows - cols)))
    expect = 2 * n if m >= 2 else (2 if n >= 2 else 1)
    assert w == expect == oracle.half_bandwidth(net)


def test_interleaved_order():
    """Unknowns ordered WL(1,1), BL(1,1), WL(1,2), BL(1,2), ... (Sec. II.B)."""
    m, n = 3, 4
    net = oracle.build_netlist(rand_G(m, n), 1, 1, 1, 1)
    for i in range(m):
        for j in range(n):
            assert oracle.wl_node(i, j, n) == 2 * (i * n + j)
            assert oracle.bl_node(i, j, n) == 2 * (i * n + j) + 1
    dev = net.kind == 2
    assert np.all(net.b[dev] - net.a[dev] == 1)          # device joins WL(i,j) to BL(i,j)
    wl = net.kind == 1
    assert np.all(net.b[wl] - net.a[wl] == 2)            # WL(i,j) - WL(i,j+1)
    bl = net.kind == 3
    assert np.all(net.b[bl] - net.a[bl] == 2 * n)        # BL(i,j) - BL(i+1,j)
    assert np.all(net.b[net.kind == 4] == GROUND)
    assert np.all(net.a[net.kind == 4] == oracle.sense_nodes(m, n))


def test_paper_stamps_eq5_eq6_eq7():
    """Rows of the matrix equal the printed stamps of Eqs. 5, 6 and 7.

    The paper's model has the source reached through a word-line segment
    (Eq. 5) and, by the same reading, the bit-line termination equal to a
    bit-line segment, so r_src = r_wl and r_sense = r_bl here.
    """
    m, n = 5, 6
    G = rand_G(m, n, 4)
    r_wl, r_bl = 2.0, 3.0
    G_WL, G_BL = 1 / r_wl, 1 / r_bl
    net, A = dense(G, r_wl=r_wl, r_bl=r_bl, r_src=r_wl, r_sense=r_bl)
    Vin = np.arange(1, m + 1) * 0.1
    I = oracle.injections(net, Vin[None, :])[:, 0]
    WL = lambda i, j: oracle.wl_node(i - 1, j - 1, n)   # 1-based as in the paper
    BL = lambda i, j: oracle.bl_node(i - 1, j - 1, n)

    def row(node):
        return {c: A[node, c] for c in np.nonzero(A[node])[0]}

    for i in range(1, m + 1):                     # Eq. 5: j = 1
        g = G[i - 1, 0]
        assert row(WL(i, 1)) == pytest.approx({WL(i, 1): 2 * G_WL + g, WL(i, 2): -G_WL,
                                                BL(i, 1): -g}, rel=1e-15)
        assert I[WL(i, 1)] == pytest.approx(Vin[i - 1] * G_WL, rel=1e-15)
    for i in range(2, m):                          # Eq. 6: interior word-line nodes
        for j in range(2, n):
            g = G[i - 1, j - 1]
            assert row(WL(i, j)) == pytest.approx({WL(i, j): 2 * G_WL + g, WL(i, j - 1): -G_WL,
                                                    WL(i, j + 1): -G_WL, BL(i, j): -g}, rel=1e-15)
            assert I[WL(i, j)] == 0
    for i in range(2, m):                          # Eq. 7: interior bit-line nodes, all j
        for j in range(1, n + 1):
            g = G[i - 1, j - 1]
            assert row(BL(i, j)) == pytest.approx({BL(i, j): 2 * G_BL + g, BL(i + 1, j): -G_BL,
                                                    BL(i - 1, j): -G_BL, WL(i, j): -g}, rel=1e-15)
            assert I[BL(i, j)] == 0
    # Boundary rows "derived similarly": Eq. 2 (j = n) and Eq. 3 (i = 1)
    for i in range(1, m + 1):
        g = G[i - 1, n - 1]
        assert row(WL(i, n)) == pytest.approx({WL(i, n): G_WL + g, WL(i, n - 1): -G_WL,
                                                BL(i, n): -g}, rel=1e-15)
    for j in range(1, n + 1):
        g = G[0, j - 1]
        assert row(BL(1, j)) == pytest.approx({BL(1, j): G_BL + g, BL(2, j): -G_BL,
                                                WL(1, j): -g}, rel=1e-15)
    assert np.count_nonzero(I) == m                # one injection per word line


def test_injection_count():
    m, n = 6, 5
    net = oracle.build_netlist(rand_G(m, n), 1, 1, 50, 50)
    I = oracle.injections(net, np.full((1, m), 0.3))
    assert np.count_nonzero(I) == m
