"""Independent circuit results used to pin the oracle (no oracle code used here).

Each function derives the answer for a special crossbar by elementary
circuit analysis (series/parallel reduction, Thevenin/Norton equivalents,
the discrete cosh solution of a uniform ladder, or the limiting circuit
obtained when wire segments become short circuits).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def single_cell(G, V, r_src, r_sense):
    """1x1 crossbar: source, device and sense resistor in series."""
    return V / (r_src + 1.0 / G + r_sense)


def one_row(G_row, V, r_wl, r_src, r_sense):
    """1xN crossbar (one word line): Thevenin reduction from the far end.

    With m = 1 every bit line is just its device in series with the sense
    resistor, a shunt y_j = 1/(1/G_j + r_sense) from word-line node j to
    ground.  Returns (word-line voltages [n], output currents [n]).
    """
    G_row = np.asarray(G_row, dtype=np.float64)
    n = G_row.size
    y = 1.0 / (1.0 / G_row + r_sense)
    Y = np.empty(n)                       # input admittance looking right from node j
    Y[n - 1] = y[n - 1]
    for j in range(n - 2, -1, -1):
        Y[j] = y[j] + 1.0 / (r_wl + 1.0 / Y[j + 1])
    v = np.empty(n)
    v[0] = V * (1.0 / r_src) / (1.0 / r_src + Y[0])
    for j in range(n - 1):
        zin = 1.0 / Y[j + 1]
        v[j + 1] = v[j] * zin / (r_wl + zin)
    return v, y * v


def one_row_uniform_cosh(G, n, V, r_wl, r_src, r_sense):
    """1xN crossbar with equal devices: v_j = A cosh(theta (n - 1/2 - j)), 0-based.

    Interior KCL gives v_{j-1} + v_{j+1} = (2 + y r_wl) v_j with
    y = 1/(1/G + r_sense), i.e. cosh(theta) = 1 + y r_wl / 2; the open far end
    makes the solution even about j = n - 1/2; the source node fixes A.
    """
    y = 1.0 / (1.0 / G + r_sense)
    g_s, g_w = 1.0 / r_src, 1.0 / r_wl
    theta = 2.0 * np.arcsinh(np.sqrt(y * r_wl / 4.0))   # cosh(t) = 1 + 2 sinh^2(t/2), no cancellation
    c = lambda j: np.cosh(theta * (n - 0.5 - j))
    A = V * g_s / ((g_s + y + g_w) * c(0) - g_w * c(1)) if n > 1 else V * g_s / ((g_s + y) * c(0))
    v = A * np.array([c(j) for j in range(n)])
    return v, y * v


def one_column(G_col, V, r_bl, r_src, r_sense):
    """Mx1 crossbar (one bit line): Thevenin reduction from the top row down.

    Row i drives bit-line node i through r_src + 1/G_i from source V_i.
    Returns the single output current.
    """
    G_col = np.asarray(G_col, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    gam = 1.0 / (r_src + 1.0 / G_col)
    E, R = V[0], 1.0 / gam[0]
    for i in range(1, G_col.size):
        a = 1.0 / (R + r_bl)
        E = (a * E + gam[i] * V[i]) / (a + gam[i])
        R = 1.0 / (a + gam[i])
    return E / (R + r_sense)


def shorted_wires(G, V, r_src, r_sense):
    """Limit of zero wire-segment resistance: each word line and each bit line
    collapses to a single node, leaving an (m+n)-node bipartite network.
    Returns output currents [B][n]."""
    G = np.asarray(G, dtype=np.float64)
    V = np.atleast_2d(V)
    m, n = G.shape
    g_s, g_t = 1.0 / r_src, 1.0 / r_sense
    K = np.zeros((m + n, m + n))
    K[:m, :m] = np.diag(g_s + G.sum(axis=1))
    K[m:, m:] = np.diag(g_t + G.sum(axis=0))
    K[:m, m:] = -G
    K[m:, :m] = -G.T
    rhs = np.zeros((m + n, V.shape[0]))
    rhs[:m] = g_s * V.T
    sol = np.linalg.solve(K, rhs)
    return (g_t * sol[m:]).T


def ideal_currents(G, V):
    """All parasitics zero: every device sees its full input voltage, I = G^T V."""
    return np.atleast_2d(V) @ np.asarray(G)


def fraction_solve(A, b):
    """Exact Gaussian elimination over the rationals (tiny systems only)."""
    n = len(A)
    M = [[Fraction(A[i][j]) for j in range(n)] + [Fraction(b[i])] for i in range(n)]
    for k in range(n):
        p = next(r for r in range(k, n) if M[r][k] != 0)
        M[k], M[p] = M[p], M[k]
        for r in range(k + 1, n):
            if M[r][k] != 0:
                f = M[r][k] / M[k][k]
                M[r] = [x - f * y for x, y in zip(M[r], M[k])]
    x = [Fraction(0)] * n
    for k in range(n - 1, -1, -1):
        s = M[k][n] - sum(M[k][j] * x[j] for j in range(k + 1, n))
        x[k] = s / M[k][k]
    return x


def mna_fraction_system(resistors, sources, num_nodes):
    """Nodal system over the rationals from a resistor list.

    resistors: iterable of (a, b, g) with b = -1 for ground; sources: iterable
    of (node, g, V).  Exact, so the conductance sums are not rounded.
    """
    A = [[Fraction(0)] * num_nodes for _ in range(num_nodes)]
    rhs = [Fraction(0)] * num_nodes
    for a, b, g in resistors:
        g = Fraction(g)
        A[a][a] += g
        if b >= 0:
            A[b][b] += g
            A[a][b] -= g
            A[b][a] -= g
    for node, g, V in sources:
        A[node][node] += Fraction(g)
        rhs[node] += Fraction(g) * Fraction(V)
    return A, rhs
