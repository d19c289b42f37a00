"""Pins of the oracle's checker functions, against values worked out by hand.

``relative_error`` gates every GPU parity test and ``kcl_imbalance`` the KCL
checks, so each gets hand-computed cases of its own (not a retyped formula):
small arrays whose row-wise and column-wise answers differ, so that a reduction
over the wrong axis, a normalisation per column or a dropped absolute floor
fails; and two tiny crossbars (1 x 2 and 2 x 1) with node voltages that are not
a solution, whose net currents into every node were summed by hand from the
circuit of Sec. II.A (source links, word-line and bit-line segments, devices,
sense terminations; Kirchhoff's current law, Eqs. 1-4).
"""
import numpy as np
import pytest

from oracle import build_netlist
from oracle import diagnostics as dg


def test_relative_error_by_hand():
    ref = np.array([[1.0, 2.5, 0.5],
                    [3.0, -5.0, 1.0],
                    [0.0, 0.0, 0.0]])
    got = np.array([[1.0, 2.0, 0.5],      # max |diff| 0.5, max |ref| 2.5 -> 0.2
                    [3.5, -5.0, 1.0],     # max |diff| 0.5, max |ref| 5.0 -> 0.1
                    [0.0, 0.0, 0.0]])     # all-zero reference, exact -> 0
    e = dg.relative_error(got, ref)
    assert e.shape == (3,)
    assert e[0] == pytest.approx(0.2, rel=1e-15)
    assert e[1] == pytest.approx(0.1, rel=1e-15)
    assert e[2] == 0.0
    # per-column normalisation would give 0.5/3 = 0.1667 for column 0; the wrong
    # axis would give 3 entries of a different kind: both differ from the above
    assert not np.isclose(e[1], 0.5 / 3.0)


def test_relative_error_absolute_floor_for_zero_reference():
    ref = np.zeros((2, 4))
    within = np.array([[0.0, 5e-19, -1e-18, 0.0],
                       [0.0, 0.0, 0.0, 0.0]])
    assert np.all(dg.relative_error(within, ref) == 0.0)
    beyond = np.array([[0.0, 0.0, 3e-18, 0.0],
                       [0.0, 2e-11, 0.0, 0.0]])
    e = dg.relative_error(beyond, ref)
    assert np.all(np.isinf(e))
    # a relative gate of 1e-10 must reject an all-zero reference answered with 2e-11 A
    assert not (e <= 1e-10).all()
    # the floor is the caller's choice
    assert np.all(dg.relative_error(beyond, ref, abs_floor=1e-10) == 0.0)


def test_relative_error_rejects_mismatched_shapes():
    with pytest.raises(ValueError):
        dg.relative_error(np.zeros((2, 3)), np.zeros((3, 2)))


def test_kcl_imbalance_one_row_by_hand():
    # 1 x 2: g_wl = 1, g_bl = 1 (unused: one row), g_src = 2, g_sense = 4, G = [1, 2]
    net = build_netlist(np.array([[1.0, 2.0]]), 1.0, 1.0, 0.5, 0.25)
    V = np.array([[3.0]])
    # node order WL(0,0), BL(0,0), WL(0,1), BL(0,1)
    v = np.array([[1.0, 2.0, 3.0, 5.0]])
    # WL(0,0): 2 (3-1) + 1 (3-1) + 1 (2-1) = 7
    # BL(0,0): 1 (1-2) + 4 (0-2)           = -9
    # WL(0,1): 1 (1-3) + 2 (5-3)           = 2
    # BL(0,1): 2 (3-5) + 4 (0-5)           = -24
    np.testing.assert_allclose(dg.kcl_imbalance(net, V, v), [[7.0, -9.0, 2.0, -24.0]], rtol=0, atol=1e-14)


def test_kcl_imbalance_one_column_two_vectors_by_hand():
    # 2 x 1: g_bl = 2, g_src = 2, g_sense = 4, G = [[1], [3]]
    net = build_netlist(np.array([[1.0], [3.0]]), 1.0, 0.5, 0.5, 0.25)
    V = np.array([[3.0, 1.0],
                  [0.0, 2.0]])
    # node order WL(0,0), BL(0,0), WL(1,0), BL(1,0)
    v = np.array([[1.0, 2.0, 3.0, 5.0],
                  [1.0, 1.0, 1.0, 1.0]])
    # vector 0:
    #   WL(0,0): 2 (3-1) + 1 (2-1)                 = 5
    #   BL(0,0): 1 (1-2) + 2 (5-2)                 = 5
    #   WL(1,0): 2 (1-3) + 3 (5-3)                 = 2
    #   BL(1,0): 3 (3-5) + 2 (2-5) + 4 (0-5)       = -32
    # vector 1 (all nodes at 1 V):
    #   WL(0,0): 2 (0-1) = -2;  BL(0,0): 0;  WL(1,0): 2 (2-1) = 2;  BL(1,0): 4 (0-1) = -4
    want = np.array([[5.0, 5.0, 2.0, -32.0],
                     [-2.0, 0.0, 2.0, -4.0]])
    np.testing.assert_allclose(dg.kcl_imbalance(net, V, v), want, rtol=0, atol=1e-14)


# ---- planted mistakes: each plausible slip in a checker fails the pins above ----

def _relerr_pins(fn) -> bool:
    ref = np.array([[1.0, 2.5, 0.5], [3.0, -5.0, 1.0], [0.0, 0.0, 0.0]])
    got = np.array([[1.0, 2.0, 0.5], [3.5, -5.0, 1.0], [0.0, 0.0, 0.0]])
    try:
        e = np.asarray(fn(got, ref))
        ok = e.shape == (3,) and np.allclose(e, [0.2, 0.1, 0.0], rtol=1e-14, atol=0)
        z = np.asarray(fn(np.array([[0.0, 2e-11]]), np.zeros((1, 2))))
        return bool(ok and not (z <= 1e-10).all())
    except Exception:
        return False


def _relerr_per_column(I, ref, abs_floor=1e-18):
    num = np.max(np.abs(I - ref), axis=1)
    den = np.max(np.abs(ref), axis=0)[: len(num)]
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num)


def _relerr_wrong_axis(I, ref, abs_floor=1e-18):
    num = np.max(np.abs(I - ref), axis=0)
    den = np.max(np.abs(ref), axis=0)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num)


def _relerr_no_floor(I, ref, abs_floor=1e-18):
    num = np.max(np.abs(I - ref), axis=1)
    den = np.max(np.abs(ref), axis=1)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num)


@pytest.mark.parametrize("fn", [_relerr_per_column, _relerr_wrong_axis, _relerr_no_floor])
def test_relative_error_pins_catch_planted_mistakes(fn):
    assert _relerr_pins(dg.relative_error)
    assert not _relerr_pins(fn)


def _kcl_pins(fn) -> bool:
    net = build_netlist(np.array([[1.0], [3.0]]), 1.0, 0.5, 0.5, 0.25)
    V = np.array([[3.0, 1.0], [0.0, 2.0]])
    v = np.array([[1.0, 2.0, 3.0, 5.0], [1.0, 1.0, 1.0, 1.0]])
    want = np.array([[5.0, 5.0, 2.0, -32.0], [-2.0, 0.0, 2.0, -4.0]])
    net1 = build_netlist(np.array([[1.0, 2.0]]), 1.0, 1.0, 0.5, 0.25)
    try:
        return bool(np.allclose(fn(net, V, v), want, rtol=0, atol=1e-12) and
                    np.allclose(fn(net1, np.array([[3.0]]), np.array([[1.0, 2.0, 3.0, 5.0]])),
                                [[7.0, -9.0, 2.0, -24.0]], rtol=0, atol=1e-12))
    except Exception:
        return False


def _kcl_source_sign(net, V, node_v):
    x = np.asarray(node_v, dtype=np.float64).T
    cur = dg.branch_currents(net, node_v)
    acc = np.zeros_like(x)
    np.add.at(acc, net.a, -cur)
    both = net.b != dg.GROUND
    np.add.at(acc, net.b[both], cur[both])
    np.add.at(acc, net.src_node, -dg.source_currents(net, V, node_v).T)
    return acc.T


def _kcl_drop_grounded(net, V, node_v):
    x = np.asarray(node_v, dtype=np.float64).T
    cur = dg.branch_currents(net, node_v)
    both = net.b != dg.GROUND
    acc = np.zeros_like(x)
    np.add.at(acc, net.a[both], -cur[both])
    np.add.at(acc, net.b[both], cur[both])
    np.add.at(acc, net.src_node, dg.source_currents(net, V, node_v).T)
    return acc.T


def _kcl_first_vector_source(net, V, node_v):
    x = np.asarray(node_v, dtype=np.float64).T
    cur = dg.branch_currents(net, node_v)
    acc = np.zeros_like(x)
    np.add.at(acc, net.a, -cur)
    both = net.b != dg.GROUND
    np.add.at(acc, net.b[both], cur[both])
    Vb = np.repeat(np.atleast_2d(V)[:1], len(node_v), axis=0)
    np.add.at(acc, net.src_node, dg.source_currents(net, Vb, node_v).T)
    return acc.T


@pytest.mark.parametrize("fn", [_kcl_source_sign, _kcl_drop_grounded, _kcl_first_vector_source])
def test_kcl_imbalance_pins_catch_planted_mistakes(fn):
    assert _kcl_pins(dg.kcl_imbalance)
    assert not _kcl_pins(fn)
