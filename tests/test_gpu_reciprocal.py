"""GPU parity of reciprocal ordering: a crossbar with more columns than rows is solved
as its reciprocal (turned by 180 degrees and transposed, word and bit lines and the
source and sense resistors exchanged), so that the row blocks have the smaller side,
as the paper's bandwidth discussion (Sec. III.B) suggests.  The inputs then drive the
reciprocal's bit-line terminations; currents and node voltages are mapped back.

Parity: currents and node voltages against the oracle (which assembles the crossbar as
given) at 32 x 700 (only reachable this way: 700 > XBAR_MAX_N) and 700 x 32, on ragged
wide shapes, in every precision mode; the transfer matrix of a wide crossbar; the
backward error measured on the crossbar as given; both orderings of a 32 x 256 pair on
blocks of the same size.
"""
import os

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import GOLDEN, TOL_FP64, TOL_IR, gpu_solve, log, node_rel_err, rel_err

pytestmark = pytest.mark.gpu

TOLS = {"fp64": TOL_FP64, "fp32_ir": TOL_IR, "bf16_gmres": TOL_IR}


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir", "bf16_gmres"])
def test_32x700_against_stored_oracle(precision):
    wl = workloads.random_crossbar(32, 700, 3, 41)
    ref = np.load(os.path.join(GOLDEN, "rev_32x700_b3.npz"))
    log(f"case reciprocal 32x700 {precision}")
    I, nv, (st, info) = gpu_solve(wl.G, wl.V, wl.geom, precision, ir_max_iter=20)      # n > 512: reciprocal
    e, ev = rel_err(I, ref["I"]), node_rel_err(nv, ref["v"])
    log(f"  status {st}, block {info.block}, steps {info.ir_iters}, current rel err {e.max():.3e}, "
        f"node {ev.max():.3e}")
    assert st == 0 and info.block == 64
    assert e.max() <= TOLS[precision] and ev.max() <= TOLS[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_700x32_against_oracle(precision):
    wl = workloads.random_crossbar(700, 32, 3, 42)
    log(f"case tall 700x32 {precision}")
    I, nv, (st, info) = gpu_solve(wl.G, wl.V, wl.geom, precision)
    ref = oracle.solve_workload(wl)
    e, ev = rel_err(I, ref.currents), node_rel_err(nv, ref.node_v)
    log(f"  status {st}, block {info.block}, current rel err {e.max():.3e}, node {ev.max():.3e}")
    assert st == 0 and info.block == 64
    assert e.max() <= TOLS[precision] and ev.max() <= TOLS[precision]


@pytest.mark.parametrize("m,n,B,seed,r_wl,r_bl", [(1, 9, 2, 43, 2.5, 2.5), (2, 3, 4, 44, 1.0, 5.0),
                                                  (5, 33, 17, 45, 3.0, 1.5), (16, 40, 8, 46, 2.5, 2.5),
                                                  (63, 65, 20, 47, 4.0, 2.0), (100, 600, 5, 48, 1.0, 1.0)])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_wide_shapes_against_oracle(m, n, B, seed, r_wl, r_bl, precision):
    wl = workloads.random_crossbar(m, n, B, seed, r_wl=r_wl, r_bl=r_bl, r_src=30.0, r_sense=70.0)
    log(f"case wide {m}x{n} B={B} {precision} r_wl={r_wl} r_bl={r_bl}, row blocks of the smaller side")
    I, nv, (st, info) = gpu_solve(wl.G, wl.V, wl.geom, precision, ordering="smaller")
    ref = oracle.solve_workload(wl)
    e, ev = rel_err(I, ref.currents), node_rel_err(nv, ref.node_v)
    log(f"  status {st}, block {info.block}, current rel err {e.max():.3e}, node {ev.max():.3e}")
    assert st == 0 and info.block == 64 * ((m + 63) // 64)
    assert e.max() <= TOLS[precision] and ev.max() <= TOLS[precision]


def test_wide_transfer_matrix_and_apply():
    import torch

    import paper_2410_19993_amd as xb
    wl = workloads.random_crossbar(6, 50, 7, 49, r_wl=2.0, r_bl=3.0)
    T_ref = oracle.solve(wl.G, np.eye(6), 2.0, 3.0, 50.0, 50.0).currents
    log("case wide 6x50 transfer matrix")
    with xb.Plan(6, 50, 2.0, 3.0, 50.0, 50.0, "fp64", max_batch=7, ordering="smaller") as p:
        p.assemble(torch.from_numpy(wl.G).cuda())
        p.factor()
        T = p.transfer().cpu().numpy()
        I = torch.empty((7, 50), dtype=torch.float64, device="cuda")
        from paper_2410_19993_amd import _lib
        _lib.xbar_transfer_apply(p._plan, torch.from_numpy(T).cuda(), torch.from_numpy(wl.V).cuda(), 7, I)
        p.check()
    e = np.abs(T - T_ref).max() / np.abs(T_ref).max()
    log(f"  transfer rel err {e:.3e}")
    assert e <= TOL_FP64
    assert rel_err(I.cpu().numpy(), oracle.solve_workload(wl).currents).max() <= TOL_FP64


def _oracle_backward_error(wl, node_v):
    from oracle import diagnostics as dg
    g = wl.geom
    net = oracle.build_netlist(wl.G, g.r_wl, g.r_bl, g.r_src, g.r_sense)
    ab, _ = oracle.assemble_band(net)
    a_inf = np.abs(ab).sum(axis=1).max()
    b = oracle.injections(net, wl.V)                      # [N][B]
    r = dg.kcl_imbalance(net, wl.V, node_v)               # [B][N] = b - A v
    den = a_inf * np.abs(node_v).max(axis=1) + np.abs(b).max(axis=0)
    return np.abs(r).max(axis=1) / den


def test_wide_backward_error_on_the_crossbar_as_given():
    """The backward error is measured on the crossbar as given (its own order, G, V and
    resistances): on an unrefined bfloat16 solution (far above rounding) it equals the
    oracle's evaluation for the same node voltages."""
    import torch

    import paper_2410_19993_amd as xb
    wl = workloads.random_crossbar(12, 90, 5, 50, r_wl=2.5, r_bl=4.0, r_src=20.0, r_sense=80.0)
    log("case wide 12x90 backward error")
    with xb.Plan(12, 90, 2.5, 4.0, 20.0, 80.0, "bf16_ir", max_batch=5, ir_tol=1e-15, ir_max_iter=1,
                 ordering="smaller") as p:
        p.set_diagnostics(True)
        p.assemble(torch.from_numpy(wl.G).cuda())
        p.factor()
        nv = torch.empty((5, 2 * 12 * 90), dtype=torch.float64, device="cuda")
        p.solve_batch(torch.from_numpy(wl.V).cuda(), nv)
        st, info = p.info()
    eta = _oracle_backward_error(wl, nv.cpu().numpy())
    log(f"  status {st}, eta {info.max_backward_err:.9e}, oracle {eta.max():.9e}")
    assert eta.max() > 1e-12
    assert abs(info.max_backward_err - eta.max()) <= 1e-8 * eta.max()


def test_both_orderings_of_a_pair_use_the_smaller_block():
    """32 x 256 and 256 x 32 with row blocks of the smaller side solve on blocks of 32
    (padded 64): the same path; 32 x 256 ordered by rows uses blocks of 256."""
    for (m, n, order, block) in ((32, 256, "smaller", 64), (256, 32, "smaller", 64), (32, 256, "rows", 256),
                                 (256, 32, "rows", 64)):
        wl = workloads.random_crossbar(m, n, 16, 51 + m)
        log(f"case pair {m}x{n} ordering {order}")
        I, _, (st, info) = gpu_solve(wl.G, wl.V, wl.geom, "fp64", node_voltages=False, ordering=order)
        e = rel_err(I, oracle.solve_workload(wl).currents)
        log(f"  block {info.block}, rel err {e.max():.3e}")
        assert st == 0 and info.block == block and e.max() <= TOL_FP64


@pytest.mark.parametrize("m,n,block", [(32, 256, 256), (128, 512, 128), (256, 512, 256), (64, 512, 512),
                                       (32, 700, 64), (300, 40, 64)])
def test_auto_ordering_follows_the_measured_cost_model(m, n, block):
    """The default ordering keeps rows where the chain of row blocks would grow more
    than the blocks shrink (32 x 256, 64 x 512), turns 128 x 512 and 256 x 512, and must
    turn past 512 columns; tall crossbars are already on their smaller side."""
    import torch

    import paper_2410_19993_amd as xb
    log(f"case auto ordering {m}x{n}")
    with xb.Plan(m, n, 2.5, 2.5, 50.0, 50.0, "fp64", max_batch=1) as p:
        st, info = p.info()
    log(f"  block {info.block}")
    assert info.block == block
