"""GPU parity of the Krylov refinement around the bfloat16 factor (XBAR_BF16_GMRES_IR):
restarted flexible GMRES in float64 preconditioned by float32 sweeps of the factor
whose inverse blocks are rounded to bfloat16.

Where the classical refinement with the same factor cannot contract (kappa u_bf16
above one), GMRES only needs the preconditioned operator's spectrum to be clustered.
Output currents (and node voltages) must match the oracle within 1e-9, or the solve
must report XBAR_ERR_NO_CONVERGENCE; every case logs the outer steps and the error.
"""
import os

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import GOLDEN, TOL_IR, gpu_solve, log, node_rel_err, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,B,seed", [(1, 1, 1, 31), (16, 16, 8, 32), (37, 53, 21, 33), (64, 64, 16, 34),
                                        (3, 130, 5, 35), (90, 20, 40, 36)])
def test_gmres_ir_matches_oracle(m, n, B, seed):
    wl = workloads.random_crossbar(m, n, B, seed, r_wl=2.5)
    log(f"case bf16_gmres {m}x{n} B={B}")
    I, nv, (st, info) = gpu_solve(wl.G, wl.V, wl.geom, "bf16_gmres", ir_tol=1e-12, ir_max_iter=20)
    ref = oracle.solve_workload(wl)
    e, ev = rel_err(I, ref.currents), node_rel_err(nv, ref.node_v)
    log(f"  status {st}, outer steps {info.ir_iters}, current rel err {e.max():.3e}, node {ev.max():.3e}")
    assert st == 0
    assert e.max() <= TOL_IR and ev.max() <= TOL_IR
    assert 1 <= info.ir_iters <= 20


def test_gmres_ir_c2_against_stored_oracle():
    """128 x 128, 1024 input vectors, 2.5-ohm segments: the configuration of the bfloat16
    trial, whose classical refinement does not contract there."""
    wl = workloads.c2()
    ref_I = np.load(os.path.join(GOLDEN, "c2_currents.npy"))
    log("case bf16_gmres c2")
    I, _, (st, info) = gpu_solve(wl.G, wl.V, wl.geom, "bf16_gmres", node_voltages=False, ir_tol=1e-12,
                                 ir_max_iter=30)
    e = rel_err(I, ref_I)
    log(f"  status {st}, outer steps {info.ir_iters}, max current rel err {e.max():.3e}")
    assert st in (0, 5)
    if st == 0:
        assert e.max() <= TOL_IR


def test_gmres_ir_zero_inputs():
    wl = workloads.random_crossbar(20, 24, 18, 37)
    wl.V[:] = 0.0
    log("case bf16_gmres zero inputs")
    I, nv, (st, info) = gpu_solve(wl.G, wl.V, wl.geom, "bf16_gmres")
    assert st == 0 and info.ir_iters == 1
    assert np.all(I == 0) and np.all(nv == 0)


def test_gmres_ir_reports_a_missed_tolerance():
    """One outer step cannot reach a tolerance below float64 rounding: the solve says so."""
    wl = workloads.random_crossbar(48, 40, 16, 38, r_wl=5.0)
    log("case bf16_gmres one step, tol 1e-18")
    from paper_2410_19993_amd import _lib
    _, _, (st, info) = gpu_solve(wl.G, wl.V, wl.geom, "bf16_gmres", ir_tol=1e-18, ir_max_iter=1)
    assert st == _lib.XBAR_ERR_NO_CONVERGENCE and info.ir_iters == 1


def test_gmres_ir_batches_share_a_plan():
    """Two batches on one factored plan (the second smaller, a ragged slab): each agrees
    with the oracle, so no state of the first leaks into the second."""
    import torch

    import paper_2410_19993_amd as xb
    wl = workloads.random_crossbar(40, 72, 35, 39, r_wl=1.0)
    ref = oracle.solve_workload(wl).currents
    log("case bf16_gmres two batches on one plan")
    with xb.Plan(40, 72, 1.0, 1.0, 50.0, 50.0, "bf16_gmres", max_batch=35, ir_tol=1e-12, ir_max_iter=20) as p:
        p.assemble(torch.from_numpy(wl.G).cuda())
        p.factor()
        for B in (35, 9):
            p.solve_batch(torch.from_numpy(wl.V[:B].copy()).cuda())
            I = p.currents().cpu().numpy()
            st, info = p.info()
            e = rel_err(I, ref[:B])
            log(f"  B={B}: status {st}, outer steps {info.ir_iters}, rel err {e.max():.3e}")
            assert st == 0 and e.max() <= TOL_IR


@pytest.mark.parametrize("r", [2.5, 5.0])
def test_gmres_ir_at_512_against_stored_oracle(r):
    """512 x 512 (the benchmark crossbar) with 32 of its stored-oracle input vectors: the
    classical refinement around the same bfloat16 factor is run beside it and its outcome
    logged; the GMRES refinement must converge to the oracle."""
    wl = workloads.c3(r=r)
    sub = workloads.c3_subset()[:32]
    ref_I = np.load(os.path.join(GOLDEN, f"c3_r{r:g}_currents.npy"))[:32]
    V = np.ascontiguousarray(wl.V[sub])
    for prec in ("bf16_ir", "bf16_gmres"):
        log(f"case {prec} c3 r={r} 32 vectors")
        I, _, (st, info) = gpu_solve(wl.G, V, wl.geom, prec, node_voltages=False, ir_tol=1e-12, ir_max_iter=30)
        e = rel_err(I, ref_I)
        log(f"  status {st}, refinement steps {info.ir_iters}, max current rel err {e.max():.3e}")
        if prec == "bf16_gmres":
            assert st == 0 and e.max() <= TOL_IR
        else:
            assert st in (0, 5) and (st == 5 or e.max() <= TOL_IR)
