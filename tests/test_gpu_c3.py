"""GPU parity at the benchmark's full size: 512 x 512 crossbar, 4096 input vectors,
in the same plan configuration the benchmark times (max_batch = 4096, node voltages on).

The oracle cannot solve all 4096 vectors in test time, so the comparison uses
stored oracle outputs (tests/golden, written by make_golden.py from oracle/ only):
currents of a seeded 256-vector subset and node voltages of 8 of those vectors at
4096 seeded nodes.  Every vector of the batch is also checked against properties
that hold at any size:
  * charge conservation: the current drawn from the sources equals the current
    into the sense resistors, sum_i g_src (V_i - w_i0) = sum_j I_j;
  * maximum principle: for inputs >= 0 every node voltage lies in [0, max_i V_i],
    so every output current is >= 0.
"""
import os

import numpy as np
import pytest

import workloads
from tests.gpu_util import GOLDEN, TOL_FP64, TOL_IR, log, rel_err

pytestmark = pytest.mark.gpu


def _solve_c3(r, precision, ir_tol=0.0):
    import torch

    import paper_2410_19993_amd as xb
    wl = workloads.c3(r=r)
    g = wl.geom
    m, n, B = wl.G.shape[0], wl.G.shape[1], wl.B
    log(f"case c3 r={r} {precision} ir_tol={ir_tol}: m={m} n={n} B={B}")
    G = torch.from_numpy(wl.G).cuda()
    V = torch.from_numpy(np.ascontiguousarray(wl.V)).cuda()
    nv = torch.empty((B, 2 * m * n), dtype=torch.float64, device="cuda")
    with xb.Plan(m, n, g.r_wl, g.r_bl, g.r_src, g.r_sense, precision, max_batch=B, ir_tol=ir_tol) as p:
        p.assemble(G)
        p.factor()
        p.solve_batch(V, nv)
        I = p.currents()
        st, info = p.info()
        torch.cuda.synchronize()
    return wl, V, nv, I, st, info


def _check(wl, V, nv, I, tol):
    import torch
    m, n = wl.G.shape
    sub = workloads.c3_subset()
    tag = f"c3_r{wl.geom.r_wl:g}"
    ref = np.load(os.path.join(GOLDEN, f"{tag}_currents.npy"))
    Ih = I.cpu().numpy()
    e = rel_err(Ih[sub], ref)
    log(f"  subset current rel err {e.max():.3e}")
    assert np.all(np.isfinite(Ih)) and e.max() <= tol
    nodes = np.load(os.path.join(GOLDEN, f"{tag}_nodes.npz"))
    idx = torch.from_numpy(nodes["idx"]).cuda()
    got = nv[torch.from_numpy(sub[:8]).cuda()][:, idx].cpu().numpy()
    ref_v = nodes["v"]
    ev = np.max(np.abs(got - ref_v), axis=1) / np.max(np.abs(ref_v), axis=1)
    log(f"  sampled node-voltage rel err {ev.max():.3e}")
    assert ev.max() <= tol
    # properties over the whole batch
    w0 = nv.view(wl.B, m, n, 2)[:, :, 0, 0]               # word-line node j = 0 of every row
    src = (V - w0).sum(dim=1) / wl.geom.r_src
    out = I.sum(dim=1)
    cons = ((src - out).abs() / out.abs().clamp_min(1e-30)).max().item()
    log(f"  charge conservation, max rel mismatch over {wl.B} vectors: {cons:.3e}")
    assert cons <= 1e-9
    assert I.min().item() >= 0.0
    vmax = V.max(dim=1).values
    assert nv.min().item() >= -1e-12 and (nv.max(dim=1).values <= vmax * (1 + 1e-12)).all().item()


@pytest.mark.parametrize("r", [1.0, 2.5, 5.0])
def test_c3_fp64(r):
    wl, V, nv, I, st, info = _solve_c3(r, "fp64")
    assert st == 0
    _check(wl, V, nv, I, TOL_FP64)


# the benchmark's refinement tolerance (its float32 + refinement leg targets 1e-9)
BENCH_IR_TOL = 1e-10


@pytest.mark.parametrize("r", [1.0, 2.5, 5.0])
def test_c3_fp32_ir(r):
    """float32 factor + float64 refinement in the benchmark's configuration (ir_tol 1e-10)
    at every segment resistance of the 512 x 512 workload."""
    wl, V, nv, I, st, info = _solve_c3(r, "fp32_ir", ir_tol=BENCH_IR_TOL)
    assert st == 0
    log(f"  refinement sweeps {info.ir_iters}")
    _check(wl, V, nv, I, TOL_IR)
