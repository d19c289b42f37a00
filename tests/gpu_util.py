"""Helpers shared by the GPU tests: run the HIP path through the C ABI on
seeded inputs and compare with the oracle."""
from __future__ import annotations

import os
import sys

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# Tolerances on per-vector relative error of the output currents.
TOL_FP64 = 1e-10
TOL_IR = 1e-9


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_solve(G, V, geom, precision="fp64", node_voltages=True, max_batch=None, ir_tol=0.0,
              ir_max_iter=0, factor_method="auto", ordering="auto"):
    """Solve on cuda:0 through the C ABI; returns (currents, node_v or None, info)."""
    import torch

    import paper_2410_19993_amd as xb
    m, n = G.shape
    B = V.shape[0]
    Gd = torch.from_numpy(np.ascontiguousarray(G, dtype=np.float64)).cuda()
    Vd = torch.from_numpy(np.ascontiguousarray(V, dtype=np.float64)).cuda()
    with xb.Plan(m, n, geom.r_wl, geom.r_bl, geom.r_src, geom.r_sense, precision,
                 max_batch=max_batch or B, ir_tol=ir_tol, ir_max_iter=ir_max_iter,
                 factor_method=factor_method, ordering=ordering) as p:
        p.assemble(Gd)
        p.factor()
        nv = torch.empty((B, 2 * m * n), dtype=torch.float64, device="cuda") if node_voltages else None
        p.solve_batch(Vd, nv)
        I = p.currents()
        st, info = p.info()
        torch.cuda.synchronize()
        return I.cpu().numpy(), (nv.cpu().numpy() if nv is not None else None), (st, info)


def rel_err(I, ref):
    from oracle import diagnostics as dg
    return dg.relative_error(I, ref)


def node_rel_err(v, ref):
    num = np.max(np.abs(v - ref), axis=1)
    den = np.max(np.abs(ref), axis=1)
    return np.where(den > 0, num / np.where(den > 0, den, 1), num)
