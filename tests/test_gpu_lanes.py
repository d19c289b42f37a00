"""GPU checks of PlanLanes: many crossbars of mixed shapes through concurrent plans.

Each crossbar's currents must equal, bit for bit, those of a single plan of its
shape run alone on the default stream (the same kernels, so the same bits), and
agree with the oracle within the float64 tolerance.
"""
import numpy as np
import pytest

import oracle
from tests.gpu_util import TOL_FP64, log, rel_err

pytestmark = pytest.mark.gpu

R = (2.5, 2.5, 50.0, 50.0)
SHAPES = [(20, 70, 5), (33, 128, 16), (64, 96, 3), (5, 130, 8), (33, 128, 7), (20, 70, 1), (48, 200, 12)]


def _inputs(seed):
    rng = np.random.default_rng(seed)
    out = []
    for m, n, B in SHAPES:
        G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (m, n)))
        V = rng.uniform(0.0, 0.5, (B, m))
        out.append((G, V))
    return out


@pytest.mark.parametrize("lanes", [1, 3])
def test_lanes_match_single_plans_and_oracle(lanes):
    import torch

    import paper_2410_19993_amd as xb
    data = _inputs(500 + lanes)
    Gs = [torch.from_numpy(G).cuda() for G, _ in data]
    Vs = [torch.from_numpy(V).cuda() for _, V in data]
    log(f"case plan lanes: {len(SHAPES)} crossbars, {lanes} lanes")
    with xb.PlanLanes(*R, lanes=lanes, max_batch=16) as pl:
        got = [I.cpu().numpy() for I in pl.currents(Gs, Vs)]
        again = [I.cpu().numpy() for I in pl.currents(Gs, Vs)]      # plans reused
        pl.check()
    worst = 0.0
    for k, ((m, n, B), (G, V)) in enumerate(zip(SHAPES, data)):
        with xb.Plan(m, n, *R, "fp64", max_batch=B) as p:
            p.assemble(Gs[k])
            p.factor()
            p.solve_batch(Vs[k], None)
            ref = p.currents().cpu().numpy()
            p.check()
        assert np.array_equal(got[k], ref), f"crossbar {k} {m}x{n}"
        assert np.array_equal(again[k], ref), f"crossbar {k} {m}x{n}, second call"
        worst = max(worst, float(rel_err(got[k], oracle.solve(G, V, *R).currents).max()))
    log(f"  max current rel err {worst:.3e}")
    assert worst <= TOL_FP64


def test_lanes_reject_bad_arguments_before_launching():
    import torch

    import paper_2410_19993_amd as xb
    G = torch.full((8, 130), 1e-5, dtype=torch.float64, device="cuda")
    V = torch.zeros((9, 8), dtype=torch.float64, device="cuda")
    with xb.PlanLanes(*R, lanes=2, max_batch=8) as pl:
        with pytest.raises(ValueError):
            pl.currents([G], [V])                                   # batch above max_batch
        with pytest.raises(ValueError):
            pl.currents([G], [V[:4, :7].contiguous()])              # V columns != m
        with pytest.raises(ValueError):
            pl.currents([G, G], [V[:4]])                            # lengths differ
        assert pl.currents([], []) == []


def test_lanes_report_each_failed_crossbar():
    """A plan clears its error flags at every assembly, so a failure must be read per
    crossbar: a negative conductance in crossbars 1 and 4 (of six of one shape, so
    later crossbars reuse the failed plans) is reported for exactly those, and the
    others still match single plans."""
    import torch

    import paper_2410_19993_amd as xb
    rng = np.random.default_rng(600)
    m, n, B = 12, 80, 4
    Gs, Vs = [], []
    for k in range(6):
        G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (m, n)))
        if k in (1, 4):
            G[3, 5] = -1e-5
        Gs.append(torch.from_numpy(G).cuda())
        Vs.append(torch.from_numpy(rng.uniform(0, 0.5, (B, m))).cuda())
    log("case plan lanes with failing crossbars 1 and 4, 2 lanes")
    with xb.PlanLanes(*R, lanes=2, max_batch=B) as pl:
        outs = pl.currents(Gs, Vs)
        assert pl.failed() == [1, 4]
        with pytest.raises(xb.XbarError):
            pl.check()
        for k in (0, 2, 3, 5):
            with xb.Plan(m, n, *R, "fp64", max_batch=B) as p:
                p.assemble(Gs[k])
                p.factor()
                p.solve_batch(Vs[k], None)
                assert np.array_equal(outs[k].cpu().numpy(), p.currents().cpu().numpy())
        pl.currents([Gs[0]], [Vs[0]])
        assert pl.failed() == []
        pl.check()
