"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Float64 path: per-vector relative error of the output currents <= 1e-10
(the tolerance of the float64 solver); node voltages <= 1e-10 relative to
the vector's largest node voltage.
"""
import os

import numpy as np
import pytest

import oracle
import workloads
from oracle import diagnostics as dg
from tests.gpu_util import GOLDEN, TOL_FP64, TOL_IR, gpu_solve, log, node_rel_err, rel_err

pytestmark = pytest.mark.gpu


def _check_against_oracle(wl, precision="fp64", tol=TOL_FP64, **kw):
    log(f"case {wl.name} precision={precision} {kw}")
    I, nv, (st, info) = gpu_solve(wl.G, wl.V, wl.geom, precision, **kw)
    assert st == 0, f"device status {st}"
    ref = oracle.solve_workload(wl)
    e = rel_err(I, ref.currents)
    log(f"  max current rel err {e.max():.3e}")
    assert np.all(np.isfinite(I))
    assert e.max() <= tol
    ev = node_rel_err(nv, ref.node_v)
    log(f"  max node-voltage rel err {ev.max():.3e}")
    assert ev.max() <= tol
    return I, nv, ref


@pytest.mark.parametrize("method", ["auto", "gj", "ns", "checked"])
def test_c1_full(method):
    _check_against_oracle(workloads.c1(), factor_method=method)


@pytest.mark.parametrize("method", ["gj", "ns"])
@pytest.mark.parametrize("m,n,B,seed", [
    (1, 1, 1, 1), (1, 7, 3, 2), (9, 1, 5, 3), (2, 2, 16, 4), (3, 70, 17, 5), (65, 64, 33, 6),
    (7, 129, 15, 7), (10, 200, 20, 8), (4, 512, 2, 9), (33, 40, 48, 10), (9, 300, 20, 17),
    (6, 420, 18, 18), (5, 380, 12, 23)])
def test_ragged_shapes(m, n, B, seed, method):
    """Sizes that are not multiples of the 64-wide blocks or 16-vector slabs, with either
    way of inverting the pivot blocks (Gauss-Jordan, Newton-Schulz)."""
    wl = workloads.random_crossbar(m, n, B, seed, r_wl=1.5, r_bl=3.0, r_src=40.0, r_sense=60.0)
    _check_against_oracle(wl, factor_method=method)


def test_strong_devices_fall_back_or_converge():
    """Devices far stronger than the wires (1 kOhm cells, 20-ohm segments) make the pivot
    blocks far from diagonal; the default factor must still match the oracle."""
    rng = np.random.default_rng(77)
    wl = workloads.random_crossbar(24, 96, 8, 16, r_wl=20.0, r_bl=20.0)
    wl.G[:] = rng.uniform(5e-4, 1e-3, wl.G.shape)
    _check_against_oracle(wl, factor_method="checked")
    _check_against_oracle(wl, factor_method="gj")
    # the asynchronous default either converges or says that it did not
    I, _, (st, _) = gpu_solve(wl.G, wl.V, wl.geom, "fp64", factor_method="auto")
    assert st in (0, 5)
    if st == 0:
        assert rel_err(I, oracle.solve_workload(wl).currents).max() <= TOL_FP64


@pytest.mark.parametrize("r", [1.0, 2.5, 5.0])
def test_segment_resistance(r):
    wl = workloads.random_crossbar(48, 96, 24, 11, r_wl=r, r_bl=r)
    _check_against_oracle(wl)


def test_paper_model_resistances():
    """The paper's own model: 5-ohm parasitics, source and termination equal to a segment."""
    wl = workloads.random_crossbar(32, 32, 16, 12, r_wl=5.0, r_bl=5.0, r_src=5.0, r_sense=5.0,
                                   g_dist="uniform")
    _check_against_oracle(wl)


def test_zero_and_unit_inputs():
    wl = workloads.random_crossbar(20, 30, 4, 13)
    wl.V[0] = 0.0
    wl.V[1] = 0.5
    I, nv, (st, _) = gpu_solve(wl.G, wl.V, wl.geom)
    assert st == 0
    assert np.max(np.abs(I[0])) <= 1e-18 and np.max(np.abs(nv[0])) <= 1e-18
    ref = oracle.solve_workload(wl)
    assert rel_err(I[1:], ref.currents[1:]).max() <= TOL_FP64


def test_c2_full_golden():
    path = os.path.join(GOLDEN, "c2_currents.npy")
    ref = np.load(path)
    wl = workloads.c2()
    log(f"case {wl.name}")
    I, nv, (st, _) = gpu_solve(wl.G, wl.V, wl.geom, node_voltages=True)
    assert st == 0
    e = rel_err(I, ref)
    log(f"  max current rel err {e.max():.3e}")
    assert e.max() <= TOL_FP64
    # KCL at every node for a few vectors, from the GPU's node voltages
    net = oracle.build_netlist(wl.G, wl.geom.r_wl, wl.geom.r_bl, wl.geom.r_src, wl.geom.r_sense)
    sel = [0, 511, 1023]
    imb = dg.kcl_imbalance(net, wl.V[sel], nv[sel])
    src = dg.source_currents(net, wl.V[sel], nv[sel])
    log(f"  max KCL imbalance {np.abs(imb).max():.3e} A (source scale {np.abs(src).max():.3e})")
    assert np.abs(imb).max() <= 1e-9 * np.abs(src).max()


def test_batch_invariance_and_determinism():
    """Input vectors are independent: a vector solved alone or inside a batch gives the
    same bits, and two identical runs are bitwise equal."""
    wl = workloads.random_crossbar(24, 80, 37, 14)
    I1, nv1, _ = gpu_solve(wl.G, wl.V, wl.geom)
    I2, nv2, _ = gpu_solve(wl.G, wl.V, wl.geom)
    assert np.array_equal(I1, I2) and np.array_equal(nv1, nv2)
    for k in (0, 17, 36):
        Ik, nvk, _ = gpu_solve(wl.G, wl.V[k:k + 1], wl.geom)
        assert np.array_equal(Ik[0], I1[k]) and np.array_equal(nvk[0], nv1[k])


def test_plan_reuse_many_batches():
    """Decompose once, solve many batches (Sec. III.A), including a smaller second batch."""
    import torch

    import paper_2410_19993_amd as xb
    wl = workloads.random_crossbar(40, 72, 64, 15)
    ref = oracle.solve_workload(wl)
    g = wl.geom
    with xb.Plan(40, 72, g.r_wl, g.r_bl, g.r_src, g.r_sense, "fp64", max_batch=64) as p:
        p.assemble(torch.from_numpy(wl.G).cuda())
        p.factor()
        for lo, hi in ((0, 64), (5, 12), (63, 64)):
            V = torch.from_numpy(np.ascontiguousarray(wl.V[lo:hi])).cuda()
            p.solve_batch(V)
            I = p.currents().cpu().numpy()
            p.check()
            assert rel_err(I, ref.currents[lo:hi]).max() <= TOL_FP64


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_user_stream_and_refactor(precision):
    """A plan queued on a non-default stream gives the bits of the default stream: the
    factor runs its second chain on the plan's own stream, forked from and joined back
    to the caller's.  Factoring the same map again on the same plan (the schedule then
    launches the slot counts the first factorization needed) gives the same bits too."""
    import torch

    import paper_2410_19993_amd as xb
    wl = workloads.random_crossbar(33, 96, 21, 16)
    log(f"case user stream {precision}: m=33 n=96 B=21")
    I0, nv0, (st0, _) = gpu_solve(wl.G, wl.V, wl.geom, precision)
    assert st0 == 0
    g = wl.geom
    s = torch.cuda.Stream()
    outs = []
    with torch.cuda.stream(s):
        Gd = torch.from_numpy(wl.G).cuda()
        Vd = torch.from_numpy(np.ascontiguousarray(wl.V)).cuda()
        with xb.Plan(33, 96, g.r_wl, g.r_bl, g.r_src, g.r_sense, precision, max_batch=21, stream=s) as p:
            for _ in range(2):
                p.assemble(Gd)
                p.factor()
                nv = torch.empty((21, 2 * 33 * 96), dtype=torch.float64, device="cuda")
                p.solve_batch(Vd, nv)
                outs.append((p.currents(), nv))
            st, _ = p.info()
    s.synchronize()
    assert st == 0
    for I, nv in outs:
        assert np.array_equal(I.cpu().numpy(), I0) and np.array_equal(nv.cpu().numpy(), nv0)


@pytest.mark.parametrize("m,n,B,seed", [(1024, 64, 24, 17), (513, 37, 9, 18)])
def test_long_chains(m, n, B, seed):
    """Tall crossbars: factor chains of 512 and 256 rows, and an odd row count."""
    wl = workloads.random_crossbar(m, n, B, seed)
    _check_against_oracle(wl)
    _check_against_oracle(wl, precision="fp32_ir", tol=TOL_IR)


@pytest.mark.parametrize("m,n,B,seed", [
    (1, 5, 3, 51), (2, 9, 4, 52), (3, 16, 17, 53), (5, 64, 16, 54), (64, 70, 33, 55),
    (65, 128, 20, 56), (200, 512, 40, 57), (513, 40, 9, 58)])
def test_currents_only_same_bits(m, n, B, seed):
    """Without node voltages the float64 sweep skips the upward back sweep (the currents
    depend only on the bottom row).  The currents must be the same bits as with node
    voltages, and within the float64 tolerance of the oracle."""
    wl = workloads.random_crossbar(m, n, B, seed)
    log(f"case currents only m={m} n={n} B={B}")
    I_full, _, (st0, _) = gpu_solve(wl.G, wl.V, wl.geom, "fp64")
    I_only, nv, (st1, _) = gpu_solve(wl.G, wl.V, wl.geom, "fp64", node_voltages=False)
    assert st0 == 0 and st1 == 0 and nv is None
    assert np.array_equal(I_full, I_only)
    e = rel_err(I_only, oracle.solve_workload(wl).currents)
    log(f"  max current rel err {e.max():.3e}")
    assert e.max() <= TOL_FP64


def test_partitioned_crossbar():
    """The partition experiment's reading: a 64 x 64 crossbar split into 32 x 32 tiles, each
    solved as a crossbar of its own (the paper's model, 5-ohm segments), column currents of a
    tile column summed.  Library tiles against oracle tiles."""
    rng = np.random.default_rng(2562)
    M, s, B, r = 64, 32, 3, 5.0
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (M, M)))
    V = rng.uniform(0.0, 0.5, (B, M))
    geom = workloads.Geometry(s, s, r, r, r, r)
    log(f"case partition {M}x{M} into {s}x{s}")
    I = np.zeros((B, M))
    I_ref = np.zeros((B, M))
    for a in range(M // s):
        for b in range(M // s):
            Gt = np.ascontiguousarray(G[a * s:(a + 1) * s, b * s:(b + 1) * s])
            Vt = np.ascontiguousarray(V[:, a * s:(a + 1) * s])
            It, _, (st, _) = gpu_solve(Gt, Vt, geom, "fp64", node_voltages=False)
            assert st == 0
            I[:, b * s:(b + 1) * s] += It
            I_ref[:, b * s:(b + 1) * s] += oracle.solve(Gt, Vt, r, r, r, r).currents
    e = rel_err(I, I_ref)
    log(f"  max rel err {e.max():.3e}")
    assert e.max() <= TOL_FP64
