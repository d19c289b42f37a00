"""GPU parity of the transfer-matrix shortcut (xbar_transfer, xbar_transfer_apply).

The nodal system of Sec. II.A is linear in the source voltages, so the output
currents of any batch are I = V T, with T[i][j] the current of bit line j for
1 V on word line i and 0 V on the others.  The oracle's T is its own solve with
identity input vectors (pinned by the CPU superposition tests); the oracle's
currents for V check the product.  Tolerances: 1e-10 per-vector relative error
in float64 (the solver's), 1e-9 for the float32 + refinement mode.  The product
kernel alone is checked against the float64 matrix product within its rounding
bound, 2 m eps (|V| |T|) per element.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import GOLDEN, TOL_FP64, TOL_IR, log, rel_err

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def _plan(wl, precision="fp64", max_batch=None):
    import paper_2410_19993_amd as xb
    g = wl.geom
    m, n = wl.G.shape
    return xb.Plan(m, n, g.r_wl, g.r_bl, g.r_src, g.r_sense, precision,
                   max_batch=max_batch or wl.V.shape[0])


def _oracle_T(wl):
    g = wl.geom
    m = wl.G.shape[0]
    return oracle.solve(wl.G, np.eye(m), g.r_wl, g.r_bl, g.r_src, g.r_sense).currents


@pytest.mark.parametrize("name,precision,max_batch", [
    ("c1", "fp64", None), ("ragged", "fp64", None), ("ragged", "fp64", 7),
    ("tall", "fp64", 64), ("c1", "fp32_ir", None), ("ragged", "fp32_ir", 5),
    ("c1", "fp64", 64), ("ragged", "fp64", 64), ("tall", "fp64", 128), ("m1", "fp64", 64),
    ("m2", "fp64", 64), ("m3", "fp64", 70), ("wide", "fp64", 256), ("ragged", "fp32_ir", 64)])
def test_transfer_matches_oracle(name, precision, max_batch):
    """T against the oracle's unit-input currents; V T against the oracle's currents.
    Float64 plans whose max_batch (rounded up to 16) reaches the padded block size n_p
    build T by block recurrences on the factorization; the others, and the refinement
    mode, solve the unit inputs, in several batches when max_batch < m (the last one
    ragged)."""
    import torch
    wl = {"c1": workloads.c1,
          "ragged": lambda: workloads.random_crossbar(37, 45, 19, 41, r_wl=1.5, r_bl=3.0,
                                                      r_src=40.0, r_sense=60.0),
          "tall": lambda: workloads.random_crossbar(150, 70, 33, 42),
          "m1": lambda: workloads.random_crossbar(1, 20, 4, 61),
          "m2": lambda: workloads.random_crossbar(2, 33, 4, 62),
          "m3": lambda: workloads.random_crossbar(3, 64, 4, 63),
          "wide": lambda: workloads.random_crossbar(21, 200, 9, 64, r_wl=1.0, r_bl=4.0)}[name]()
    m, n = wl.G.shape
    tol = TOL_FP64 if precision == "fp64" else TOL_IR
    log(f"case transfer {name} m={m} n={n} {precision} max_batch={max_batch}")
    with _plan(wl, precision, max_batch) as p:
        p.assemble(torch.from_numpy(wl.G).cuda())
        p.factor()
        T = p.transfer()
        V = torch.from_numpy(np.ascontiguousarray(wl.V)).cuda()
        I = p.transfer_apply(T, V)
        st, _ = p.info()
    assert st == 0
    T_ref = _oracle_T(wl)
    eT = rel_err(T.cpu().numpy(), T_ref)
    eI = rel_err(I.cpu().numpy(), oracle.solve_workload(wl).currents)
    log(f"  T rel err {eT.max():.3e}, V T rel err {eI.max():.3e}")
    assert eT.max() <= tol and eI.max() <= tol


def test_transfer_c3_full_size():
    """512 x 512 crossbar, 4096 input vectors, r = 2.5 ohm: V T on the seeded 256-vector
    subset against the oracle's stored currents, and on every vector against the plan's
    own substitution sweeps."""
    import torch
    wl = workloads.c3(r=2.5)
    log("case transfer c3 512x512 B=4096 r=2.5")
    ref = np.load(f"{GOLDEN}/c3_r2.5_currents.npy")
    with _plan(wl) as p:
        p.assemble(torch.from_numpy(wl.G).cuda())
        p.factor()
        V = torch.from_numpy(np.ascontiguousarray(wl.V)).cuda()
        p.solve_batch(V)
        I_solve = p.currents().cpu().numpy()
        T = p.transfer()
        I = p.transfer_apply(T, V).cpu().numpy()
        st, _ = p.info()
    assert st == 0
    e = rel_err(I[workloads.c3_subset()], ref)
    e_all = rel_err(I, I_solve)
    log(f"  subset rel err {e.max():.3e}; against the sweeps {e_all.max():.3e}")
    assert e.max() <= TOL_FP64 and e_all.max() <= TOL_FP64


def test_transfer_call_order():
    """xbar_transfer needs a factorization, drops the last solved batch, and leaves the
    factorization in place: a solve after it gives the same bits as before."""
    import torch

    from paper_2410_19993_amd import _lib
    wl = workloads.random_crossbar(20, 30, 9, 43)
    log("case transfer call order m=20 n=30 B=9")
    with _plan(wl) as p:
        T = torch.empty((20, 30), dtype=torch.float64, device="cuda")
        with pytest.raises(_lib.XbarError) as ex:
            p.transfer(T)
        assert ex.value.status == _lib.XBAR_ERR_STATE
        p.assemble(torch.from_numpy(wl.G).cuda())
        with pytest.raises(_lib.XbarError) as ex:
            p.transfer(T)
        assert ex.value.status == _lib.XBAR_ERR_STATE
        p.factor()
        V = torch.from_numpy(np.ascontiguousarray(wl.V)).cuda()
        p.solve_batch(V)
        I0 = p.currents().cpu().numpy()
        p.transfer(T)
        out = torch.empty((9, 30), dtype=torch.float64, device="cuda")
        assert _lib.lib().xbar_currents(p._plan, _lib._ptr(out)) == _lib.XBAR_ERR_STATE
        p.solve_batch(V)
        I1 = p.currents().cpu().numpy()
        st, _ = p.info()
    assert st == 0 and np.array_equal(I0, I1)


@pytest.mark.parametrize("B,m,n,shift", [
    (1, 1, 1, 0), (3, 5, 7, 0), (130, 17, 65, 0), (129, 34, 62, 0), (129, 34, 62, 1),
    (1024, 20, 64, 0), (200, 33, 130, 0), (257, 1000, 130, 0), (4096, 512, 512, 0),
    (4095, 512, 511, 1), (5000, 64, 1, 0)])
def test_apply_product_shapes(B, m, n, shift):
    """The product kernel alone on random signed operands: ragged rows, columns and
    contraction chunks, one and several launches' worth of row panels (XCD-grouped when
    they divide by 8), and (shift = 1) operands that start 8 bytes past a 16-byte boundary."""
    import torch
    log(f"case apply B={B} m={m} n={n} shift={shift}")
    rng = np.random.default_rng(B * 7 + m * 3 + n)
    Vh = rng.standard_normal((B, m))
    Th = rng.standard_normal((m, n))
    Vs = torch.zeros(B * m + 2, dtype=torch.float64, device="cuda")
    Ts = torch.zeros(m * n + 2, dtype=torch.float64, device="cuda")
    V = Vs[shift:shift + B * m].view(B, m)
    T = Ts[shift:shift + m * n].view(m, n)
    V.copy_(torch.from_numpy(Vh))
    T.copy_(torch.from_numpy(Th))
    wl = workloads.random_crossbar(m, n, 1, 44)
    with _plan(wl, max_batch=1) as p:
        I = p.transfer_apply(T, V).cpu().numpy()
    ref = Vh @ Th
    bound = 2 * m * EPS * (np.abs(Vh) @ np.abs(Th)) + 1e-300
    worst = float(np.max(np.abs(I - ref) / bound))
    log(f"  max error / rounding bound {worst:.3f}")
    assert np.all(np.isfinite(I)) and worst <= 1.0


def test_apply_rejects_bad_arguments():
    import torch

    from paper_2410_19993_amd import _lib
    wl = workloads.random_crossbar(8, 6, 4, 45)
    L = _lib.lib()
    log("case apply argument checks m=8 n=6")
    with _plan(wl) as p:
        buf = torch.from_numpy(np.random.default_rng(46).standard_normal(4 * 8 + 8 * 6)).cuda()
        V = buf[:32].view(4, 8)
        T = buf[32:].view(8, 6)
        I = torch.zeros((4, 6), dtype=torch.float64, device="cuda")
        assert L.xbar_transfer_apply(p._plan, _lib._ptr(T), _lib._ptr(V), 0, _lib._ptr(I)) == _lib.XBAR_ERR_ARG
        # I overlapping V, then T
        assert L.xbar_transfer_apply(p._plan, _lib._ptr(T), _lib._ptr(V), 4,
                                     _lib._ptr(buf[8:32])) == _lib.XBAR_ERR_ARG
        assert L.xbar_transfer_apply(p._plan, _lib._ptr(T), _lib._ptr(V), 4,
                                     _lib._ptr(buf[40:])) == _lib.XBAR_ERR_ARG
        assert L.xbar_transfer_apply(p._plan, _lib._ptr(T), _lib._ptr(V), 4, _lib._ptr(I)) == _lib.XBAR_OK
        st, _ = p.info()
    assert st == 0
    Vh, Th = V.cpu().numpy(), T.cpu().numpy()
    assert np.all(np.abs(I.cpu().numpy() - Vh @ Th) <= 2 * 8 * EPS * (np.abs(Vh) @ np.abs(Th)))
