"""Error handling of the C ABI on a GPU: call order, bad inputs, sticky flags.

Every condition is forced from the host (bad arguments, out-of-order calls,
non-positive conductances); every kernel still runs to completion.
"""
import numpy as np
import pytest

import workloads
from paper_2410_19993_amd import _lib
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def _plan(m=8, n=8, max_batch=4):
    import torch  # noqa: F401
    return _lib.xbar_create(_lib.Geometry(m, n, 1.0, 1.0, 50.0, 50.0), 0, max_batch)


def test_call_order_state_machine():
    import torch
    L = _lib.lib()
    wl = workloads.random_crossbar(8, 8, 4, 1)
    G = torch.from_numpy(wl.G).cuda()
    V = torch.from_numpy(wl.V).cuda()
    I = torch.empty((4, 8), dtype=torch.float64, device="cuda")
    p = _plan()
    try:
        assert L.xbar_factor(p) == _lib.XBAR_ERR_STATE
        assert L.xbar_solve_batch(p, _lib._ptr(V), 4, None) == _lib.XBAR_ERR_STATE
        assert L.xbar_currents(p, _lib._ptr(I)) == _lib.XBAR_ERR_STATE
        assert L.xbar_assemble(p, _lib._ptr(G)) == _lib.XBAR_OK
        assert L.xbar_solve_batch(p, _lib._ptr(V), 4, None) == _lib.XBAR_ERR_STATE
        assert L.xbar_factor(p) == _lib.XBAR_OK
        assert L.xbar_factor(p) == _lib.XBAR_ERR_STATE          # factor needs a fresh assembly
        assert L.xbar_currents(p, _lib._ptr(I)) == _lib.XBAR_ERR_STATE
        assert L.xbar_solve_batch(p, _lib._ptr(V), 5, None) == _lib.XBAR_ERR_ARG   # > max_batch
        assert L.xbar_solve_batch(p, _lib._ptr(V), 0, None) == _lib.XBAR_ERR_ARG
        assert L.xbar_solve_batch(p, None, 4, None) == _lib.XBAR_ERR_ARG
        assert L.xbar_solve_batch(p, _lib._ptr(V), 4, None) == _lib.XBAR_OK
        assert L.xbar_currents(p, _lib._ptr(I)) == _lib.XBAR_OK
        st, info = _lib.xbar_get_info(p)
        assert st == _lib.XBAR_OK and info.state == 3 and info.last_batch == 4
        assert L.xbar_assemble(p, _lib._ptr(G)) == _lib.XBAR_OK  # re-assembly drops the factor
        assert L.xbar_solve_batch(p, _lib._ptr(V), 4, None) == _lib.XBAR_ERR_STATE
    finally:
        _lib.xbar_destroy(p)


@pytest.mark.parametrize("bad", [0.0, -1e-5, np.nan, np.inf])
def test_bad_conductance_sets_input_flag(bad):
    import torch
    L = _lib.lib()
    wl = workloads.random_crossbar(8, 8, 4, 2)
    Gb = wl.G.copy()
    Gb[3, 5] = bad
    log(f"case bad conductance {bad}")
    p = _plan()
    try:
        assert L.xbar_assemble(p, _lib._ptr(torch.from_numpy(Gb).cuda())) == _lib.XBAR_OK
        L.xbar_factor(p)
        st, info = _lib.xbar_get_info(p)
        assert st == _lib.XBAR_ERR_INPUT and info.device_error == _lib.XBAR_ERR_INPUT
        # a clean re-assembly clears the sticky flag
        assert L.xbar_assemble(p, _lib._ptr(torch.from_numpy(wl.G).cuda())) == _lib.XBAR_OK
        st, _ = _lib.xbar_get_info(p)
        assert st == _lib.XBAR_OK
    finally:
        _lib.xbar_destroy(p)


def test_python_front_end_raises():
    import torch

    import paper_2410_19993_amd as xb
    with pytest.raises(_lib.XbarError):
        xb.Plan(0, 4, 1.0, 1.0)
    with xb.Plan(4, 4, 1.0, 1.0, max_batch=2) as p:
        with pytest.raises(ValueError):
            p.assemble(torch.zeros((4, 4), dtype=torch.float32, device="cuda"))
        with pytest.raises(_lib.XbarError):
            p.factor()
