"""The allocation-free weight gradient (xbar_sg_conv_backward_weight_noalloc) against
the workspace form (xbar_sg_conv_backward_weight) through the C ABI: the same bits,
on two calls in a row whose second input is smaller (the library's device array keeps
the first call's partial sums; the second must not read them), and within the float32
bound of the oracle's weight gradient."""
import ctypes

import numpy as np
import pytest

from oracle import surrogate as osg
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _call_both(B, H, W, C, O, seed):
    import torch

    from paper_2410_19993_amd import _lib
    L = _lib.lib()
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(B, C, H, W)).astype(np.float32)
    gy = rng.normal(size=(B, O, H, W)).astype(np.float32)
    xd, gd = _t(x), _t(gy)
    outs = []
    for noalloc in (False, True):
        gw = torch.full((O * C * 9,), float("nan"), dtype=torch.float32, device="cuda")
        gb = torch.full((O,), float("nan"), dtype=torch.float32, device="cuda")
        s = torch.cuda.current_stream().cuda_stream
        if noalloc:
            st = L.xbar_sg_conv_backward_weight_noalloc(B, H, W, C, O, _lib._ptr(xd), _lib._ptr(gd), None,
                                                         _lib._ptr(gw), _lib._ptr(gb), ctypes.c_void_p(s))
        else:
            work = torch.empty(_lib.xbar_sg_workspace_floats(C, O), dtype=torch.float32, device="cuda")
            st = L.xbar_sg_conv_backward_weight(B, H, W, C, O, _lib._ptr(xd), _lib._ptr(gd), None, _lib._ptr(gw),
                                                _lib._ptr(gb), _lib._ptr(work), work.numel(), ctypes.c_void_p(s))
        assert st == _lib.XBAR_OK
        torch.cuda.synchronize()
        outs.append((gw.cpu().numpy(), gb.cpu().numpy()))
    ref_w, ref_b = osg.conv2d_grad_weight(x.astype(np.float64), gy.astype(np.float64))
    abs_w, abs_b = osg.conv2d_grad_weight(np.abs(x).astype(np.float64), np.abs(gy).astype(np.float64))
    return outs, (ref_w.reshape(-1), ref_b), (abs_w.reshape(-1), abs_b), B * H * W


@pytest.mark.parametrize("first,second", [((40, 64, 64, 32, 32), (3, 20, 17, 5, 7)),
                                          ((8, 33, 40, 7, 32), (1, 16, 16, 7, 32))])
def test_noalloc_weight_gradient_matches_workspace_form(first, second):
    for k, shape in enumerate((first, second)):
        log(f"case no-alloc weight gradient call {k}: B,H,W,C,O = {shape}")
        (ws, na), ref, absref, K = _call_both(*shape, seed=100 + k)
        assert np.array_equal(ws[0], na[0]) and np.array_equal(ws[1], na[1])
        for got, r, a in zip(na, ref, absref):
            bound = 2.0 * K * U32 * a + 1e-30
            assert np.all(np.abs(got - r) <= bound)
