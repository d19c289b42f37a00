"""The surrogate's convolutions on the bfloat16 matrix cores (xbar_sg_conv_*_bf16)
against the float64 oracle (oracle/surrogate.py) applied to the same operands
rounded to bfloat16.

The kernels round every operand (activations, gradients, weights) to bfloat16,
nearest with ties to even, and accumulate the exact products in float32.  So the
oracle's convolution of the bfloat16-rounded operands, in float64, differs from
the kernel only by the float32 accumulation: an output that sums K products is
within 2 (K + 1) u (sum of |terms|), u = 2^-24 (the + 1 covers the bias and the
final rounding), with sum of |terms| the oracle applied to absolute values.  Each
case also reports the error against the unrounded (float32) operands, which is
the bfloat16 rounding itself, about 2^-9 of the terms.
"""
import numpy as np
import pytest

from oracle import surrogate as osg
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def bf16(a):
    """float32 values rounded to the nearest bfloat16 (ties to even), as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _lib():
    from paper_2410_19993_amd import _lib
    return _lib


def _within(got, ref, absref, K, what):
    bound = 2.0 * (K + 1) * U32 * absref + 1e-30
    err = np.abs(got - ref)
    worst = float((err / bound).max())
    log(f"  {what}: max error / bound {worst:.3f}")
    assert np.all(err <= bound), what


CASES = [(2, 13, 17, 5, 7), (1, 20, 33, 32, 32), (3, 1, 1, 1, 1), (2, 16, 16, 32, 1), (1, 5, 40, 3, 32),
         (2, 40, 35, 7, 32), (1, 17, 16, 32, 2), (1, 33, 47, 24, 20)]


def test_bf16_rounding_helper():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 1.0 + 2 ** -7 + 2 ** -8], dtype=np.float32)
    r = bf16(x)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even gives 1; 1 + 3 2^-9 rounds up;
    # 1 + 3 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even gives 1 + 2^-6
    assert list(r) == [1.0, 1.0, 1.0 + 2 ** -7, -2.5, 1.0 + 2 ** -6]


@pytest.mark.parametrize("B,H,W,C,O", CASES)
@pytest.mark.parametrize("relu", [False, True])
def test_conv_forward_bf16(B, H, W, C, O, relu):
    import torch
    rng = np.random.default_rng(B * 1000 + H * 10 + C + O + relu + 7)
    x, w, b = _f32(rng.normal(size=(B, C, H, W))), _f32(rng.normal(size=(O, C, 3, 3))), _f32(rng.normal(size=O))
    log(f"case bf16 conv forward B={B} H={H} W={W} C={C} O={O} relu={relu}")
    y = torch.empty((B, O, H, W), dtype=torch.float32, device="cuda")
    _lib().xbar_sg_conv_forward(B, H, W, C, O, relu, _t(x), _t(w), _t(b), y, bf16=True)
    got = y.cpu().numpy().astype(np.float64)
    xb, wb = bf16(x), bf16(w)
    ref = osg.conv2d(xb, wb, b)
    absref = osg.conv2d(np.abs(xb), np.abs(wb), np.abs(b))
    if relu:
        ref = np.maximum(ref, 0.0)           # ReLU is 1-Lipschitz: the bound still holds
    _within(got, ref, absref, 9 * C, "forward")
    e32 = np.abs(got - (np.maximum(osg.conv2d(x, w, b), 0) if relu else osg.conv2d(x, w, b))).max() / absref.max()
    log(f"  against float32 operands: {e32:.2e} of the largest |terms| sum")


@pytest.mark.parametrize("B,H,W,C,O", CASES)
@pytest.mark.parametrize("masked", [False, True])
def test_conv_backward_data_bf16(B, H, W, C, O, masked):
    import torch
    rng = np.random.default_rng(B * 977 + H * 7 + C * 3 + O + masked)
    g, w = _f32(rng.normal(size=(B, O, H, W))), _f32(rng.normal(size=(O, C, 3, 3)))
    ymask = _f32(rng.normal(size=(B, O, H, W))) if masked else None
    xmask = _f32(rng.normal(size=(B, C, H, W))) if masked else None
    log(f"case bf16 conv input gradient B={B} H={H} W={W} C={C} O={O} masked={masked}")
    gx = torch.empty((B, C, H, W), dtype=torch.float32, device="cuda")
    _lib().xbar_sg_conv_backward_data(B, H, W, C, O, _t(g), _t(ymask) if masked else None, _t(w), gx,
                                      xmask=_t(xmask) if masked else None, bf16=True)
    got = gx.cpu().numpy().astype(np.float64)
    gm = g * (ymask > 0) if masked else g
    gb, wb = bf16(gm), bf16(w)
    ref = osg.conv2d_grad_input(gb, wb)
    absref = osg.conv2d_grad_input(np.abs(gb), np.abs(wb))
    if masked:
        ref = ref * (xmask > 0)
        absref = absref * (xmask > 0)
    _within(got, ref, absref, 9 * O, "input gradient")


@pytest.mark.parametrize("B,H,W,C,O", CASES + [(3, 64, 64, 32, 32)])
@pytest.mark.parametrize("masked", [False, True])
def test_conv_backward_weight_bf16(B, H, W, C, O, masked):
    import torch
    L = _lib()
    rng = np.random.default_rng(B * 31 + H + W * 5 + C + O * 11 + masked)
    x, g = _f32(rng.normal(size=(B, C, H, W))), _f32(rng.normal(size=(B, O, H, W)))
    ymask = _f32(rng.normal(size=(B, O, H, W))) if masked else None
    log(f"case bf16 conv weight gradient B={B} H={H} W={W} C={C} O={O} masked={masked}")
    gw = torch.empty((O, C, 3, 3), dtype=torch.float32, device="cuda")
    gbias = torch.empty((O,), dtype=torch.float32, device="cuda")
    work = torch.empty(L.xbar_sg_workspace_floats(C, O), dtype=torch.float32, device="cuda")
    L.xbar_sg_conv_backward_weight(B, H, W, C, O, _t(x), _t(g), _t(ymask) if masked else None, gw, gbias, work,
                                   bf16=True)
    gm = g * (ymask > 0) if masked else g
    xb, gmb = bf16(x), bf16(gm)
    ref_w, ref_b = osg.conv2d_grad_weight(xb, gmb)
    abs_w, abs_b = osg.conv2d_grad_weight(np.abs(xb), np.abs(gmb))
    K = B * H * W
    _within(gw.cpu().numpy().astype(np.float64), ref_w, abs_w, K, "weight gradient")
    _within(gbias.cpu().numpy().astype(np.float64), ref_b, abs_b, K, "bias gradient")


def test_bf16_network_trains_and_matches_fp32_forward():
    """The default (bfloat16) network: its forward pass agrees with the float32 kernels'
    within the bfloat16 rounding of four layers, and a few training steps lower the loss."""
    import torch

    import paper_2410_19993_amd.surrogate as sgm
    rng = np.random.default_rng(71)
    B, m, n = 6, 24, 20
    G = torch.from_numpy(np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (B, m, n)))).cuda()
    V = torch.from_numpy(rng.uniform(0, 0.5, (B, m))).cuda()
    r = torch.from_numpy(rng.uniform(1, 5, B)).cuda()
    d = torch.from_numpy(rng.normal(scale=0.05, size=(B, n))).cuda()
    a = sgm.Surrogate(channels=16, seed=5, zero_last=False, precision="bf16")
    f = sgm.Surrogate(channels=16, seed=5, zero_last=False, precision="fp32")
    ya, yf = a.forward(G, V, r).cpu().numpy(), f.forward(G, V, r).cpu().numpy()
    rel = np.abs(ya - yf).max() / np.abs(yf).max()
    log(f"case bf16 network: forward differs from float32 by {rel:.2e} of the largest output")
    assert rel < 0.05
    losses = [a.train_step(G, V, r, d)[0] for _ in range(30)]
    log(f"  loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert losses[-1] < 0.5 * losses[0]
