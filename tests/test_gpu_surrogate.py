"""GPU parity of the surrogate's kernels (xbar_sg_*) against the float64 oracle
(oracle/surrogate.py), and a training run that must beat the ideal currents G^T V.

Tolerance of a float32 kernel: an output that sums K products is compared with the
oracle within 2 K u (sum of |terms|), u = 2^-24, the float32 unit roundoff times the
accumulation length; sum of |terms| is the oracle applied to absolute values."""
import numpy as np
import pytest

import oracle
from oracle import surrogate as osg
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _rand(rng, *shape):
    return _f32(rng.normal(size=shape))


def _lib():
    from paper_2410_19993_amd import _lib
    return _lib


def _assert_within(got, ref, absref, K, what):
    bound = 2.0 * K * U32 * absref + 1e-30
    err = np.abs(got - ref)
    worst = float((err / bound).max())
    log(f"  {what}: max error / bound {worst:.3f}")
    assert np.all(err <= bound), what


CONV_CASES = [(2, 13, 17, 5, 7), (1, 20, 33, 32, 32), (3, 1, 1, 1, 1), (2, 16, 16, 32, 1), (1, 5, 40, 3, 32)]


@pytest.mark.parametrize("B,H,W,C,O", CONV_CASES)
@pytest.mark.parametrize("relu", [False, True])
def test_conv_forward(B, H, W, C, O, relu):
    import torch
    rng = np.random.default_rng(B * 1000 + H * 10 + C + O + relu)
    x, w, b = _rand(rng, B, C, H, W), _rand(rng, O, C, 3, 3), _rand(rng, O)
    log(f"case conv forward B={B} H={H} W={W} C={C} O={O} relu={relu}")
    y = torch.empty((B, O, H, W), dtype=torch.float32, device="cuda")
    _lib().xbar_sg_conv_forward(B, H, W, C, O, relu, _t(x, torch.float32), _t(w, torch.float32),
                                _t(b, torch.float32), y)
    got = y.cpu().numpy().astype(np.float64)
    ref = osg.conv2d(x, w, b)
    absref = osg.conv2d(np.abs(x), np.abs(w), np.abs(b))
    if relu:
        ref = np.maximum(ref, 0.0)
        got_neg = got[ref == 0.0]
        assert np.all(got_neg >= 0.0)
    _assert_within(got, ref, absref, C * 9 + 1, "conv forward")


@pytest.mark.parametrize("B,H,W,C,O", CONV_CASES)
@pytest.mark.parametrize("masked", [False, True])
@pytest.mark.parametrize("xmasked", [False, True])
def test_conv_backward_data(B, H, W, C, O, masked, xmasked):
    import torch
    rng = np.random.default_rng(7 + B * 1000 + H * 10 + C + O + masked + 2 * xmasked)
    g, w = _rand(rng, B, O, H, W), _rand(rng, O, C, 3, 3)
    ymask = _f32(np.maximum(rng.normal(size=(B, O, H, W)), 0.0)) if masked else None
    xmask = _f32(np.maximum(rng.normal(size=(B, C, H, W)), 0.0)) if xmasked else None
    log(f"case conv backward data B={B} H={H} W={W} C={C} O={O} masked={masked} xmasked={xmasked}")
    gx = torch.empty((B, C, H, W), dtype=torch.float32, device="cuda")
    _lib().xbar_sg_conv_backward_data(B, H, W, C, O, _t(g, torch.float32),
                                      None if ymask is None else _t(ymask, torch.float32), _t(w, torch.float32), gx,
                                      xmask=None if xmask is None else _t(xmask, torch.float32))
    gm = g * (ymask > 0) if masked else g
    ref = osg.conv2d_grad_input(gm, w)
    absref = osg.conv2d_grad_input(np.abs(gm), np.abs(w))
    if xmasked:
        ref, absref = ref * (xmask > 0), absref * (xmask > 0)
    _assert_within(gx.cpu().numpy().astype(np.float64), ref, absref, O * 9, "conv backward data")


@pytest.mark.parametrize("B,H,W,C,O", CONV_CASES + [(40, 64, 64, 3, 4), (3, 50, 37, 2, 5)])
@pytest.mark.parametrize("masked", [False, True])
def test_conv_backward_weight(B, H, W, C, O, masked):
    """Includes a shape with more 16 x 16 tiles (640) than partial-sum workgroups (512)."""
    import torch
    rng = np.random.default_rng(11 + B * 1000 + H * 10 + C + O + masked)
    x, g = _rand(rng, B, C, H, W), _rand(rng, B, O, H, W)
    ymask = _f32(np.maximum(rng.normal(size=(B, O, H, W)), 0.0)) if masked else None
    log(f"case conv backward weight B={B} H={H} W={W} C={C} O={O} masked={masked}")
    L = _lib()
    work = torch.empty(L.xbar_sg_workspace_floats(C, O), dtype=torch.float32, device="cuda")
    gw = torch.empty((O, C, 3, 3), dtype=torch.float32, device="cuda")
    gb = torch.empty(O, dtype=torch.float32, device="cuda")
    L.xbar_sg_conv_backward_weight(B, H, W, C, O, _t(x, torch.float32), _t(g, torch.float32),
                                   None if ymask is None else _t(ymask, torch.float32), gw, gb, work)
    gm = g * (ymask > 0) if masked else g
    rw, rb = osg.conv2d_grad_weight(x, gm)
    aw, ab = osg.conv2d_grad_weight(np.abs(x), np.abs(gm))
    K = B * H * W
    _assert_within(gw.cpu().numpy().astype(np.float64), rw, aw, K, "weight gradient")
    _assert_within(gb.cpu().numpy().astype(np.float64), rb, ab, K, "bias gradient")


def test_features_readout_predict_adam():
    import torch
    rng = np.random.default_rng(21)
    B, m, n = 3, 9, 14
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (B, m, n)))
    V = rng.uniform(0, 0.5, (B, m))
    r = np.array([1.0, 2.75, 5.0])
    L = _lib()
    log("case features, readout + loss, prediction, Adam")
    X = torch.empty((B, 7, m, n), dtype=torch.float32, device="cuda")
    L.xbar_sg_features(B, m, n, _t(G), _t(V), _t(r), X)
    ref = osg.features(G, V, r)
    assert np.allclose(X.cpu().numpy(), ref, rtol=2 * U32, atol=2 * U32 * 4)

    Y = _rand(rng, B, 2, m, n)
    delta = rng.normal(scale=0.1, size=(B, n))
    gY = torch.empty((B, 2, m, n), dtype=torch.float32, device="cuda")
    err2 = torch.empty((B, 2), dtype=torch.float64, device="cuda")
    L.xbar_sg_readout_loss(B, m, n, _t(Y, torch.float32), _t(delta), osg.LAM, gY, err2)
    loss, est_loss, dY = osg.loss_and_grad(Y, delta)
    e2 = err2.cpu().numpy().sum(axis=0) / (B * n)
    assert e2[0] == pytest.approx(loss, rel=1e-12) and e2[1] == pytest.approx(est_loss, rel=1e-12)
    assert np.allclose(gY.cpu().numpy(), dY, rtol=2 * U32, atol=0)

    I = torch.empty((B, n), dtype=torch.float64, device="cuda")
    est = torch.empty((B, n), dtype=torch.float64, device="cuda")
    L.xbar_sg_predict(B, m, n, _t(Y, torch.float32), _t(G), _t(V), I, est)
    refI = osg.ideal_currents(G, V) * (1.0 + osg.readout(Y))
    assert np.allclose(I.cpu().numpy(), refI, rtol=1e-12, atol=0)
    assert np.allclose(est.cpu().numpy(), osg.estimate(Y), rtol=1e-12, atol=0)

    p, g = _rand(rng, 1000), _rand(rng, 1000)
    m1, m2 = np.zeros(1000), np.zeros(1000)
    pd, gd = _t(p, torch.float32), _t(g, torch.float32)
    m1d, m2d = torch.zeros(1000, device="cuda"), torch.zeros(1000, device="cuda")
    for t in range(1, 4):
        L.xbar_sg_adam(pd, gd, m1d, m2d, 1e-2, 0.9, 0.999, 1e-8, t)
        p, m1, m2 = osg.adam_step(p, g, m1, m2, t, 1e-2)
    assert np.allclose(pd.cpu().numpy(), p, rtol=0, atol=1e-6)


def test_network_gradients_and_update_match_oracle():
    """Surrogate.train_step on a five-layer network: every entry of every gradient
    equals the oracle's backward pass, evaluated at the network's own forward
    activations (read back from the GPU, so both sides apply the same ReLU masks),
    within a float32 bound derived from the accumulation lengths:

      dY   = the readout kernel's loss gradient: float64 arithmetic rounded to float32,
             |error| <= u |dY|;
      g_l  = the gradient at layer l's output, formed by the input-gradient kernels of
             the layers above, each a sum of 9 O_k products: relative error
             gamma_l = sum_{k > l} (2 * 9 O_k + 1) u of the same chain in absolute values;
      dW_l = a sum of B m n products of x and g_l: gamma_l + (2 B m n + 1) u, again
             relative to the absolute-value chain.

    The absolute-value chain is the oracle's backward pass applied to |W|, |x| and
    |dY| (first order in u).  The new weights must equal the oracle's Adam step."""
    import torch

    import paper_2410_19993_amd.surrogate as sgm
    rng = np.random.default_rng(31)
    B, m, n = 4, 12, 19
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (B, m, n)))
    V = rng.uniform(0, 0.5, (B, m))
    r = rng.uniform(1, 5, B)
    delta = rng.normal(scale=0.05, size=(B, n))
    net = sgm.Surrogate(channels=8, seed=3, lr=1e-3, zero_last=False, depth=5, precision="fp32")
    params = [(w.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)) for w, b in net.layers()]
    log("case network gradients element by element, channels 8, depth 5, B=4 12x19")
    loss = net.train_step(_t(G), _t(V), _t(r), _t(delta))
    L = len(params)
    acts = [net.X[:B].cpu().numpy().astype(np.float64)] + \
           [a[:B].cpu().numpy().astype(np.float64) for a in net.acts] + [net.Y[:B].cpu().numpy().astype(np.float64)]
    ref_loss, ref_est, dY = osg.loss_and_grad(acts[-1], delta)
    assert loss[0] == pytest.approx(ref_loss, rel=1e-6) and loss[1] == pytest.approx(ref_est, rel=1e-6)
    grads = osg.backward(params, acts, dY)
    absg = osg.backward([(np.abs(w), np.abs(b)) for w, b in params], [np.abs(a) for a in acts], np.abs(dY))
    dims = net.dims
    gv = net._views(net.grads)
    worst = 0.0
    for k in range(L):
        gamma = sum((2 * 9 * dims[j + 1] + 1) * U32 for j in range(k + 1, L)) + U32      # g_k, incl. dY
        gamma_w = gamma + (2 * B * m * n + 1) * U32
        for part in range(2):
            got = gv[k][part].cpu().numpy().astype(np.float64).reshape(grads[k][part].shape)
            bound = gamma_w * absg[k][part] + 1e-30
            err = np.abs(got - grads[k][part])
            worst = max(worst, float((err / bound).max()))
            assert np.all(err <= bound), (k, part, float((err / bound).max()))
    log(f"  max error / bound over all gradient entries {worst:.3f}")
    new = [(w.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)) for w, b in net.layers()]
    for k in range(L):
        for part in range(2):
            g = gv[k][part].cpu().numpy().astype(np.float64).reshape(params[k][part].shape)
            p1, _, _ = osg.adam_step(params[k][part], g, 0.0, 0.0, 1, 1e-3)
            assert np.allclose(new[k][part], p1, rtol=0, atol=2e-6), (k, part)


def test_training_beats_ideal_currents_and_flags_its_errors():
    """Trained on oracle-labelled 16 x 16 crossbars, the surrogate's currents on held-out
    maps are closer to the exact currents than G^T V is (by at least a factor 2 in mean
    relative error).  Its error estimate ranks its errors: the samples it flags (the
    largest fifth of the estimates) have larger actual errors on average than the rest,
    and predict_checked returns the exact currents for them."""
    import torch

    import paper_2410_19993_amd.surrogate as sgm
    rng = np.random.default_rng(41)
    m = n = 16
    vectors = 8

    def data(maps):
        G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (maps, m, n)))
        r = rng.choice(np.arange(1.0, 5.01, 0.5), maps)
        V = rng.uniform(0, 0.5, (maps, vectors, m))
        I = np.stack([oracle.solve(G[k], V[k], r[k], r[k], 50.0, 50.0).currents for k in range(maps)])
        S = maps * vectors
        Gs = np.repeat(G, vectors, axis=0)
        return Gs, V.reshape(S, m), np.repeat(r, vectors), I.reshape(S, n)

    Gt, Vt, rt, It = data(48)
    Gh, Vh, rh, Ih = data(16)
    dt = osg.targets(It, Gt, Vt)
    net = sgm.Surrogate(channels=16, seed=1, lr=3e-3)
    Gd, Vd, rd, dd = _t(Gt), _t(Vt), _t(rt), _t(dt)
    log("case surrogate training: 384 samples of 16 x 16, 600 steps of 32")
    g = torch.Generator().manual_seed(5)
    for step in range(600):
        idx = torch.randint(0, len(Gt), (32,), generator=g).cuda()
        net.train_step(Gd[idx].contiguous(), Vd[idx].contiguous(), rd[idx].contiguous(), dd[idx].contiguous(),
                       want_loss=False)
    est = torch.empty((len(Gh), n), dtype=torch.float64, device="cuda")
    I_sg = net.predict(_t(Gh), _t(Vh), _t(rh), est=est).cpu().numpy()
    I0 = osg.ideal_currents(Gh, Vh)
    err = np.abs(I_sg - Ih) / np.abs(Ih)
    e_sg = float(err.mean())
    e_0 = float(np.mean(np.abs(I0 - Ih) / np.abs(Ih)))
    log(f"  held-out mean relative error: surrogate {e_sg:.4f}, G^T V {e_0:.4f}")
    assert np.all(np.isfinite(I_sg))
    assert e_sg < 0.5 * e_0

    worst_est = est.cpu().numpy().max(axis=1)
    worst_err = err.max(axis=1)
    tol = float(np.quantile(worst_est, 0.8))
    hi = worst_est > tol
    log(f"  flagged {hi.sum()} of {len(hi)}: mean worst error {worst_err[hi].mean():.4f} flagged, "
        f"{worst_err[~hi].mean():.4f} not flagged")
    assert hi.any() and (~hi).any()
    assert worst_err[hi].mean() > worst_err[~hi].mean()
    I_chk, flagged = net.predict_checked(_t(Gh), _t(Vh), _t(rh), tol=tol)
    assert np.array_equal(flagged, hi)
    I_chk = I_chk.cpu().numpy()
    assert np.abs(I_chk[hi] - Ih[hi]).max() <= 1e-10 * np.abs(Ih[hi]).max()
    assert np.array_equal(I_chk[~hi], I_sg[~hi])
    I_ir, flagged_ir = net.predict_checked(_t(Gh), _t(Vh), _t(rh), tol=tol, precision="fp32_ir")
    I_ir = I_ir.cpu().numpy()
    assert np.array_equal(flagged_ir, hi)
    assert np.abs(I_ir[hi] - Ih[hi]).max() <= 1e-9 * np.abs(Ih[hi]).max()
    net.close()


def test_surrogate_rejects_bad_inputs_before_launching():
    """Wrong dtypes, shapes or layouts raise on the host: a float32 G of the right
    shape would otherwise be read as float64, past its end."""
    import torch

    import paper_2410_19993_amd.surrogate as sgm
    net = sgm.Surrogate(channels=4, seed=0)
    B, m, n = 2, 5, 6
    G = torch.full((B, m, n), 1e-5, dtype=torch.float64, device="cuda")
    V = torch.zeros((B, m), dtype=torch.float64, device="cuda")
    r = torch.full((B,), 2.0, dtype=torch.float64, device="cuda")
    d = torch.zeros((B, n), dtype=torch.float64, device="cuda")
    log("case surrogate argument checks")
    with pytest.raises(ValueError):
        net.predict(G.float(), V, r)
    with pytest.raises(ValueError):
        net.predict(G, V[:, :4].contiguous(), r)
    with pytest.raises(ValueError):
        net.predict(G.transpose(1, 2), V, r)
    with pytest.raises(ValueError):
        net.train_step(G, V, r, d[:, :3].contiguous())
    with pytest.raises(ValueError):
        net.predict(G, V, r, est=torch.empty((B, n), dtype=torch.float32, device="cuda"))
    assert net.predict(G, V, r).shape == (B, n)


def test_checkpoint_round_trip():
    """state() / load(): a restored network predicts the same bits and trains on to the
    same weights as the original."""
    import torch

    import paper_2410_19993_amd.surrogate as sgm
    rng = np.random.default_rng(51)
    B, m, n = 4, 10, 12
    G = _t(np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (B, m, n))))
    V = _t(rng.uniform(0, 0.5, (B, m)))
    r = _t(rng.uniform(1, 5, B))
    d = _t(rng.normal(scale=0.05, size=(B, n)))
    log("case surrogate checkpoint round trip")
    a = sgm.Surrogate(channels=6, seed=2, lr=1e-3)
    for _ in range(5):
        a.train_step(G, V, r, d, want_loss=False)
    a.kappa = 3.5
    st = a.state()
    b = sgm.Surrogate(channels=6, seed=99, lr=1e-3)
    b.load(st)
    assert b.t == a.t and b.kappa == 3.5
    assert torch.equal(a.predict(G, V, r), b.predict(G, V, r))
    a.train_step(G, V, r, d, want_loss=False)
    b.train_step(G, V, r, d, want_loss=False)
    assert torch.equal(a.params, b.params)
    with pytest.raises(ValueError):
        sgm.Surrogate(channels=5).load(st)


@pytest.mark.parametrize("method,maps,vectors,chunk", [("lanes", 3, 2, 1024), ("tiles", 3, 2, 1024),
                                                       ("tiles", 11, 1, 4)])
def test_solver_dataset_labels_match_the_oracle(method, maps, vectors, chunk):
    """solver_dataset: every sample's currents equal the oracle's for its map, input
    vector and segment resistance, and delta = (I - G^T V) / G^T V; through PlanLanes
    and through the batched tile pipeline (11 maps in calls of at most 4: ragged)."""
    import paper_2410_19993_amd.surrogate as sgm
    log(f"case solver dataset ({method}): {maps} maps x {vectors} vectors of 16 x 16, chunks of {chunk}")
    ds = sgm.solver_dataset(maps, vectors, 16, 16, seed=7, r_levels=[1.5, 4.0], method=method, chunk=chunk)
    G, r, V, I = (x.cpu().numpy() for x in (ds.G, ds.r, ds.V, ds.I))
    S = maps * vectors
    assert G.shape == (maps, 16, 16) and V.shape == (S, 16) and I.shape == (S, 16) and set(r) <= {1.5, 4.0}
    for s in range(S):
        k = s // vectors
        ref = oracle.solve(G[k], V[s:s + 1], r[k], r[k], 50.0, 50.0).currents[0]
        assert rel_err_vec(I[s], ref) <= 1e-10
    Gs = np.repeat(G, vectors, axis=0)
    assert np.allclose(ds.delta.cpu().numpy(), osg.targets(I, Gs, V), rtol=1e-12, atol=1e-15)


def rel_err_vec(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_predict_checked_sends_bad_inputs_to_the_solver():
    """A sample with a conductance that is not finite and positive, or a NaN input, gives
    non-finite features and a NaN estimate; predict_checked must not trust it (a NaN
    compares false against the tolerance): it goes to the exact solver, which reports the
    bad input instead of returning surrogate values.  Good samples stay trusted."""
    import torch

    import paper_2410_19993_amd.surrogate as sgm
    from paper_2410_19993_amd import _lib as L
    rng = np.random.default_rng(61)
    B, m, n = 6, 8, 10
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (B, m, n)))
    V = rng.uniform(0, 0.5, (B, m))
    r = np.full(B, 2.5)
    net = sgm.Surrogate(channels=4, seed=0)
    net.kappa = 1e-12                      # every good sample's estimate is far below tol
    Gb = G.copy()
    Gb[3, 2, 5] = 0.0
    log("case predict_checked with a zero conductance")
    with pytest.raises(L.XbarError) as ex:
        net.predict_checked(_t(Gb), _t(V), _t(r), tol=0.05)
    assert ex.value.status == L.XBAR_ERR_INPUT
    # a NaN input voltage: the sample is flagged and solved exactly (NaN in, NaN out),
    # never returned as a trusted surrogate value
    Vb = V.copy()
    Vb[4, 1] = np.nan
    log("case predict_checked with a NaN input voltage")
    out, flagged = net.predict_checked(_t(G), _t(Vb), _t(r), tol=0.05)
    assert flagged[4] and flagged.sum() == 1
    out, flagged = net.predict_checked(_t(G), _t(V), _t(r), tol=0.05)
    assert not flagged.any() and torch.isfinite(out).all()
    net.close()


def test_calibrate_skips_zero_current_samples():
    """A calibration set holding an all-zero input vector (exact currents 0, a relative
    error 0/0) must still give a finite, positive kappa."""
    import torch

    import paper_2410_19993_amd.surrogate as sgm
    rng = np.random.default_rng(62)
    maps, vectors, m, n = 3, 4, 8, 8
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (maps, m, n)))
    V = rng.uniform(0, 0.5, (maps * vectors, m))
    V[5] = 0.0
    r = np.full(maps, 2.0)
    I = np.stack([oracle.solve(G[k // vectors], V[k:k + 1], 2.0, 2.0, 50.0, 50.0).currents[0]
                  for k in range(maps * vectors)])
    ds = sgm.Dataset(_t(G), _t(r), _t(V), _t(I), vectors)
    net = sgm.Surrogate(channels=4, seed=1)
    log("case calibrate with a zero-input vector")
    kappa = net.calibrate(ds)
    log(f"  kappa {kappa:.4f}")
    assert np.isfinite(kappa) and kappa > 0


def test_train_step_with_few_channels_on_many_tiles():
    """channels < 7: the first layer (7 features -> C) needs the largest weight-gradient
    workspace; a batch of more tiles than partial-sum workgroups must train (the buffer
    was once sized for C -> C) and match the oracle's gradient of the first layer."""
    import paper_2410_19993_amd.surrogate as sgm
    rng = np.random.default_rng(63)
    B, m, n = 40, 64, 64                 # 40 x 16 = 640 tiles of 16 x 16
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (B, m, n)))
    V = rng.uniform(0, 0.5, (B, m))
    r = rng.uniform(1, 5, B)
    delta = rng.normal(scale=0.05, size=(B, n))
    net = sgm.Surrogate(channels=3, seed=4, zero_last=False, precision="fp32")
    params = [(w.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)) for w, b in net.layers()]
    log("case train_step channels 3 on 640 tiles")
    net.train_step(_t(G), _t(V), _t(r), _t(delta))
    acts = [net.X[:B].cpu().numpy().astype(np.float64)] + \
           [a[:B].cpu().numpy().astype(np.float64) for a in net.acts] + [net.Y[:B].cpu().numpy().astype(np.float64)]
    _, _, dY = osg.loss_and_grad(acts[-1], delta)
    ref = osg.backward(params, acts, dY)[0][0]
    got = net._views(net.grads)[0][0].cpu().numpy().astype(np.float64).reshape(ref.shape)
    assert np.all(np.isfinite(got))
    assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)


def test_targets_calibration_ratios_and_routing_kernels():
    """xbar_sg_targets, xbar_sg_calib_ratios and xbar_sg_route against numpy on crafted
    inputs: zero exact currents (left out), NaN and zero estimates, a non-finite
    prediction, a negative conductance and a NaN input."""
    import torch

    from paper_2410_19993_amd import _lib
    rng = np.random.default_rng(91)
    B, m, n = 7, 5, 6
    I = rng.uniform(1e-6, 1e-4, (B, n))
    I[2, :] = 0.0                                # no live column: NaN ratio
    I[3, 1] = 0.0                                # one dead column
    I0 = I * rng.uniform(1.2, 2.0, (B, n))
    Ip = I * (1 + rng.normal(scale=1e-3, size=(B, n)))
    est = rng.uniform(1e-4, 5e-3, (B, n))
    est[4, 2] = np.nan                           # NaN estimate: NaN ratio
    est[5, :] = 0.0                              # zero estimate: NaN ratio
    Ip[6, 3] = np.inf                            # non-finite prediction
    G = rng.uniform(1e-6, 1e-4, (B, m, n))
    G[1, 2, 3] = -1e-5                           # bad conductance
    V = rng.uniform(0, 0.5, (B, m))
    V[0, 4] = np.nan                             # bad input
    t = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()
    Id, I0d, Ipd, ed = t(I), t(I0), t(Ip), t(est)

    delta = torch.empty((B, n), dtype=torch.float64, device="cuda")
    _lib.xbar_sg_targets(B, n, Id, I0d, delta)
    with np.errstate(invalid="ignore"):                      # 0 / 0 in the dead row, NaN on both sides
        np.testing.assert_array_equal(delta.cpu().numpy(), (I - I0) / I0)

    ratio = torch.empty(B, dtype=torch.float64, device="cuda")
    _lib.xbar_sg_calib_ratios(B, n, Ipd, Id, ed, ratio)
    got = ratio.cpu().numpy()
    for b in range(B):
        live = I[b] != 0
        if not live.any() or not np.all(np.isfinite(est[b])) or est[b].max() <= 0:
            assert np.isnan(got[b]), b
            continue
        worst = (np.abs(Ip[b] - I[b])[live] / np.abs(I[b])[live]).max()
        if not np.isfinite(worst):
            assert np.isnan(got[b]), b
            continue
        assert got[b] == worst / est[b].max(), b

    flag = torch.empty(B, dtype=torch.int32, device="cuda")
    kappa, tol = 2.0, 0.0098
    _lib.xbar_sg_route(B, m, n, t(G), t(V), Ipd, ed, kappa, tol, flag)
    want = []
    for b in range(B):
        ok = (np.all(np.isfinite(est[b])) and kappa * est[b].max() <= tol and np.all(np.isfinite(Ip[b])) and
              np.all(np.isfinite(G[b])) and np.all(G[b] > 0) and np.all(np.isfinite(V[b])))
        want.append(0 if ok else 1)
    log(f"case surrogate host kernels: flags {flag.cpu().numpy().tolist()}, want {want}")
    assert flag.cpu().numpy().tolist() == want
    assert 0 in want and want[0] == 1 and want[1] == 1 and want[6] == 1


def test_routing_and_calibration_keep_a_nan_in_an_early_column():
    """With more columns than threads each thread folds several columns: a NaN estimate
    or error in column 0 must survive the finite columns 256 and later (a plain fmax
    would drop it): the sample goes to the solver and its calibration ratio is NaN."""
    import torch

    from paper_2410_19993_amd import _lib
    rng = np.random.default_rng(93)
    B, m, n = 3, 4, 300
    I = rng.uniform(1e-6, 1e-4, (B, n))
    Ip = I * (1 + rng.normal(scale=1e-4, size=(B, n)))
    est = rng.uniform(1e-5, 1e-4, (B, n))
    est[0, 0] = np.nan                           # estimate NaN in the thread's first column
    Ip[1, 0] = np.nan                            # prediction NaN in the thread's first column
    G = rng.uniform(1e-6, 1e-4, (B, m, n))
    V = rng.uniform(0, 0.5, (B, m))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ratio = torch.empty(B, dtype=torch.float64, device="cuda")
    _lib.xbar_sg_calib_ratios(B, n, t(Ip), t(I), t(est), ratio)
    got = ratio.cpu().numpy()
    log(f"case NaN in column 0 of {n}: ratios {got.tolist()}")
    assert np.isnan(got[0]) and np.isnan(got[1]) and np.isfinite(got[2])
    flag = torch.empty(B, dtype=torch.int32, device="cuda")
    _lib.xbar_sg_route(B, m, n, t(G), t(V), t(Ip), t(est), 2.0, 0.01, flag)
    assert flag.cpu().numpy().tolist() == [1, 1, 0]
