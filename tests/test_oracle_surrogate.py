"""Pins of the surrogate oracle (oracle/surrogate.py) against things other than itself:
brute-force loops, a library correlation, finite differences, adjoint identities,
Adam's closed-form first step and the zero-resistance limit of the circuit."""
import numpy as np
import pytest
from scipy.signal import correlate2d

import oracle
from oracle import surrogate as sg


def _conv_loops(x, w, b):
    B, C, H, W = x.shape
    O = w.shape[0]
    y = np.zeros((B, O, H, W))
    for bb in range(B):
        for o in range(O):
            for p in range(H):
                for q in range(W):
                    s = b[o]
                    for c in range(C):
                        for dy in range(3):
                            for dx in range(3):
                                yy, xx = p + dy - 1, q + dx - 1
                                if 0 <= yy < H and 0 <= xx < W:
                                    s += w[o, c, dy, dx] * x[bb, c, yy, xx]
                    y[bb, o, p, q] = s
    return y


def test_conv_matches_brute_force_loops():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 2, 3, 4))
    w = rng.normal(size=(3, 2, 3, 3))
    b = rng.normal(size=3)
    assert np.allclose(sg.conv2d(x, w, b), _conv_loops(x, w, b), rtol=0, atol=1e-13)


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(1, 3, 9, 7))
    w = rng.normal(size=(2, 3, 3, 3))
    b = np.array([0.5, -1.0])
    y = sg.conv2d(x, w, b)
    for o in range(2):
        ref = b[o] + sum(correlate2d(x[0, c], w[o, c], mode="same", boundary="fill") for c in range(3))
        assert np.allclose(y[0, o], ref, rtol=0, atol=1e-12)


def test_conv_adjoints():
    """<conv(x), g> = <x, grad_input(g)> = <w, grad_weight(x, g)> for a bias-free conv."""
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 4, 6, 5))
    w = rng.normal(size=(3, 4, 3, 3))
    g = rng.normal(size=(2, 3, 6, 5))
    lhs = float(np.sum(sg.conv2d(x, w, np.zeros(3)) * g))
    assert lhs == pytest.approx(float(np.sum(x * sg.conv2d_grad_input(g, w))), rel=1e-12)
    gw, gb = sg.conv2d_grad_weight(x, g)
    assert lhs == pytest.approx(float(np.sum(w * gw)), rel=1e-12)
    assert np.allclose(gb, g.sum(axis=(0, 2, 3)))


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(4)
    params = sg.init_params(channels=3, seed=5, depth=5)
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (2, 4, 5)))
    V = rng.uniform(0, 0.5, (2, 4))
    X = sg.features(G, V, np.array([2.0, 4.0]))
    delta = rng.normal(scale=0.1, size=(2, 5))

    def loss(ps, k):
        """Layers 0-3 follow the main loss alone; the last layer the main loss plus lam
        times the estimate loss with its target frozen at the unperturbed error."""
        Y = sg.forward(ps, X)[-1]
        e = sg.readout(Y) - delta
        s = Y[:, 1].mean(axis=1)
        main = float(np.mean(e * e))
        return main + (sg.LAM * float(np.mean((s - t_frozen) ** 2)) if k == 4 else 0.0)

    acts = sg.forward(params, X)
    e0 = sg.readout(acts[-1]) - delta
    t_frozen = (np.log(e0 * e0 + sg.EPS) - sg.MU) / sg.SIG
    _, _, dY = sg.loss_and_grad(acts[-1], delta)
    grads = sg.backward(params, acts, dY)
    h = 1e-6
    for k in range(5):
        for part in range(2):
            arr = params[k][part]
            idx = [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(4)]
            for ix in idx:
                saved = arr[ix]
                arr[ix] = saved + h
                lp = loss(params, k)
                arr[ix] = saved - h
                lm = loss(params, k)
                arr[ix] = saved
                fd = (lp - lm) / (2 * h)
                assert grads[k][part][ix] == pytest.approx(fd, rel=1e-5, abs=1e-10), (k, part, ix)


def test_adam_first_step_closed_form():
    """At t = 1 the bias-corrected moments are g and g^2, so each entry moves by
    lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p, m1, m2 = sg.adam_step(np.ones(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(p, 1.0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)


def test_features_definition_values():
    G = np.full((1, 3, 4), 1e-5)
    G[0, 1, 2] = 1e-4
    X = sg.features(G, np.array([[0.0, 0.25, 0.5]]), np.array([5.0]))
    assert X[0, 0, 0, 0] == pytest.approx(0.0, abs=1e-15) and X[0, 0, 1, 2] == pytest.approx(1.0)
    assert np.allclose(X[0, 1, :, 0], [0.0, 0.5, 1.0]) and np.allclose(X[0, 2], 1.0)
    assert np.allclose(X[0, 3, 0], [-1, -1 / 3, 1 / 3, 1]) and np.allclose(X[0, 4, :, 0], [-1, 0, 1])
    assert np.all(sg.features(G[:, :1, :1], np.array([[0.1]]), np.array([1.0]))[0, 3:5] == 0.0)
    # line totals: row 1 holds one 1e-4 among four columns; column 2 sees 2 V_i G_i2 summed
    assert np.allclose(X[0, 5, :, 3], [0.1, (3e-5 + 1e-4) / 4 * 1e4, 0.1])
    assert np.allclose(X[0, 6, 0], [1e4 * (1e-5 * 0.5 + 1e-5 * 1.0) / 3] * 2
                       + [1e4 * (1e-4 * 0.5 + 1e-5 * 1.0) / 3] + [1e4 * (1e-5 * 0.5 + 1e-5 * 1.0) / 3])
    assert np.allclose(X[0, 6, 0], 1e4 * sg.ideal_currents(G, np.array([[0.0, 0.25, 0.5]]))[0] * 2 / 3)


def test_targets_vanish_without_wire_resistance():
    """As the wire resistances go to 0 the exact currents reach G^T V (Sec. II.A), so the
    correction the surrogate learns goes to 0; with real wires it is negative (IR drop)."""
    rng = np.random.default_rng(6)
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (1, 6, 5)))
    V = rng.uniform(0, 0.5, (1, 6))
    tiny = oracle.solve(G[0], V, 1e-9, 1e-9, 1e-9, 1e-9).currents
    assert np.abs(sg.targets(tiny, G, V)).max() < 1e-7
    real = oracle.solve(G[0], V, 5.0, 5.0, 5.0, 5.0).currents
    assert np.all(sg.targets(real, G, V) < 0)


def test_loss_gradient_of_the_readouts():
    """dLoss/dY spreads 2 e / (B n) evenly over the m rows of each column (channel 0)
    and lam 2 (s - t) / (B n) (channel 1), t the normalised log of e^2 + eps; the
    estimate loss is zero when s equals t, and the estimate is then |e|."""
    Y = np.zeros((2, 2, 3, 4))
    delta = np.arange(1.0, 9.0).reshape(2, 4) / 10
    loss, est_loss, dY = sg.loss_and_grad(Y, delta)
    assert loss == pytest.approx(np.mean(delta ** 2))
    assert np.allclose(dY[:, 0].sum(axis=1), -2 * delta / 8)
    t = (np.log(delta ** 2 + sg.EPS) - sg.MU) / sg.SIG
    assert est_loss == pytest.approx(np.mean(t ** 2))
    assert np.allclose(dY[:, 1].sum(axis=1), sg.LAM * 2 * (0 - t) / 8)
    Y[:, 1] = t[:, None, :]
    _, est_loss, dY = sg.loss_and_grad(Y, delta)
    assert est_loss == pytest.approx(0.0, abs=1e-20) and np.allclose(dY[:, 1], 0.0)
    assert np.allclose(sg.estimate(Y), np.sqrt(delta ** 2 + sg.EPS))     # yhat = 0 here
    Y[:, 0] = -0.5
    assert np.allclose(sg.estimate(Y), np.sqrt(delta ** 2 + sg.EPS) / 0.5)
