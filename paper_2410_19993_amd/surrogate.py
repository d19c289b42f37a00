"""Learned current surrogate: a small convolutional network, trained on solver output.

The network predicts the relative parasitic correction of each bit-line current,
delta_j = (I_j - I0_j) / I0_j, where I0 = G^T V are the currents without wire
resistance (the zero-resistance limit of the nodal equations of Sec. II.A), so
that the surrogate's currents are I0 (1 + yhat).  The exact solver (Plan,
PlanLanes) produces the training targets and stays the reference for the error.

Network: 7 features per crosspoint (log10 G + 5, 2 V_i, (r - 3) / 2, column and
row position, and the row's mean conductance and the column's mean G 2 V, which set
the drops across the source and sense resistors at the line ends), four 3 x 3
convolutions 7 -> C -> ... -> C -> 2 (four layers by default, `depth`) with ReLU after
all but the last.  The row means of
the last map's two channels are the correction yhat_j and the error estimate s_j.
Loss: mean squared error of yhat against delta, plus lam times the squared error of
s against the normalised log((yhat - delta)^2 + eps), that target held constant; the
second term trains the last layer's estimate channel only, so the correction keeps
the shared layers to itself.  Optimizer: Adam.  Every step (features,
convolutions, their gradients, readouts, loss, update, prediction) runs in the
library's kernels (xbar_sg_*); torch only holds the device buffers.
predict_checked() re-solves with the exact solver every sample whose estimate
exceeds a tolerance.
"""
from __future__ import annotations

import time

import numpy as np

from . import _check_tensor, _lib
from .lanes import PlanLanes

N_FEATURES = 7


def _torch():
    import torch
    return torch


class Surrogate:
    """Weights, Adam state and activation buffers of the surrogate on the current device.

    channels: width C of the hidden layers (<= 32).  seed: weight initialisation
    (He-normal weights, zero biases).  zero_last: start the last layer at zero, so
    that the untrained network predicts the ideal currents G^T V exactly."""

    def __init__(self, channels: int = 32, seed: int = 0, lr: float = 1e-3, betas=(0.9, 0.999),
                 eps: float = 1e-8, zero_last: bool = True, lam: float = 0.1, depth: int = 4,
                 precision: str = "bf16"):
        torch = _torch()
        if not 1 <= channels <= 32:
            raise ValueError("channels must be in [1, 32]")
        if depth < 2:
            raise ValueError("depth must be >= 2")
        if precision not in ("bf16", "fp32"):
            raise ValueError("precision must be 'bf16' (matrix cores) or 'fp32' (vector ALUs)")
        # the convolutions' arithmetic: bfloat16 operands with float32 accumulation on the
        # matrix cores, or float32 throughout; weights, activations and Adam stay float32
        self.precision = precision
        self._bf16 = precision == "bf16"
        self.C = int(channels)
        self.L = int(depth)
        self.dims = [N_FEATURES] + [self.C] * (self.L - 1) + [2]
        self.lr, self.betas, self.eps, self.lam = float(lr), tuple(betas), float(eps), float(lam)
        self.t = 0
        sizes = []
        for k in range(self.L):
            sizes += [self.dims[k + 1] * self.dims[k] * 9, self.dims[k + 1]]
        self._sizes = sizes
        total = sum(sizes)
        rng = np.random.default_rng(seed)
        host = np.zeros(total, dtype=np.float32)
        off = 0
        for k in range(self.L):
            nw = sizes[2 * k]
            w = rng.normal(0.0, np.sqrt(2.0 / (self.dims[k] * 9)), nw)
            host[off:off + nw] = 0.0 if (zero_last and k == self.L - 1) else w
            off += nw + sizes[2 * k + 1]
        self.params = torch.from_numpy(host).cuda()
        self.grads = torch.zeros_like(self.params)
        self.m1 = torch.zeros_like(self.params)
        self.m2 = torch.zeros_like(self.params)
        # the weight gradient's partial sums: the largest need over the layers (the first
        # maps 7 features to C channels, which needs more than C -> C when C < 7)
        ws = max(_lib.xbar_sg_workspace_floats(self.dims[k], self.dims[k + 1]) for k in range(self.L))
        self.work = torch.empty(ws, dtype=torch.float32, device="cuda")
        self._buf_shape = None
        self._solvers = {}
        self.kappa = 1.0

    # -- parameter views -----------------------------------------------------------------
    def _views(self, flat):
        out, off = [], 0
        for k in range(self.L):
            nw, nb = self._sizes[2 * k], self._sizes[2 * k + 1]
            out.append((flat[off:off + nw], flat[off + nw:off + nw + nb]))
            off += nw + nb
        return out

    def layers(self):
        """[(w [O][C][3][3], b [O])] views of the weights."""
        return [(w.view(self.dims[k + 1], self.dims[k], 3, 3), b) for k, (w, b) in enumerate(self._views(self.params))]

    def state(self) -> dict:
        """Host copies of the weights and optimizer state (for checkpoints)."""
        return {"params": self.params.cpu().numpy(), "m1": self.m1.cpu().numpy(), "m2": self.m2.cpu().numpy(),
                "t": self.t, "channels": self.C, "depth": self.L, "kappa": self.kappa, "precision": self.precision}

    def load(self, state: dict) -> None:
        torch = _torch()
        if int(state["channels"]) != self.C or int(state.get("depth", 4)) != self.L:
            raise ValueError("checkpoint has a different width or depth")
        for name in ("params", "m1", "m2"):
            getattr(self, name).copy_(torch.from_numpy(np.asarray(state[name], dtype=np.float32)))
        self.t = int(state["t"])
        self.kappa = float(state.get("kappa", 1.0))

    # -- buffers -------------------------------------------------------------------------
    def _buffers(self, B, m, n):
        torch = _torch()
        if self._buf_shape is not None and self._buf_shape[0] >= B and self._buf_shape[1:] == (m, n):
            return
        f = dict(dtype=torch.float32, device="cuda")
        self.X = torch.empty((B, N_FEATURES, m, n), **f)
        self.acts = [torch.empty((B, self.C, m, n), **f) for _ in range(self.L - 1)]
        self.Y = torch.empty((B, 2, m, n), **f)
        self.gY = torch.empty((B, 2, m, n), **f)
        self.ga = [torch.empty((B, self.C, m, n), **f) for _ in range(2)]
        self.err2 = torch.empty((B, 2), dtype=torch.float64, device="cuda")
        self._buf_shape = (B, m, n)

    @staticmethod
    def _stream():
        return _torch().cuda.current_stream().cuda_stream

    # -- steps ---------------------------------------------------------------------------
    @staticmethod
    def _check_inputs(G, V, r, delta=None):
        """G [B][m][n], V [B][m], r [B] (and delta [B][n]): contiguous float64 device
        tensors of exactly these shapes, checked before any kernel reads them."""
        if getattr(G, "dim", lambda: 0)() != 3:
            raise ValueError("G must be a [B][m][n] tensor")
        B, m, n = (int(x) for x in G.shape)
        _check_tensor("G", G, (B, m, n))
        _check_tensor("V", V, (B, m))
        _check_tensor("r", r, (B,))
        if delta is not None:
            _check_tensor("delta", delta, (B, n))
        return B, m, n

    def forward(self, G, V, r):
        """Last map Y [B][2][m][n] for G [B][m][n], V [B][m], r [B] (float64 device tensors)."""
        B, m, n = self._check_inputs(G, V, r)
        self._buffers(B, m, n)
        s = self._stream()
        _lib.xbar_sg_features(B, m, n, G, V, r, self.X, s)
        x = self.X
        outs = self.acts + [self.Y]
        for k, (w, b) in enumerate(self._views(self.params)):
            _lib.xbar_sg_conv_forward(B, m, n, self.dims[k], self.dims[k + 1], k < self.L - 1, x, w, b, outs[k], s,
                                      bf16=self._bf16)
            x = outs[k]
        return self.Y[:B]

    def train_step(self, G, V, r, delta, want_loss: bool = True):
        """One forward, backward and Adam step on a batch (delta [B][n] float64 device
        tensor).  Returns (mean (yhat - delta)^2, mean (s - t)^2), t the normalised log
        squared error, which waits for the step to finish, or None when want_loss is
        false."""
        B, m, n = self._check_inputs(G, V, r, delta)
        self.forward(G, V, r)
        s = self._stream()
        _lib.xbar_sg_readout_loss(B, m, n, self.Y, delta, self.lam, self.gY, self.err2, s)
        ins = [self.X] + self.acts                  # input of layer k
        gv = self._views(self.grads)
        wv = self._views(self.params)
        g_out = self.gY                             # dLoss / d(output of layer k)
        last = self.L - 1
        for k in range(last, -1, -1):
            # g_out is already the gradient before layer k's ReLU: the input gradient of
            # layer k + 1 wrote it masked by [layer k's output > 0]
            C, O = self.dims[k], self.dims[k + 1]
            _lib.xbar_sg_conv_backward_weight(B, m, n, C, O, ins[k], g_out, None, gv[k][0], gv[k][1], self.work, s,
                                              bf16=self._bf16)
            if k == last:
                self.gY[:B, 1].zero_()              # the estimate trains the last layer only
            if k > 0:
                g_in = self.ga[k % 2]
                _lib.xbar_sg_conv_backward_data(B, m, n, C, O, g_out, None, wv[k][0], g_in, xmask=ins[k], stream=s,
                                                bf16=self._bf16)
                g_out = g_in
        self.t += 1
        _lib.xbar_sg_adam(self.params, self.grads, self.m1, self.m2, self.lr, self.betas[0], self.betas[1],
                          self.eps, self.t, s)
        if not want_loss:
            return None
        e = self.err2[:B].cpu().numpy().sum(axis=0) / (B * n)
        return float(e[0]), float(e[1])

    def predict(self, G, V, r, out=None, est=None):
        """Surrogate currents I [B][n] float64 = (G^T V)_j (1 + yhat_j); when est (a
        [B][n] float64 tensor) is given, it receives the predicted relative errors."""
        torch = _torch()
        B, m, n = self._check_inputs(G, V, r)
        if out is None:
            out = torch.empty((B, n), dtype=torch.float64, device="cuda")
        _check_tensor("out", out, (B, n))
        if est is not None:
            _check_tensor("est", est, (B, n))
        self.forward(G, V, r)
        _lib.xbar_sg_predict(B, m, n, self.Y, G, V, out, est, self._stream())
        return out

    def calibrate(self, data: "Dataset", quantile: float = 0.99, batch: int = 256) -> float:
        """Set kappa so that kappa times the largest estimated error of a sample covers its
        largest actual relative current error on `quantile` of the samples of `data`
        (solver-labelled samples the network was not trained on: a split-conformal
        calibration).  Returns kappa."""
        torch = _torch()
        n = int(data.G.shape[2])
        ratios = []
        for a in range(0, len(data), batch):
            idx = torch.arange(a, min(len(data), a + batch), device="cuda")
            G, V, r, _, I = data.batch(idx)
            est = torch.empty((len(idx), n), dtype=torch.float64, device="cuda")
            Ip = self.predict(G, V, r, est=est)
            # per sample, the worst relative error over the columns with a nonzero exact
            # current divided by the largest estimate (NaN: left out of the quantile)
            ratio = torch.empty(len(idx), dtype=torch.float64, device="cuda")
            _lib.xbar_sg_calib_ratios(len(idx), n, Ip, I, est, ratio, self._stream())
            x = ratio.cpu().numpy()
            ratios.append(x[np.isfinite(x)])
        ratios = np.concatenate(ratios)
        if ratios.size == 0:
            raise ValueError("calibration set has no sample with a nonzero exact current and a finite estimate")
        kappa = float(np.quantile(ratios, quantile))
        if not np.isfinite(kappa) or kappa <= 0:
            raise ValueError(f"calibration gave a kappa that is not finite and positive: {kappa}")
        self.kappa = kappa
        return self.kappa

    def predict_checked(self, G, V, r, tol: float = 0.01, r_src: float = 50.0, r_sense: float = 50.0,
                        lanes: int = 4, precision: str = "fp64"):
        """Currents for every sample, from the surrogate where kappa times its error
        estimate is at most tol in every column (kappa = 1 until calibrate()), and from
        the exact solver for the others, grouped by segment resistance: in float64
        (`precision` "fp64") through the batched tile pipeline, the group padded to a
        power of two (at least 32) by repeating its last map; with "fp32_ir" (float32
        with float64 refinement) through PlanLanes, one plan per map on `lanes` host
        threads.  Returns (I, flagged), flagged a host bool array of the samples that
        were solved exactly.  The solvers are kept for later calls until close()."""
        torch = _torch()
        from .tiles import TileBatch, TileConfig
        B, m, n = (int(x) for x in G.shape)
        est = torch.empty((B, n), dtype=torch.float64, device="cuda")
        out = self.predict(G, V, r, est=est)
        # a sample is trusted only when its scaled estimate is a number <= tol in every
        # column and its currents are finite; samples whose conductances are not finite
        # and positive, or whose inputs are not finite, go to the exact solver, which
        # reports them (XBAR_ERR_INPUT) instead of returning surrogate values
        flag = torch.empty(B, dtype=torch.int32, device="cuda")
        _lib.xbar_sg_route(B, m, n, G, V, out, est, self.kappa, tol, flag, self._stream())
        flagged = flag.cpu().numpy().astype(bool)
        idx = np.nonzero(flagged)[0]
        if len(idx):
            rs = r.cpu().numpy()
            for lv in np.unique(rs[idx]):
                sel = idx[rs[idx] == lv]
                if precision == "fp64":
                    cnt = len(sel)
                    bucket = max(32, 1 << (cnt - 1).bit_length())
                    key = ("tiles", float(lv), float(r_src), float(r_sense), m, n, bucket)
                    tb = self._solvers.get(key)
                    if tb is None:
                        tb = self._solvers[key] = TileBatch([(m, n, bucket, 1)], lv, lv, r_src, r_sense,
                                                            configs=[TileConfig("pipeline")], streams=1)
                    st = torch.from_numpy(np.concatenate([sel, np.full(bucket - cnt, sel[-1])])).cuda()
                    Ib = tb.run([G[st].contiguous()], [V[st].unsqueeze(1).contiguous()])[0][:cnt, 0]
                    # the pipeline gives a crossbar with a bad conductance (or pivot) NaN
                    # currents where a plan reports the input; a NaN input gives NaN
                    # currents either way
                    bad = ~torch.isfinite(Ib).all(dim=1) & torch.isfinite(V[st[:cnt]]).all(dim=1)
                    if bool(bad.any()):
                        raise _lib.XbarError("predict_checked", _lib.XBAR_ERR_INPUT)
                    out[st[:cnt]] = Ib
                    continue
                key = (float(lv), float(r_src), float(r_sense), int(lanes), precision)
                pl = self._solvers.get(key)
                if pl is None:
                    pl = self._solvers[key] = PlanLanes(key[0], key[0], key[1], key[2], lanes=key[3], max_batch=1,
                                                        precision=precision)
                pl.currents([G[k] for k in sel], [V[k:k + 1] for k in sel], [out[k:k + 1] for k in sel])
                pl.check()
        return out, flagged

    def close(self) -> None:
        """Free the solvers predict_checked keeps (per segment resistance: tile batches
        and plan lanes)."""
        for pl in self._solvers.values():
            pl.close()
        self._solvers.clear()


class Dataset:
    """Solver-labelled samples: maps G [M][m][n] with segment resistances r [M], and
    `vectors` input vectors per map, V [M * vectors][m], with their exact currents
    I [M * vectors][n] and targets delta (all float64 device tensors).  Sample s uses
    map s // vectors."""

    def __init__(self, G, r, V, I, vectors):
        self.G, self.r, self.V, self.I, self.vectors = G, r, V, I, int(vectors)
        self.delta, self.I0 = targets_of(self)

    def __len__(self):
        return int(self.V.shape[0])

    def batch(self, idx):
        """(G, V, r, delta, I) of the samples idx (a device int64 tensor), gathered."""
        maps = idx // self.vectors
        return (self.G[maps].contiguous(), self.V[idx].contiguous(), self.r[maps].contiguous(),
                self.delta[idx].contiguous(), self.I[idx].contiguous())


def solver_dataset(maps: int, vectors: int, m: int, n: int, seed: int, r_levels=None, r_src: float = 50.0,
                   r_sense: float = 50.0, lanes: int = 4, method: str = "tiles", chunk: int = 1024) -> Dataset:
    """Training data from the exact solver: `maps` conductance maps (log-uniform on
    [1e-6, 1e-4] S), each with `vectors` input vectors (uniform on [0, 0.5] V) and one
    segment resistance r = r_wl = r_bl drawn from r_levels (default 1.0, 1.25, ..., 5.0
    ohm).  The maps of one resistance level are solved together: with method "tiles"
    through TileBatch's batched pipeline (condensation, block factor and sweep over up
    to `chunk` maps per call), with "lanes" through PlanLanes (one plan per map on
    `lanes` host threads)."""
    from .tiles import TileBatch, TileConfig
    torch = _torch()
    if method not in ("tiles", "lanes"):
        raise ValueError(f"method must be 'tiles' or 'lanes', not {method!r}")
    levels = np.arange(1.0, 5.0001, 0.25) if r_levels is None else np.asarray(r_levels, dtype=np.float64)
    rng = np.random.default_rng(seed)
    # the maps in draws of about 1 GiB of host memory (the same stream as one draw)
    Gd = torch.empty((maps, m, n), dtype=torch.float64, device="cuda")
    step = max(1, (1 << 27) // (m * n))
    for a in range(0, maps, step):
        b = min(maps, a + step)
        Gd[a:b].copy_(torch.from_numpy(np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (b - a, m, n)))))
    Vm = rng.uniform(0.0, 0.5, (maps, vectors, m))
    rm = levels[rng.integers(0, len(levels), maps)]
    Vd = torch.from_numpy(Vm).cuda()
    Id = torch.empty((maps, vectors, n), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lv in np.unique(rm):
        idx = np.nonzero(rm == lv)[0]
        if method == "lanes":
            with PlanLanes(lv, lv, r_src, r_sense, lanes=lanes, max_batch=vectors) as pl:
                pl.currents([Gd[k] for k in idx], [Vd[k] for k in idx], [Id[k] for k in idx])
                pl.check()
            continue
        batches = {}
        try:
            for a in range(0, len(idx), chunk):
                sel = torch.from_numpy(idx[a:a + chunk]).cuda()
                count = int(sel.numel())
                if count not in batches:
                    batches[count] = TileBatch([(m, n, count, vectors)], lv, lv, r_src, r_sense,
                                               configs=[TileConfig("pipeline")], streams=1)
                Id[sel] = batches[count].run([Gd[sel].contiguous()], [Vd[sel].contiguous()])[0]
        finally:
            for tb in batches.values():
                tb.close()
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - t0
    if not bool(torch.isfinite(Id).all()):
        raise RuntimeError("solver_dataset: a label is not finite (a map the solver rejected)")
    ds = Dataset(Gd, torch.from_numpy(rm).cuda(), Vd.reshape(maps * vectors, m), Id.reshape(maps * vectors, n),
                 vectors)
    ds.solve_seconds = solve_s           # the solver's share: the maps are drawn on the host before
    return ds


def targets_of(ds: Dataset):
    """delta = (I - I0) / I0 with I0 = G^T V formed by the library's prediction kernel
    (a zero correction map), chunked over samples."""
    torch = _torch()
    S, n = (int(x) for x in ds.I.shape)
    m = int(ds.G.shape[1])
    I0 = torch.empty((S, n), dtype=torch.float64, device="cuda")
    step = 4096
    zero = torch.zeros((min(step, S), 2, m, n), dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    for a in range(0, S, step):
        idx = torch.arange(a, min(S, a + step), device="cuda")
        Gb = ds.G[idx // ds.vectors].contiguous()
        _lib.xbar_sg_predict(len(idx), m, n, zero, Gb, ds.V[idx].contiguous(), I0[a:a + len(idx)], None, st)
    delta = torch.empty_like(I0)
    _lib.xbar_sg_targets(S, n, ds.I, I0, delta, st)
    return delta, I0
