"""Learned current surrogate on 128 x 128 crossbars: data, training, accuracy, speed.

    python bench_surrogate.py [--maps 200000] [--held-out-maps 20000] [--vectors 1]
                              [--epochs 160] [--batch 32] [--lr 1e-3] [--channels 32]
                              [--precision bf16|fp32]

Workload (seeded, synthetic): conductance maps log-uniform on [1e-6, 1e-4] S, the
segment resistance r = r_wl = r_bl drawn from {1.0, 1.25, ..., 5.0} ohm per map,
r_src = r_sense = 50 ohm, input vectors uniform on [0, 0.5] V; `vectors` input vectors
per map.  The defaults give 200,000 training and 20,000 held-out samples, each with a
conductance map of its own.

Steps, all on the GPU through the library:
1. labels: exact float64 currents of every sample from the solver (the batched tile
   pipeline over the maps of each resistance level, 1024 maps per call), timed: that
   is the solver's throughput on new maps;
2. training: Adam on the mean squared error of the predicted correction, timed per
   step (features, 4 convolutions, readout and loss, 7 gradient kernels, update);
3. held-out accuracy: relative current error of the surrogate and of G^T V against the
   exact currents, mean, 99th percentile and maximum, and the share of samples whose
   worst column is within 1%; how well the error estimate ranks the errors; after
   calibrating its scale kappa on a third set (--cal-maps maps, 99% coverage), the
   held-out coverage, and at the tolerance (--tol) the share of samples it flags and
   the errors of the rest;
4. inference: surrogate currents for batches of held-out samples, timed;
5. checked predictions: the surrogate, with every flagged sample re-solved exactly,
   over the first 2048 held-out samples in one call, timed beside the same call with
   every sample solved exactly;
6. convolution rates: each layer's forward, input-gradient and weight-gradient
   convolution at the training batch, timed with HIP events on the launch stream, as
   TFLOP/s (2 flops per multiply-add of the 3 x 3 convolution) against the dense peak of
   the arithmetic they run on (bfloat16 matrix cores 2500, float32 vector 157.3).
One JSON line goes to stdout at the end; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--maps", type=int, default=200000)
    ap.add_argument("--held-out-maps", type=int, default=20000)
    ap.add_argument("--vectors", type=int, default=1)
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--epochs", type=int, default=160)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--channels", type=int, default=32)
    ap.add_argument("--depth", type=int, default=4, help="3 x 3 convolution layers")
    ap.add_argument("--seed", type=int, default=1005)
    ap.add_argument("--infer-batch", type=int, default=256)
    ap.add_argument("--tol", type=float, default=0.01, help="error-estimate threshold of the checked predictions")
    ap.add_argument("--cal-maps", type=int, default=4096, help="maps of the calibration set of the error estimate")
    ap.add_argument("--precision", choices=("bf16", "fp32"), default="bf16",
                    help="convolution arithmetic: bfloat16 matrix cores or float32 vector units")
    ap.add_argument("--rates-only", action="store_true", help="only the convolution rates (step 6)")
    args = ap.parse_args()

    import torch

    import paper_2410_19993_amd.surrogate as sgm
    from paper_2410_19993_amd import _lib
    _lib.lib()
    assert torch.cuda.is_available(), "no GPU visible"
    m = n = args.size
    if args.rates_only:
        print(json.dumps({"conv_rates": conv_rates(args, m, n)}), flush=True)
        return

    # 1. labels from the exact solver (the maps are drawn on the host first; the rate
    #    counts the solver's time)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    train = sgm.solver_dataset(args.maps, args.vectors, m, n, seed=args.seed)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    t_label = train.solve_seconds
    held = sgm.solver_dataset(args.held_out_maps, args.vectors, m, n, seed=args.seed + 1)
    cal = sgm.solver_dataset(args.cal_maps, args.vectors, m, n, seed=args.seed + 2)
    torch.cuda.synchronize()
    log(f"labels: {args.maps} maps x {args.vectors} vectors solved in {t_label:.1f} s "
        f"({args.maps / t_label:.0f} maps/s, {len(train) / t_label:.0f} solves/s; {t_data:.1f} s with drawing the maps)")

    # 2. training
    net = sgm.Surrogate(channels=args.channels, seed=args.seed, lr=args.lr, depth=args.depth,
                        precision=args.precision)
    S = len(train)
    steps_per_epoch = S // args.batch
    total = steps_per_epoch * args.epochs
    g = torch.Generator(device="cuda")
    g.manual_seed(args.seed)
    losses = []
    step = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep in range(args.epochs):
        perm = torch.randperm(S, device="cuda", generator=g)
        run = 0.0
        for k in range(steps_per_epoch):
            net.lr = args.lr * (0.1 + 0.9 * 0.5 * (1.0 + math.cos(math.pi * step / total)))
            G, V, r, d, _ = train.batch(perm[k * args.batch:(k + 1) * args.batch])
            want = (k % 200 == 199) or k == steps_per_epoch - 1
            loss = net.train_step(G, V, r, d, want_loss=want)
            if want:
                run = loss[0]
                losses.append((step + 1, loss[0], loss[1]))
            step += 1
        log(f"epoch {ep + 1}/{args.epochs}: loss {run:.3e} after {step} steps, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0

    kappa = net.calibrate(cal, quantile=0.99)
    log(f"error estimate calibrated on {len(cal)} samples: kappa {kappa:.2f}")

    # 3. held-out accuracy and the error estimate
    rel_sg, rel_0, ests = [], [], []
    for a in range(0, len(held), args.infer_batch):
        idx = torch.arange(a, min(len(held), a + args.infer_batch), device="cuda")
        G, V, r, _, I = held.batch(idx)
        est = torch.empty((len(idx), n), dtype=torch.float64, device="cuda")
        Ip = net.predict(G, V, r, est=est)
        I0 = held.I0[idx]
        rel_sg.append(((Ip - I).abs() / I.abs()).cpu().numpy())
        rel_0.append(((I0 - I).abs() / I.abs()).cpu().numpy())
        ests.append(est.cpu().numpy())
    rel_sg, rel_0, ests = np.concatenate(rel_sg), np.concatenate(rel_0), np.concatenate(ests)
    worst_err, worst_est = rel_sg.max(axis=1), ests.max(axis=1)
    rank = lambda x: np.argsort(np.argsort(x))
    spearman = float(np.corrcoef(rank(worst_est), rank(worst_err))[0, 1])
    flag = kappa * worst_est > args.tol
    covered = float(np.mean(worst_err <= kappa * worst_est))
    estimate = {"spearman_worst_column": spearman, "kappa": kappa, "calibration_samples": len(cal),
                "held_out_covered": covered, "tol": args.tol, "flagged_share": float(flag.mean()),
                "max_error_not_flagged": float(worst_err[~flag].max()) if (~flag).any() else None,
                "mean_worst_error_not_flagged": float(worst_err[~flag].mean()) if (~flag).any() else None,
                "share_not_flagged_within_tol": float(np.mean(worst_err[~flag] <= args.tol)) if (~flag).any()
                else None}
    for t in (0.01, 0.02, 0.05):
        f = kappa * worst_est > t
        estimate[f"at_{t:g}"] = {"flagged_share": float(f.mean()),
                                 "max_error_not_flagged": float(worst_err[~f].max()) if (~f).any() else None}
    log(f"error estimate: rank correlation {spearman:.2f}, kappa x estimate covers {100 * covered:.1f}% of held-out "
        f"samples; at tol {args.tol}: {100 * flag.mean():.1f}% flagged, "
        f"unflagged worst-column error max {estimate['max_error_not_flagged']}")

    def stats(e):
        worst = e.max(axis=1)
        return {"mean": float(e.mean()), "p99": float(np.percentile(e, 99)), "max": float(e.max()),
                "samples_within_1pct": float(np.mean(worst <= 0.01))}

    acc_sg, acc_0 = stats(rel_sg), stats(rel_0)
    log(f"held-out relative current error: surrogate mean {acc_sg['mean']:.2e} p99 {acc_sg['p99']:.2e} "
        f"max {acc_sg['max']:.2e}; G^T V mean {acc_0['mean']:.2e} max {acc_0['max']:.2e}")

    # 4. inference speed on held-out samples (inputs resident)
    B = min(args.infer_batch, len(held))
    idx = torch.arange(0, B, device="cuda")
    G, V, r, _, _ = held.batch(idx)
    out = torch.empty((B, n), dtype=torch.float64, device="cuda")
    for _ in range(3):
        net.predict(G, V, r, out)
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        net.predict(G, V, r, out)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / reps
    # 5. checked predictions: the first 2048 held-out samples in one call, the surrogate
    #    with the solver for every flagged sample; beside them the same samples all
    #    solved exactly through the same call (tol 0 flags every sample: the estimates
    #    are positive)
    chk_n = min(len(held), 2048)
    G, V, r, _, I = held.batch(torch.arange(0, chk_n, device="cuda"))
    net.predict_checked(G, V, r, tol=args.tol)            # warm-up: the solvers are created
    net.predict_checked(G, V, r, tol=0.0)
    reps = 3

    def timed(tol):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out, flagged = net.predict_checked(G, V, r, tol=tol)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, out, flagged

    t_chk, out, flagged = timed(args.tol)
    nflag = int(flagged.sum())
    t_all, out_all, flagged_all = timed(0.0)
    assert bool(flagged_all.all()), "tol 0 left a sample unflagged"
    e_chk = float(((out - I).abs() / I.abs()).max())
    net.close()
    estimate["checked_samples_per_s"] = chk_n / t_chk
    estimate["checked_samples"] = chk_n
    estimate["checked_flagged"] = nflag
    estimate["checked_max_error"] = e_chk
    estimate["all_exact_samples_per_s"] = chk_n / t_all
    log(f"checked predictions: {chk_n} samples ({nflag} re-solved exactly) in {t_chk * 1e3:.1f} ms, "
        f"max error {e_chk:.3e}; all {chk_n} solved exactly by the same call: {t_all * 1e3:.1f} ms")
    result = {
        "metric": "surrogate_samples_per_s", "value": B / t_inf, "unit": "samples/s",
        "workload": f"{m}x{n} crossbars, r_wl = r_bl in [1, 5] ohm, r_src = r_sense = 50 ohm, synthetic",
        "train_samples": S, "held_out_samples": len(held), "channels": args.channels, "depth": args.depth,
        "epochs": args.epochs,
        "batch": args.batch, "steps": total,
        "dtype": ("bf16 operands, f32 accumulate (convolutions)" if args.precision == "bf16" else
                  "f32 (convolutions)") + "; f32 (features, Adam), f64 (labels, readout)",
        "precision": args.precision,
        "label_solves_per_s": len(train) / t_label, "label_maps_per_s": args.maps / t_label,
        "label_seconds_with_drawing": t_data,
        "train_s": t_train, "train_ms_per_step": 1e3 * t_train / max(total, 1),
        "train_samples_per_s": total * args.batch / t_train,
        "infer_ms_per_batch": 1e3 * t_inf, "infer_batch": B,
        "speedup_vs_solver_new_maps": (B / t_inf) / (args.maps / t_label),
        "error_surrogate": acc_sg, "error_ideal_GtV": acc_0, "error_estimate": estimate, "loss_curve": losses[-10:],
        "conv_rates": conv_rates(args, m, n),
    }
    print(json.dumps(result), flush=True)
    net.close()


def conv_rates(args, m, n, reps: int = 50):
    """Per-launch time and rate of each convolution kind, summed over the network's layers
    at the training batch, with random operands of the layers' shapes."""
    import torch

    from paper_2410_19993_amd import _lib
    from paper_2410_19993_amd.surrogate import N_FEATURES
    bf = args.precision == "bf16"
    peak = 2500.0 if bf else 157.3
    B, L, Cw = args.batch, args.depth, args.channels
    dims = [N_FEATURES] + [Cw] * (L - 1) + [2]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    rnd = lambda *sh: torch.randn(*sh, generator=gen, device="cuda", dtype=torch.float32)
    s = torch.cuda.Stream()
    sp = s.cuda_stream
    work = torch.empty(max(_lib.xbar_sg_workspace_floats(dims[k], dims[k + 1]) for k in range(L)),
                       dtype=torch.float32, device="cuda")
    calls = {"forward": [], "input_gradient": [], "weight_gradient": []}
    flops = 0.0
    for k in range(L):
        C, O = dims[k], dims[k + 1]
        x, y, gy, gx = rnd(B, C, m, n), rnd(B, O, m, n), rnd(B, O, m, n), rnd(B, C, m, n)
        w, b, gw, gb = rnd(O, C, 3, 3), rnd(O), rnd(O, C, 3, 3), rnd(O)
        relu = k < L - 1
        calls["forward"].append(lambda C=C, O=O, x=x, w=w, b=b, y=y, relu=relu: _lib.xbar_sg_conv_forward(
            B, m, n, C, O, relu, x, w, b, y, sp, bf16=bf))
        if k > 0:
            # as in training: the output gradient arrives already masked by the ReLU, the
            # input gradient is masked by the layer input's ReLU
            calls["input_gradient"].append(lambda C=C, O=O, gy=gy, w=w, gx=gx, x=x: _lib.xbar_sg_conv_backward_data(
                B, m, n, C, O, gy, None, w, gx, xmask=x, stream=sp, bf16=bf))
        calls["weight_gradient"].append(lambda C=C, O=O, x=x, gy=gy, gw=gw, gb=gb: _lib.xbar_sg_conv_backward_weight(
            B, m, n, C, O, x, gy, None, gw, gb, work, sp, bf16=bf))
    out = {"peak_tflops": peak, "arithmetic": "bf16 matrix cores" if bf else "f32 vector", "batch": B}
    torch.cuda.synchronize()
    for kind, fs in calls.items():
        layer_flops = [2.0 * B * m * n * 9 * dims[k] * dims[k + 1] for k in range(L)]
        if kind == "input_gradient":
            layer_flops = layer_flops[1:]
        with torch.cuda.stream(s):
            for f in fs:
                f()
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record(s)
            for _ in range(reps):
                for f in fs:
                    f()
            t1.record(s)
        t1.synchronize()
        ms = t0.elapsed_time(t1) / reps
        tf = sum(layer_flops) / (ms * 1e-3) / 1e12
        out[kind] = {"ms_per_pass": ms, "launches_per_pass": len(fs), "tflops": tf, "frac": tf / peak}
        log(f"conv {kind}: {len(fs)} layers in {ms:.3f} ms, {tf:.1f} TFLOP/s, {tf / peak:.3f} of {peak} peak")
    # reference: a plain device copy of one hidden activation tensor (B x C x m x n float32),
    # the traffic of a layer that reads and writes one such tensor
    src, dst = rnd(B, Cw, m, n), torch.empty((B, Cw, m, n), dtype=torch.float32, device="cuda")
    with torch.cuda.stream(s):
        dst.copy_(src)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(s)
        for _ in range(reps):
            dst.copy_(src)
        t1.record(s)
    t1.synchronize()
    ms = t0.elapsed_time(t1) / reps
    nbytes = 2 * src.numel() * 4
    out["copy_reference"] = {"bytes": nbytes, "ms": ms, "gbps": nbytes / (ms * 1e-3) / 1e9}
    log(f"plain copy of a {tuple(src.shape)} float32 tensor: {ms * 1e3:.1f} us, {nbytes / (ms * 1e-3) / 1e9:.0f} GB/s")
    work = None
    return out


if __name__ == "__main__":
    main()
