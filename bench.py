"""Benchmark: input-vector solves/s of the crossbar nodal solve on one MI355X.

A step is one pass of the whole path on the 512x512 crossbar workload
(G log-uniform on [1e-6, 1e-4] S, 4096 input vectors ~ U[0, 0.5] V, 50-ohm
source and sense resistors, segment resistance --r): assemble, factor,
forward/back substitution with every node voltage written to HBM, and the
output currents.  Inputs are resident in HBM before timing starts.

    python bench.py [--steps K] [--warmup W] [--r 2.5] [--precision fp64]

Prints one JSON line.  --gpus N > 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA = 78.6e12     # MI355X dense FP64 matrix, FLOP/s
PEAK_FP32_MFMA = 157.3e12
PEAK_HBM = 8.0e12            # B/s
METRIC = ("input-vector solves/s, 512×512 xbar: FP64 LU vs FP32+IR at 1e-9 rel err")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(wl, rows=16, vectors=64):
    """Time the oracle on a bounded slice of the same workload and scale it.

    The oracle's banded LU costs rows x (half-bandwidth)^2 and its substitution
    rows x half-bandwidth per vector; the half-bandwidth (2n) is that of the full
    crossbar, so the time scales linearly in rows and (for the solve) in vectors.
    """
    import oracle
    g = wl.geom
    Gs = np.ascontiguousarray(wl.G[:rows])
    Vs = np.ascontiguousarray(wl.V[:vectors, :rows])
    t0 = time.perf_counter()
    net = oracle.build_netlist(Gs, g.r_wl, g.r_bl, g.r_src, g.r_sense)
    ab, w = oracle.assemble_band(net)
    oracle.lu_factor(ab, w)
    t_fact = time.perf_counter() - t0
    del ab
    t0 = time.perf_counter()
    oracle.solve(Gs, Vs, g.r_wl, g.r_bl, g.r_src, g.r_sense)
    t_all = time.perf_counter() - t0
    per_vec = max(t_all - t_fact, 0.0) / vectors
    scale = wl.G.shape[0] / rows
    t_full = scale * (t_fact + wl.B * per_vec)
    return {"value": wl.B / t_full, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle on rows 0-{rows - 1} of the {wl.G.shape[0]}x{wl.G.shape[1]} "
                       f"conductance map (same {2 * wl.G.shape[1]}-wide half band) with {vectors} "
                       f"input vectors; measured {t_fact + per_vec * vectors:.1f} s; time scaled "
                       f"x{scale:g} in rows and to {wl.B} vectors (banded LU and substitution "
                       f"cost are linear in rows)"),
            "seconds_measured": t_all + t_fact, "extrapolated_seconds": t_full}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--r", type=float, default=2.5)
    ap.add_argument("--precision", default="fp64", choices=["fp64"])
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the solver has no multi-GPU path in this build.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2410_19993_amd as xb
    import workloads
    from paper_2410_19993_amd import _lib
    _lib.lib()                                   # fails loudly when libxbar.so is missing
    assert torch.cuda.is_available(), "no GPU visible"

    wl = workloads.c3(r=args.r, batch=args.batch)
    m, n, B = wl.G.shape[0], wl.G.shape[1], wl.B
    g = wl.geom
    log(f"workload {wl.name}: m={m} n={n} B={B} r={g.r_wl}")
    G = torch.from_numpy(wl.G).cuda()
    V = torch.from_numpy(np.ascontiguousarray(wl.V)).cuda()
    node_v = torch.empty((B, 2 * m * n), dtype=torch.float64, device="cuda")
    I = torch.empty((B, n), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    plan = xb.Plan(m, n, g.r_wl, g.r_bl, g.r_src, g.r_sense, args.precision, max_batch=B,
                   stream=stream)

    def step():
        plan.assemble(G)
        plan.factor()
        plan.solve_batch(V, node_v)
        plan.currents(I)

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {w} done")
    plan.check()
    plan.set_timing(True)
    plan.timing(reset=True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for s in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    tm = plan.timing()
    plan.check()
    ms_per_step = 1e3 * wall / args.steps
    log(f"timed {args.steps} steps: wall {wall:.3f} s, events {gpu_ms:.1f} ms")

    # kernels: algorithmic work per launch
    sweep_flops = 2.0 * n * n * B * (2 * m - 1)          # forward m products + back (m-1)
    factor_flops = float(m) * n ** 3                     # m SPD inverses of n x n
    k_sweep = tm.sweep_ms / max(tm.sweep_launches, 1)
    k_factor = tm.factor_ms / max(tm.factor_launches, 1)
    k_recover = tm.recover_ms / max(tm.recover_launches, 1)
    k_condense = tm.condense_ms / max(tm.condense_launches, 1)
    recover_bytes = 8.0 * B * m * n * (1 + 2) + 8.0 * 3 * m * n     # read u, write w and u
    phases = {"condense_ms": k_condense, "factor_ms": k_factor, "sweep_ms": k_sweep,
              "recover_ms": k_recover}
    achieved = sweep_flops / (k_sweep * 1e-3)
    roof = {"bound": "mfma", "kernel": "sweep_kernel<double,8>", "achieved": achieved / 1e12,
            "peak": PEAK_FP64_MFMA / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_MFMA,
            "traffic": None, "flops_per_launch": sweep_flops, "avg_launch_ms": k_sweep}

    result = {
        "metric": METRIC, "value": B / (ms_per_step * 1e-3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "m": m, "n": n, "batch": B, "r_segment_ohm": g.r_wl,
                   "r_src_ohm": g.r_src, "r_sense_ohm": g.r_sense, "precision": args.precision,
                   "node_voltages": True, "parallelism": "single-gpu"},
        "phases_ms": phases,
        "factor": {"algorithmic_flops": factor_flops, "ms": k_factor,
                   "tflops": factor_flops / (k_factor * 1e-3) / 1e12,
                   "kernel_launches": int(tm.factor_launches)},
        "recover": {"ms": k_recover, "bytes": recover_bytes,
                    "gbps": recover_bytes / (k_recover * 1e-3) / 1e9 if k_recover > 0 else None},
        "roofline": roof,
    }
    if not args.no_verify:
        gold = os.path.join(ROOT, "tests", "golden", f"c3_r{g.r_wl:g}_currents.npy")
        if os.path.exists(gold) and B == 4096:
            ref = np.load(gold)
            sub = workloads.c3_subset()
            Ih = I.cpu().numpy()[sub]
            err = np.max(np.abs(Ih - ref), axis=1) / np.max(np.abs(ref), axis=1)
            result["max_rel_err_vs_oracle"] = float(err.max())
            result["verified_vectors"] = int(len(sub))
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample ...")
        result["cpu_baseline"] = cpu_baseline(wl)
    plan.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
