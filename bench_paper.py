"""The paper's experiment shapes (Sec. III) measured on one MI355X with this solver.

    python bench_paper.py [--reps 10] [--quick]

Three tables, printed as markdown (and one JSON line per measurement on stderr):

1. Simulation time (Sec. III.B): m x n crossbars, m, n in {2, 4, ..., 256}, one
   input vector: assemble + factor + forward/back substitution with every node
   voltage + output currents, mean wall time over --reps runs.
2. Partitioning (Sec. III.C): a 256 x 256 crossbar split into s x s sub-crossbars,
   s in {2, ..., 256}, one input vector; every tile is solved as a crossbar of its
   own (sources on its rows, terminations at its bottom row) and the column
   currents of a tile column are summed.  Time for all tiles, one plan per tile
   size reused across its tiles.
3. Batch processing (Sec. III.D): n x n crossbars with batches of 1, 2, 10, 100 and
   1000 input vectors: decomposition time (assemble + factor) against solve time
   (substitution + currents), from HIP events on the plan stream.
4. Block ordering (Sec. III.B, bandwidth): m x n and n x m pairs (32 x 256, 128 x 512,
   32 x 700) with row blocks along the word lines ("rows") and of the smaller side
   ("smaller": a wide crossbar solved as its reciprocal), one input vector with node
   voltages, the block size each plan used, and which one the default ("auto") picks.

Inputs are seeded and synthetic: G log-uniform on [1e-6, 1e-4] S, V uniform on
[0, 0.5] V, and the paper's model of 5-ohm wire segments, with the source and
the termination each reached through one segment (r_src = r_wl, r_sense = r_bl).
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

SIZES = [2, 4, 8, 16, 32, 64, 128, 256]
BATCHES = [1, 2, 10, 100, 1000]
R = 5.0


def log(rec):
    print(json.dumps(rec), file=sys.stderr, flush=True)


def inputs(m, n, B, seed):
    rng = np.random.default_rng(seed)
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (m, n)))
    V = rng.uniform(0.0, 0.5, (B, m))
    return G, V


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--quick", action="store_true", help="fewer sizes (smoke run)")
    args = ap.parse_args()

    import torch

    import paper_2410_19993_amd as xb
    from paper_2410_19993_amd import _lib
    _lib.lib()
    assert torch.cuda.is_available(), "no GPU visible"
    sizes = [4, 32, 256] if args.quick else SIZES
    dev = torch.device("cuda")

    def run_plan(p, Gd, Vd, nv):
        p.assemble(Gd)
        p.factor()
        p.solve_batch(Vd, nv)
        return p.currents()

    # 1. simulation time, one input vector
    print("## Simulation time, one input vector (ms, mean of %d)\n" % args.reps)
    print("| m \\ n | " + " | ".join(str(n) for n in sizes) + " |")
    print("|---|" + "---:|" * len(sizes))
    for m in sizes:
        row = []
        for n in sizes:
            G, V = inputs(m, n, 1, 7 * m + n)
            Gd, Vd = torch.from_numpy(G).to(dev), torch.from_numpy(V).to(dev)
            nv = torch.empty((1, 2 * m * n), dtype=torch.float64, device=dev)
            with xb.Plan(m, n, R, R, R, R, "fp64", max_batch=1) as p:
                run_plan(p, Gd, Vd, nv)
                torch.cuda.synchronize()
                p.check()
                ts = []
                for _ in range(args.reps):
                    t0 = time.perf_counter()
                    run_plan(p, Gd, Vd, nv)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                p.check()
            ms = 1e3 * float(np.mean(ts))
            log({"table": "size", "m": m, "n": n, "ms": ms})
            row.append(f"{ms:.2f}")
        print(f"| {m} | " + " | ".join(row) + " |")

    # 2. partitioning of a 256 x 256 crossbar
    M = 256
    G, V = inputs(M, M, 1, 2561)
    print("\n## 256 x 256 crossbar partitioned into s x s sub-crossbars, one input vector\n")
    print("| s | tiles | total ms | ms per tile |")
    print("|---:|---:|---:|---:|")
    for s in sizes:
        k = M // s
        tiles = [(a, b) for a in range(k) for b in range(k)]
        Gt = [torch.from_numpy(np.ascontiguousarray(G[a * s:(a + 1) * s, b * s:(b + 1) * s])).to(dev)
              for a, b in tiles]
        Vt = [torch.from_numpy(np.ascontiguousarray(V[:, a * s:(a + 1) * s])).to(dev) for a, b in tiles]
        nv = torch.empty((1, 2 * s * s), dtype=torch.float64, device=dev)
        I = torch.zeros((1, M), dtype=torch.float64, device=dev)
        reps = max(1, min(args.reps, 64 // len(tiles) if len(tiles) < 64 else 1))
        with xb.Plan(s, s, R, R, R, R, "fp64", max_batch=1) as p:
            run_plan(p, Gt[0], Vt[0], nv)
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                I.zero_()
                t0 = time.perf_counter()
                for t, (a, b) in enumerate(tiles):
                    I[:, b * s:(b + 1) * s] += run_plan(p, Gt[t], Vt[t], nv)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            p.check()
        ms = 1e3 * float(np.mean(ts))
        log({"table": "partition", "s": s, "tiles": len(tiles), "ms": ms})
        print(f"| {s} | {len(tiles)} | {ms:.1f} | {ms / len(tiles):.3f} |")

    # 3. decomposition against solve time over batch sizes
    print("\n## Decomposition and solve time by batch size (ms, HIP events, mean of %d)\n" % args.reps)
    print("| n x n | B | decomposition | solve | solve share |")
    print("|---|---:|---:|---:|---:|")
    for n in [s for s in sizes if s >= 4]:
        for B in BATCHES:
            G, V = inputs(n, n, B, 11 * n + B)
            Gd, Vd = torch.from_numpy(G).to(dev), torch.from_numpy(V).to(dev)
            nv = torch.empty((B, 2 * n * n), dtype=torch.float64, device=dev)
            with xb.Plan(n, n, R, R, R, R, "fp64", max_batch=B) as p:
                run_plan(p, Gd, Vd, nv)
                torch.cuda.synchronize()
                p.set_timing(True)
                p.timing(reset=True)
                for _ in range(args.reps):
                    run_plan(p, Gd, Vd, nv)
                tm = p.timing()
                p.check()
            dec = (tm.condense_ms + tm.factor_ms) / args.reps
            sol = (tm.sweep_ms + tm.recover_ms) / args.reps
            log({"table": "batch", "n": n, "B": B, "decomposition_ms": dec, "solve_ms": sol})
            print(f"| {n} x {n} | {B} | {dec:.3f} | {sol:.3f} | {100 * sol / (dec + sol):.0f}% |")

    # 4. block ordering of wide and tall crossbars
    print("\n## Block ordering, one input vector with node voltages (ms, mean of %d)\n" % args.reps)
    print("| m x n | ordering | block | ms | auto picks |")
    print("|---|---|---:|---:|---|")
    pairs = [(32, 256), (256, 32), (128, 512), (512, 128), (32, 700), (700, 32)]
    if args.quick:
        pairs = pairs[:2]
    for (m, n) in pairs:
        G, V = inputs(m, n, 1, 13 * m + n)
        Gd, Vd = torch.from_numpy(G).to(dev), torch.from_numpy(V).to(dev)
        nv = torch.empty((1, 2 * m * n), dtype=torch.float64, device=dev)
        orders = ["rows", "smaller"] if n > m and n <= 512 else (["smaller"] if n > m else ["rows"])
        with xb.Plan(m, n, R, R, R, R, "fp64", max_batch=1) as p:
            auto_block = p.info()[1].block
        for order in orders:
            with xb.Plan(m, n, R, R, R, R, "fp64", max_batch=1, ordering=order) as p:
                run_plan(p, Gd, Vd, nv)
                torch.cuda.synchronize()
                ts = []
                for _ in range(args.reps):
                    t0 = time.perf_counter()
                    run_plan(p, Gd, Vd, nv)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                p.check()
                block = p.info()[1].block
            ms = 1e3 * float(np.mean(ts))
            log({"table": "ordering", "m": m, "n": n, "ordering": order, "block": block, "ms": ms})
            print(f"| {m} x {n} | {order} | {block} | {ms:.2f} | {'yes' if block == auto_block else ''} |")


if __name__ == "__main__":
    main()
