"""Benchmark: input-vector solves/s of the crossbar nodal solve on one MI355X.

A step is one pass of the whole path on the 512x512 crossbar workload
(G log-uniform on [1e-6, 1e-4] S, 4096 input vectors ~ U[0, 0.5] V, 50-ohm
source and sense resistors, segment resistance --r): assemble, factor,
forward/back substitution with every node voltage written to HBM, and the
output currents.  Inputs are resident in HBM before timing starts.

    python bench.py [--steps K] [--warmup W] [--r 2.5] [--no-fp32-ir] [--no-cpu-baseline]
                    [--no-shortcuts] [--no-tiles] [--no-r-sweep]
    python bench.py --copy-probe GIB    # a plain device copy of GIB GiB, three times
                                        # (calibrates the HBM traffic counters)

Besides the metric (float64, node voltages written) the line reports the
float32 + float64-refinement leg and exact shortcuts that skip work the metric
does: the same path without node voltages, the sweeps alone, and the output
currents through the transfer matrix (one product per batch once T is built).
It also reports the heterogeneous tiles workload (2048 crossbars of 32-256 rows
and columns, 256 input vectors each) through one batched library call.

The CPU baseline has two parts: the oracle (one core) on a bounded slice,
scaled to the workload, and LAPACK's banded Cholesky (dpbtrf / dpbtrs through
SciPy) factored once with the input vectors split over worker processes on the
host's cores, also on a bounded slice and scaled.

Prints one JSON line.  --gpus N > 1 is refused: the solver runs on one GPU.
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
IR_TOL = 1e-10               # refinement stop of the float32 leg (its target is 1e-9 rel err)
# HBM traffic of the dominant kernel per launch, from two counter runs (FETCH_SIZE,
# WRITE_SIZE) scaled by what the same counters read for a plain copy; valid only
# while the kernel's sources are unchanged since the counters were taken.
CSRC = os.path.join(ROOT, "paper_2410_19993_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_kernel_c3_512x512_b4096_traffic.txt")
KERNEL_SOURCES = [os.path.join(CSRC, f) for f in ("sweep.hip", "common.h")]
APPLY_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "transfer_apply_kernel_c3_512x512_b4096.md")
APPLY_SOURCES = [os.path.join(CSRC, "transfer.hip")]
METRIC = ("input-vector solves/s, 512×512 xbar: FP64 LU vs FP32+IR at 1e-9 rel err")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(wl, rows=64, vectors=128):
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
                       f"input vectors: assembly and banded LU alone {t_fact:.1f} s, then the whole "
                       f"solve (LU and substitution) {t_all:.1f} s; time scaled x{scale:g} in rows "
                       f"and to {wl.B} vectors (banded LU and substitution cost are linear in rows)"),
            "seconds_measured": t_all + t_fact, "extrapolated_seconds": t_full}


def host_description():
    """CPU model, logical CPU count and BLAS thread setting of this host."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        import threadpoolctl
        blas = [{"api": d.get("internal_api"), "threads": d.get("num_threads")}
                for d in threadpoolctl.threadpool_info() if d.get("user_api") == "blas"]
    except Exception:
        pass
    return {"cpu_model": model, "cpu_count": os.cpu_count(), "blas": blas}


def _lapack_worker(args):
    """Worker process: attach the shared Cholesky factor and solve a chunk of vectors."""
    name, shape, rhs = args
    import threadpoolctl
    from multiprocessing import shared_memory

    import scipy.linalg as sl
    with threadpoolctl.threadpool_limits(1):
        shm = shared_memory.SharedMemory(name=name)
        try:
            c = np.ndarray(shape, dtype=np.float64, buffer=shm.buf)
            t0 = time.perf_counter()
            sl.cho_solve_banded((c, False), rhs, check_finite=False)
            return time.perf_counter() - t0
        finally:
            shm.close()


def lapack_baseline(wl, rows=64, per_worker=8, workers=None):
    """LAPACK banded Cholesky on the host's cores: the nodal matrix of rows 0..rows-1
    of the crossbar (the same half-bandwidth 2n as the full one) is factored once
    (dpbtrf, all BLAS threads), then `workers` processes (one BLAS thread each) solve
    `per_worker` input vectors each (dpbtrs) against the shared factor.  Factor and
    per-vector solve cost are linear in the rows, so the full workload's time is
    estimated as 8 x (factor) + ceil(B / workers) x 8 x (per-vector solve)."""
    import multiprocessing as mp
    from multiprocessing import shared_memory

    import scipy.linalg as sl

    import oracle
    g = wl.geom
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    Gs = np.ascontiguousarray(wl.G[:rows])
    net = oracle.build_netlist(Gs, g.r_wl, g.r_bl, g.r_src, g.r_sense)
    ab, w = oracle.assemble_band(net)              # ab[r][c - r + w]
    N = ab.shape[0]
    au = np.zeros((w + 1, N))                      # LAPACK upper band: au[w + r - c][c]
    for d in range(w + 1):
        au[w - d, d:] = ab[:N - d, w + d]
    del ab
    t0 = time.perf_counter()
    c = sl.cholesky_banded(au, lower=False, overwrite_ab=True, check_finite=False)
    t_fact = time.perf_counter() - t0
    shm = shared_memory.SharedMemory(create=True, size=c.nbytes)
    try:
        np.ndarray(c.shape, dtype=np.float64, buffer=shm.buf)[:] = c
        del c, au
        rhs = oracle.injections(net, wl.V[:per_worker * workers, :rows])
        jobs = [(shm.name, (w + 1, N), np.ascontiguousarray(rhs[:, k * per_worker:(k + 1) * per_worker]))
                for k in range(workers)]
        ctx = mp.get_context("spawn")
        with ctx.Pool(workers) as pool:
            pool.map(_lapack_worker, jobs[:1])              # start-up and first touch
            t0 = time.perf_counter()
            times = pool.map(_lapack_worker, jobs)
            t_solve = time.perf_counter() - t0
    finally:
        shm.close()
        shm.unlink()
    per_vec = t_solve / per_worker                 # wall time per vector per worker, all busy
    scale = wl.G.shape[0] / rows
    t_full = scale * (t_fact + -(-wl.B // workers) * per_vec)
    return {"value": wl.B / t_full, "unit": "solves/s", "cores": workers, "kind": "lapack_banded_cholesky",
            "sample": (f"dpbtrf of rows 0-{rows - 1} ({N} unknowns, half-bandwidth {w}) in {t_fact:.2f} s, "
                       f"then {workers} processes x {per_worker} vectors (dpbtrs, one BLAS thread each) in "
                       f"{t_solve:.2f} s; scaled x{scale:g} in rows and to {wl.B} vectors"),
            "factor_s_measured": t_fact, "solve_s_measured": t_solve,
            "worker_s": [round(x, 3) for x in times], "extrapolated_seconds": t_full}


def copy_probe(gib):
    """A plain device copy of known size (torch's elementwise copy, three times), run
    under the traffic counters to calibrate FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = int(gib * (1 << 30)) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8, "copies": 3}))


def kernel_source_hash(sources=KERNEL_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, record=TRAFFIC_FILE, sources=KERNEL_SOURCES):
    """Bytes per launch of a kernel from its committed counter summary, or None."""
    try:
        with open(record) as fh:
            rec = json.loads(fh.read().split("JSON:", 1)[1])
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash(sources) or rec.get("workload") != workload:
        return None
    return rec.get("bytes_per_launch")


def run_bf16(steps, r=2.5):
    """The bfloat16 factor with the classical float64 refinement and with the GMRES
    refinement around it, each timed per step (assemble, factor, solve, currents) with its
    status, refinement steps and error against stored oracle currents, on two workloads:
    128 x 128 with 1024 input vectors (2.5-ohm segments), and the 512 x 512 crossbar with
    32 of its stored-oracle input vectors (segment resistance r)."""
    import torch

    import paper_2410_19993_amd as xb
    import workloads
    cases = []
    wl = workloads.c2()
    path = os.path.join(ROOT, "tests", "golden", "c2_currents.npy")
    cases.append(("c2_128x128_b1024_r2.5", wl.G, np.ascontiguousarray(wl.V), wl.geom,
                  np.load(path) if os.path.exists(path) else None))
    w3 = workloads.c3(r=r)
    sub = workloads.c3_subset()[:32]
    path = os.path.join(ROOT, "tests", "golden", f"c3_r{r:g}_currents.npy")
    cases.append((f"c3_512x512_b32_r{r:g}", w3.G, np.ascontiguousarray(w3.V[sub]), w3.geom,
                  np.load(path)[:32] if os.path.exists(path) else None))
    out = {"ir_tol": 1e-12, "ir_max_iter": 30}
    for name, Gh, Vh, g, ref in cases:
        m, n = Gh.shape
        B = Vh.shape[0]
        G = torch.from_numpy(Gh).cuda()
        V = torch.from_numpy(Vh).cuda()
        I = torch.empty((B, n), dtype=torch.float64, device="cuda")
        entry = {}
        for prec in ("bf16_ir", "bf16_gmres"):
            plan = xb.Plan(m, n, g.r_wl, g.r_bl, g.r_src, g.r_sense, prec, max_batch=B, ir_tol=1e-12,
                           ir_max_iter=30)

            def step():
                plan.assemble(G)
                plan.factor()
                plan.solve_batch(V)
                plan.currents(I)

            step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                step()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            st, info = plan.info()
            err = None
            if ref is not None:
                Ih = I.cpu().numpy()
                err = float((np.max(np.abs(Ih - ref), axis=1) / np.max(np.abs(ref), axis=1)).max())
            plan.close()
            entry[prec] = {"status": xb.status_string(st), "refinement_steps": int(info.ir_iters),
                           "ms_per_step": ms, "solves_per_s": B / (ms * 1e-3), "max_rel_err_vs_oracle": err}
            log(f"bf16 {name} {prec}: {xb.status_string(st)}, {info.ir_iters} refinement steps, {ms:.2f} ms/step, "
                f"max rel err {err}")
        out[name] = entry
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--r", type=float, default=2.5)
    ap.add_argument("--no-fp32-ir", action="store_true", help="skip the float32+refinement leg")
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-shortcuts", action="store_true",
                    help="skip the currents-only and transfer-matrix legs")
    ap.add_argument("--no-tiles", action="store_true", help="skip the heterogeneous tiles leg")
    ap.add_argument("--no-r-sweep", action="store_true",
                    help="skip the float64 and float32+refinement steps at the other segment resistances")
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the bfloat16-factor legs (classical and GMRES refinement)")
    ap.add_argument("--copy-probe", type=float, default=None, metavar="GIB",
                    help="only run a plain device copy of GIB GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the solver has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe is not None:
        copy_probe(args.copy_probe)
        return

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
    gold = os.path.join(ROOT, "tests", "golden", f"c3_r{g.r_wl:g}_currents.npy")

    def verify(path=None):
        path = path or gold
        if args.no_verify or not os.path.exists(path) or B != 4096:
            return None
        ref = np.load(path)
        Ih = I.cpu().numpy()[workloads.c3_subset()]
        return float((np.max(np.abs(Ih - ref), axis=1) / np.max(np.abs(ref), axis=1)).max())

    def run(precision, steps, warmup, ir_tol=0.0, nodes=True, geom=None, verify_fn=None):
        gg = geom or g
        plan = xb.Plan(m, n, gg.r_wl, gg.r_bl, gg.r_src, gg.r_sense, precision, max_batch=B,
                       ir_tol=ir_tol, stream=stream)

        def step():
            plan.assemble(G)
            plan.factor()
            plan.solve_batch(V, node_v if nodes else None)
            plan.currents(I)

        for w in range(warmup):
            step()
            torch.cuda.synchronize()
            log(f"{precision}: warmup step {w} done")
        plan.check()
        plan.set_timing(True)
        plan.timing(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        tm = plan.timing()
        st, info = plan.info()
        plan.check()
        err = (verify_fn or verify)()
        plan.close()
        log(f"{precision}{'' if nodes else ' currents only'}: {steps} steps in {wall:.3f} s")
        return wall * 1e3 / steps, tm, info, err

    def run_transfer(steps, reps=50):
        """Currents through the transfer matrix: per conductance map assemble, factor and
        T (block recurrences on the factorization); per batch one float64 matrix-core
        product I = V T."""
        plan = xb.Plan(m, n, g.r_wl, g.r_bl, g.r_src, g.r_sense, "fp64", max_batch=B, stream=stream)
        T = torch.empty((m, n), dtype=torch.float64, device="cuda")

        def per_map():
            plan.assemble(G)
            plan.factor()
            plan.transfer(T)

        per_map()
        plan.transfer_apply(T, V, I)
        torch.cuda.synchronize()
        plan.check()
        t0 = time.perf_counter()
        for _ in range(steps):
            per_map()
            plan.transfer_apply(T, V, I)
        torch.cuda.synchronize()
        step_ms = (time.perf_counter() - t0) * 1e3 / steps
        t0 = time.perf_counter()
        for _ in range(steps):
            per_map()
        torch.cuda.synchronize()
        map_ms = (time.perf_counter() - t0) * 1e3 / steps
        # the product alone, timed with events on the stream it is launched on
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            plan.transfer_apply(T, V, I)
        e1.record(stream)
        torch.cuda.synchronize()
        apply_ms = e0.elapsed_time(e1) / reps
        plan.check()
        err = verify()
        plan.close()
        flops = 2.0 * B * m * n
        log(f"transfer: per map {map_ms:.2f} ms, product {apply_ms * 1e3:.1f} us")
        return {"value": B / (step_ms * 1e-3), "unit": "solves/s", "ms_per_step": step_ms,
                "per_map_ms": map_ms, "apply_ms": apply_ms,
                "apply_solves_per_s": B / (apply_ms * 1e-3),
                "apply_roofline": {"bound": "mfma", "kernel": "transfer_apply_kernel<true>",
                                   "achieved": flops / (apply_ms * 1e-3) / 1e12,
                                   "peak": PEAK_FP64_MFMA / 1e12, "unit": "TFLOP/s",
                                   "frac": flops / (apply_ms * 1e-3) / PEAK_FP64_MFMA,
                                   "traffic": measured_traffic(wl.name, APPLY_TRAFFIC_FILE, APPLY_SOURCES),
                                   "flops_per_launch": flops},
                "max_rel_err_vs_oracle": err}

    def run_tiles(steps):
        """The heterogeneous tiles workload: 2048 crossbars of 32..256 rows and columns,
        256 input vectors each, currents only, in one library call (TileBatch) with the
        tuned configuration of every class; eager, and captured once into a HIP graph
        and replayed."""
        tl = workloads.c4()
        by = {}
        for t in tl:
            by.setdefault((t.G.shape[0], t.G.shape[1], t.V.shape[0]), []).append(t)
        keys = sorted(by)
        classes = [(mm, nn, len(by[(mm, nn, bb)]), bb) for (mm, nn, bb) in keys]
        Gs = [torch.from_numpy(np.stack([t.G for t in by[k]])).cuda() for k in keys]
        Vs = [torch.from_numpy(np.stack([t.V for t in by[k]])).cuda() for k in keys]
        Is = [torch.empty((c, bb, nn), dtype=torch.float64, device="cuda") for (mm, nn, c, bb) in classes]
        g4 = workloads.C4_GEOM
        # the method's work, rows ordered as the crossbar's (m n^3 factor, 2 m n^2 per vector)
        flops = sum(c * (mm * nn ** 3 + 2.0 * mm * nn * nn * bb) for (mm, nn, c, bb) in classes)
        with xb.TileBatch(classes, g4["r_wl"], g4["r_bl"], g4["r_src"], g4["r_sense"], stream=stream) as tb:
            tb.run(Gs, Vs, Is)
            torch.cuda.synchronize()
            assert all(bool(torch.isfinite(I).all()) for I in Is), "tile currents not finite"
            t0 = time.perf_counter()
            for _ in range(steps):
                tb.run(Gs, Vs, Is)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            side = torch.cuda.Stream()
            side.wait_stream(stream)
            with xb.TileBatch(classes, g4["r_wl"], g4["r_bl"], g4["r_src"], g4["r_sense"], stream=side) as tg:
                with torch.cuda.stream(side):
                    tg.run(Gs, Vs, Is)
                side.synchronize()
                graph = torch.cuda.CUDAGraph()
                with torch.cuda.graph(graph, stream=side):
                    tg.run(Gs, Vs, Is)
                graph.replay()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    graph.replay()
                torch.cuda.synchronize()
                ms_graph = (time.perf_counter() - t0) * 1e3 / steps
            configs = {f"{mm}x{nn}": {"tiles": c, "method": cf.method, "block": cf.block, "split": cf.split,
                                      "transpose": cf.transpose, "source": src}
                       for (mm, nn, c, bb), cf, src in zip(classes, tb.configs, tb.sources)}
            streams = tb.streams
            ws_bytes = tb.workspace_bytes
        vecs = 256 * len(tl)
        log(f"tiles: {len(tl)} crossbars in {len(classes)} classes, {ms:.2f} ms per pass "
            f"({ms_graph:.2f} ms as a graph replay)")
        return {"value": vecs / (ms * 1e-3), "unit": "solves/s", "ms_per_pass": ms,
                "ms_per_pass_graph_replay": ms_graph, "tiles": len(tl), "classes": len(classes),
                "tiles_per_s": len(tl) / (ms * 1e-3), "streams": streams, "workspace_bytes": ws_bytes,
                "per_class": configs,
                "workload": "c4 tiles (seed 1004): 2048 crossbars of {32,64,128,256}^2, 256 vectors each, "
                            "currents only, one TileBatch call",
                "algorithmic_flops": flops, "tflops": flops / (ms * 1e-3) / 1e12,
                "roofline": {"bound": "mfma", "achieved": flops / (ms * 1e-3) / 1e12, "peak": PEAK_FP64_MFMA / 1e12,
                             "unit": "TFLOP/s", "frac": flops / (ms * 1e-3) / PEAK_FP64_MFMA,
                             "note": "work counted as the row-ordered method's m n^3 + 2 m n^2 B per crossbar"}}

    ms64, tm, info64, err64 = run("fp64", args.steps, args.warmup)
    # kernels: algorithmic work per launch
    sweep_flops = 2.0 * n * n * B * (2 * m - 1)          # forward m products + back (m-1)
    factor_flops = float(m) * n ** 3                     # m SPD inverses of n x n
    per = lambda ms, k: ms / max(k, 1)
    k_sweep = per(tm.sweep_ms, tm.sweep_launches)
    k_factor = per(tm.factor_ms, tm.factor_launches)
    k_recover = per(tm.recover_ms, tm.recover_launches)
    k_condense = per(tm.condense_ms, tm.condense_launches)
    recover_bytes = 8.0 * B * m * n * (1 + 2) + 8.0 * 3 * m * n     # read u, write w and u
    achieved = sweep_flops / (k_sweep * 1e-3)
    # each phase at its own roof: the condensed blocks written once (HBM), the method's
    # m n^3 factor flops and the sweep's flops at the float64 matrix peak
    condense_bytes = 8.0 * m * (64 * ((n + 63) // 64)) ** 2 + 8.0 * m * n
    bound_ms = {"condense": condense_bytes / PEAK_HBM * 1e3, "factor": factor_flops / PEAK_FP64_MFMA * 1e3,
                "sweep": sweep_flops / PEAK_FP64_MFMA * 1e3}
    roof = {"bound": "mfma", "kernel": "sweep_kernel<double,8>", "achieved": achieved / 1e12,
            "peak": PEAK_FP64_MFMA / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_MFMA,
            "traffic": measured_traffic(wl.name), "flops_per_launch": sweep_flops,
            "avg_launch_ms": k_sweep}
    result = {
        "metric": METRIC, "value": B / (ms64 * 1e-3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms64,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "m": m, "n": n, "batch": B, "r_segment_ohm": g.r_wl,
                   "r_src_ohm": g.r_src, "r_sense_ohm": g.r_sense, "precision": "fp64",
                   "node_voltages": True, "parallelism": "single-gpu"},
        "phases_ms": {"condense": k_condense, "factor": k_factor, "sweep": k_sweep,
                      "recover": k_recover},
        "factor": {"algorithmic_flops": factor_flops, "ms": k_factor,
                   "tflops": factor_flops / (k_factor * 1e-3) / 1e12},
        "recover": {"ms": k_recover, "bytes": recover_bytes,
                    "gbps": recover_bytes / (k_recover * 1e-3) / 1e9 if k_recover > 0 else None},
        "roofline": roof,
        "step_roofline": {"bound_ms": bound_ms, "t_bound_ms": sum(bound_ms.values()),
                          "frac": sum(bound_ms.values()) / ms64},
        "max_rel_err_vs_oracle": err64,
    }
    # Exact shortcuts, outside the metric: the same fp64 path without node voltages, the
    # substitution sweeps alone, and currents through the transfer matrix.
    if not args.no_shortcuts:
        msc, tmc, _, errc = run("fp64", args.steps, args.warmup, nodes=False)
        result["currents_only"] = {
            "value": B / (msc * 1e-3), "unit": "solves/s", "ms_per_step": msc,
            "sweep_ms": per(tmc.sweep_ms, tmc.sweep_launches),
            "solve_only_solves_per_s": B / (per(tmc.sweep_ms, tmc.sweep_launches) * 1e-3),
            "max_rel_err_vs_oracle": errc}
        result["solve_only"] = {"value": B / (k_sweep * 1e-3), "unit": "solves/s",
                                "note": "fp64 sweeps with node voltages, factor excluded"}
        result["transfer"] = run_transfer(args.steps)
    if not args.no_tiles:
        result["tiles"] = run_tiles(args.steps)
    if not args.no_fp32_ir:
        # The metric's accuracy target for this leg is 1e-9 relative error on the currents:
        # refinement stops once its error estimate is below 1e-10 (the error actually
        # reached, measured against the oracle, is reported beside it, and a result above
        # 1e-9 marks the leg invalid).
        ms32, tm32, info32, err32 = run("fp32_ir", args.steps, args.warmup, ir_tol=IR_TOL)
        # the refined solve launches 1 + ir_max_iter sweeps (and a residual before each but
        # the first); slabs that have converged leave the later launches at once, so the
        # work is counted per solve: `sweeps` full sweeps and sweeps - 1 full residuals
        nsw = max(int(info32.ir_iters), 1)
        k_ir = tm32.ir_sweep_ms / max(args.steps, 1) / nsw          # per full sweep
        k_res = tm32.residual_ms / max(args.steps, 1) / max(nsw - 1, 1)
        ir_flops = 2.0 * n * n * B * (2 * m - 1)        # one float32 sweep: forward m, back m - 1 products
        res_bytes = 8.0 * B * m * n + 4.0 * B * m * n   # reads U (float64), writes R (float32)
        ok32 = err32 is not None and err32 <= 1e-9
        result["fp32_ir"] = {
            "value": B / (ms32 * 1e-3), "unit": "solves/s", "ms_per_step": ms32, "dtype": "f32+f64",
            "valid": ok32 if err32 is not None else None,
            "sweeps": int(info32.ir_iters), "ir_tol": IR_TOL, "max_rel_err_vs_oracle": err32,
            "phases_ms": {"condense": per(tm32.condense_ms, tm32.condense_launches),
                          "factor": per(tm32.factor_ms, tm32.factor_launches),
                          "refined_solve": per(tm32.sweep_ms, tm32.sweep_launches),
                          "recover": per(tm32.recover_ms, tm32.recover_launches),
                          "float32_sweep_per_full_sweep": k_ir, "float64_residual_per_full_pass": k_res},
            "roofline": {"bound": "mfma", "kernel": "sweep_kernel<float,8,true,false>",
                         "achieved": ir_flops / (k_ir * 1e-3) / 1e12 if k_ir > 0 else None,
                         "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s",
                         "frac": ir_flops / (k_ir * 1e-3) / PEAK_FP32_MFMA if k_ir > 0 else None,
                         "flops_per_sweep": ir_flops, "ms_per_sweep": k_ir,
                         "note": "sweep time per solve / sweeps the slowest slab took"},
            "residual_roofline": {"bound": "hbm", "kernel": "residual_kernel",
                                  "achieved": res_bytes / (k_res * 1e-3) / 1e9 if k_res > 0 else None,
                                  "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                                  "frac": res_bytes / (k_res * 1e-3) / PEAK_HBM if k_res > 0 else None,
                                  "bytes_per_pass": res_bytes},
            "speedup_vs_fp64": ms64 / ms32}
        if not ok32 and err32 is not None:
            log(f"fp32_ir: error {err32:.3e} above 1e-9: leg marked invalid")
    if not args.no_r_sweep and B == 4096:
        # the other segment resistances of the 512 x 512 workload (same G and V): both
        # precisions, fewer steps, each with its error against the stored oracle currents
        sweep = {}
        for rr in workloads.C3_R:
            if rr == g.r_wl:
                continue
            wr = workloads.c3(r=rr, batch=B)
            path = os.path.join(ROOT, "tests", "golden", f"c3_r{rr:g}_currents.npy")
            entry = {}
            for prec, tol in (("fp64", 0.0), ("fp32_ir", IR_TOL)):
                if prec == "fp32_ir" and args.no_fp32_ir:
                    continue
                msr, tmr, infor, errr = run(prec, max(2, args.steps // 4), 1, ir_tol=tol, geom=wr.geom,
                                            verify_fn=lambda p=path: verify(p))
                entry[prec] = {"value": B / (msr * 1e-3), "ms_per_step": msr, "max_rel_err_vs_oracle": errr,
                               "sweeps": int(infor.ir_iters) if prec != "fp64" else None,
                               "factor_ms": per(tmr.factor_ms, tmr.factor_launches),
                               "sweep_ms": per(tmr.sweep_ms, tmr.sweep_launches)}
            sweep[f"r{rr:g}"] = entry
        result["r_sweep"] = sweep
    if not args.no_bf16:
        result["bf16"] = run_bf16(max(2, args.steps))
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample ...")
        cb = cpu_baseline(wl)
        cb.update(host_description())
        log("timing LAPACK banded Cholesky over the host's cores on a bounded sample ...")
        try:
            cb["lapack_all_cores"] = lapack_baseline(wl)
        except Exception as e:                     # reported, not fatal: the oracle figure stands
            cb["lapack_all_cores"] = {"error": repr(e)}
        result["cpu_baseline"] = cb
    print(json.dumps(result))


if __name__ == "__main__":
    main()
