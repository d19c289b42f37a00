"""Heterogeneous batches of crossbars through one library call (xbar_tiles_*), and
the tuner that picks how each class of crossbars is solved.

A batch is a list of classes (m, n, count, B): `count` crossbars of m x n with B
input vectors each.  Each class is solved either by one workgroup per crossbar
("one_wg", n <= 64, with a padded block size and a split of the vectors over 1-4
workgroups) or by the plan path's kernels batched over the class ("pipeline").
The choice per class comes from the tuning cache (tiles_tuning.json next to this
file, written by `python -m paper_2410_19993_amd.tiles tune`), keyed by the GPU's
name and the class's m, n and B; classes the cache does not hold get the default
(one_wg with the smallest block for n <= 64, pipeline otherwise).  All arithmetic
runs in the library's kernels; this module only groups, times and marshals.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import asdict, dataclass

from . import _check_tensor, _lib

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE_PATH = os.path.join(HERE, "tiles_tuning.json")
METHODS = {"one_wg": _lib.XBAR_TILE_ONE_WG, "pipeline": _lib.XBAR_TILE_PIPELINE}
DEFAULT_STREAMS = 4


def _torch():
    import torch
    return torch


@dataclass(frozen=True)
class TileConfig:
    """How one class is solved: method "one_wg" (block 16/32/64 or 0 = smallest,
    split 1..4) or "pipeline" (block 0, split 1), applied to the class itself or, with
    transpose, to its reciprocal problem (the crossbar turned and transposed, n rows of
    m columns, driven by n unit inputs; then I = V T)."""
    method: str
    block: int = 0
    split: int = 1
    transpose: bool = False

    def valid_for(self, m: int, n: int, B: int = 256) -> bool:
        ni, Bi = (m, n) if self.transpose else (n, B)
        if Bi > 256:
            return False
        if self.method == "pipeline":
            return self.block == 0 and self.split == 1 and ni <= 512
        if self.method != "one_wg" or ni > 64 or not 1 <= self.split <= 4:
            return False
        return self.block == 0 or (self.block in (16, 32, 64) and self.block >= ni)


def default_config(m: int, n: int) -> TileConfig:
    """One workgroup per crossbar for n <= 64; for wider crossbars with fewer rows
    than columns the reciprocal problem (blocks of m), else the batched plan kernels."""
    if n <= 64:
        return TileConfig("one_wg", 0, 1)
    if m < n and n <= 256:
        return TileConfig("one_wg" if m <= 64 else "pipeline", 0, 1, True)
    return TileConfig("pipeline")


def class_key(m: int, n: int, B: int) -> str:
    return f"{m}x{n}x{B}"


def device_name() -> str:
    """The cache's device key: the GPU's architecture and compute-unit count."""
    props = _torch().cuda.get_device_properties(0)
    arch = str(getattr(props, "gcnArchName", "")).split(":")[0] or props.name
    return f"{arch} with {props.multi_processor_count} CUs"


def load_cache(path: str = CACHE_PATH) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def resolve(classes, cache: dict, device: str):
    """(configs, streams, sources): the cached configuration of every class (m, n,
    count, B) for `device`, or the default where the cache has none or an invalid one.
    sources[k] is "cache" or "default"."""
    entry = cache.get("devices", {}).get(device, {})
    tuned = entry.get("classes", {})
    configs, sources = [], []
    for (m, n, _count, B) in classes:
        rec = tuned.get(class_key(m, n, B))
        cfg = None
        if rec is not None:
            cfg = TileConfig(rec["method"], int(rec.get("block", 0)), int(rec.get("split", 1)),
                             bool(rec.get("transpose", False)))
            if not cfg.valid_for(m, n, B):
                cfg = None
        configs.append(cfg or default_config(m, n))
        sources.append("cache" if cfg is not None else "default")
    streams = int(entry.get("streams", DEFAULT_STREAMS))
    return configs, streams, sources


class TileBatch:
    """One heterogeneous batch: classes [(m, n, count, B)] with the resistances of every
    crossbar; configs and streams from the tuning cache unless given."""

    def __init__(self, classes, r_wl, r_bl, r_src=50.0, r_sense=50.0, configs=None, streams=None,
                 cache_path: str = CACHE_PATH, stream=None):
        torch = _torch()
        self.classes = [tuple(int(x) for x in c) for c in classes]
        cfgs, cstreams, sources = resolve(self.classes, load_cache(cache_path), device_name())
        if configs is not None:
            cfgs, sources = list(configs), ["given"] * len(configs)
        self.configs, self.sources = cfgs, sources
        self.streams = int(streams if streams is not None else cstreams)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        tc = []
        for (m, n, count, B), cfg in zip(self.classes, self.configs):
            if not cfg.valid_for(m, n, B):
                raise ValueError(f"class {m}x{n}: configuration {cfg} is not valid")
            tc.append(_lib.TileClass(m, n, count, B, METHODS[cfg.method], cfg.block, cfg.split, int(cfg.transpose)))
        self.r = (float(r_wl), float(r_bl), float(r_src), float(r_sense))
        self._t = _lib.xbar_tiles_create(tc, *self.r, self.streams, self.stream.cuda_stream)

    @property
    def workspace_bytes(self) -> int:
        return _lib.xbar_tiles_workspace_bytes(self._t)

    def run(self, Gs, Vs, Is=None):
        """Gs[k] [count][m][n], Vs[k] [count][B][m] float64 device tensors (class k);
        returns Is[k] [count][B][n], queued on the batch's stream."""
        torch = _torch()
        if len(Gs) != len(self.classes) or len(Vs) != len(self.classes):
            raise ValueError("one G and one V tensor per class")
        if Is is None:
            Is = [torch.empty((c, B, n), dtype=torch.float64, device="cuda") for (m, n, c, B) in self.classes]
        for k, (m, n, c, B) in enumerate(self.classes):
            _check_tensor(f"Gs[{k}]", Gs[k], (c, m, n))
            _check_tensor(f"Vs[{k}]", Vs[k], (c, B, m))
            _check_tensor(f"Is[{k}]", Is[k], (c, B, n))
        _lib.xbar_tiles_run(self._t, Gs, Vs, Is)
        return Is

    def close(self) -> None:
        if getattr(self, "_t", None) is not None:
            _lib.xbar_tiles_destroy(self._t)
            self._t = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def group(tiles):
    """Classes of a list of (G [m][n], V [B][m]) numpy crossbars: {(m, n, B): [indices]}."""
    out = {}
    for k, (G, V) in enumerate(tiles):
        out.setdefault((G.shape[0], G.shape[1], V.shape[0]), []).append(k)
    return out


def candidates(m: int, n: int, B: int = 256):
    """Configurations the tuner times for a class of m x n crossbars with B vectors:
    both methods on the class itself and, when m < n, on its reciprocal problem."""
    out = []
    for tr in ((False, True) if m < n else (False,)):
        ni = m if tr else n
        if ni <= 64:
            blocks = [b for b in (16, 32, 64) if b >= ni]
            out += [TileConfig("one_wg", b, s, tr) for b in blocks for s in (1, 2, 4)]
        out.append(TileConfig("pipeline", 0, 1, tr))
    return [c for c in out if c.valid_for(m, n, B)]


def _time(fn, reps: int, stream) -> float:
    """Median milliseconds of fn() over reps, HIP events on `stream` after one warm-up."""
    torch = _torch()
    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def tune(class_data, r, reps: int = 5, stream_choices=(2, 4, 6, 8), log=print):
    """Time every candidate of every class alone, then the whole batch with the chosen
    configurations for each stream count.  class_data: {(m, n, B): (G, V)} device
    tensors [count][m][n], [count][B][m].  Returns the cache entry for this device."""
    torch = _torch()
    stream = torch.cuda.current_stream()
    chosen, record = {}, {}
    for (m, n, B), (G, V) in sorted(class_data.items()):
        count = int(G.shape[0])
        times = {}
        for cfg in candidates(m, n, B):
            with TileBatch([(m, n, count, B)], *r, configs=[cfg], streams=1) as tb:
                I = [torch.empty((count, B, n), dtype=torch.float64, device="cuda")]
                times[cfg] = _time(lambda: tb.run([G], [V], I), reps, stream)
        best = min(times, key=times.get)
        chosen[(m, n, B)] = best
        record[class_key(m, n, B)] = {**asdict(best), "count": count, "ms": times[best],
                                      "candidates": {f"{c.method}/{c.block}/{c.split}{'/T' if c.transpose else ''}": t
                                                     for c, t in times.items()}}
        log(f"tune {m}x{n} B={B} ({count} crossbars): {best.method} block {best.block} split {best.split} "
            f"{'transposed ' if best.transpose else ''}{times[best]:.3f} ms")
    keys = sorted(class_data)
    classes = [(m, n, int(class_data[(m, n, B)][0].shape[0]), B) for (m, n, B) in keys]
    Gs = [class_data[k][0] for k in keys]
    Vs = [class_data[k][1] for k in keys]
    Is = [torch.empty((c, B, n), dtype=torch.float64, device="cuda") for (m, n, c, B) in classes]
    whole = {}
    for ns in stream_choices:
        with TileBatch(classes, *r, configs=[chosen[k] for k in keys], streams=ns) as tb:
            whole[ns] = _time(lambda: tb.run(Gs, Vs, Is), reps, stream)
        log(f"tune whole batch, {ns} streams: {whole[ns]:.3f} ms")
    best_ns = min(whole, key=whole.get)
    return {"classes": record, "streams": best_ns, "whole_batch_ms": {str(k): v for k, v in whole.items()},
            "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S"), "resistances_ohm": list(r)}


def write_cache(entry: dict, device: str, path: str = CACHE_PATH) -> None:
    cache = load_cache(path)
    cache.setdefault("format", 1)
    cache.setdefault("devices", {})[device] = entry
    with open(path, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
        fh.write("\n")


def _main(argv):
    """python -m paper_2410_19993_amd.tiles tune [--reps R] [--out PATH]: tune the
    heterogeneous tiles workload's classes (2048 crossbars of 32..256 rows and columns,
    256 input vectors each, seed 1004) on this GPU and write the cache."""
    import argparse
    import sys

    import numpy as np
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["tune"])
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=CACHE_PATH)
    args = ap.parse_args(argv)
    torch = _torch()
    sys.path.insert(0, os.path.dirname(HERE))
    import workloads
    g = workloads.C4_GEOM
    r = (g["r_wl"], g["r_bl"], g["r_src"], g["r_sense"])
    by_class = {}
    for t in workloads.c4():
        by_class.setdefault((t.G.shape[0], t.G.shape[1], t.V.shape[0]), []).append(t)
    data = {k: (torch.from_numpy(np.stack([t.G for t in ts])).cuda(),
                torch.from_numpy(np.stack([t.V for t in ts])).cuda()) for k, ts in by_class.items()}
    entry = tune(data, r, reps=args.reps, log=lambda *a: print(*a, flush=True))
    entry["workload"] = "c4 (seed 1004): 2048 crossbars, 16 classes, 256 vectors each"
    write_cache(entry, device_name(), args.out)
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    import sys
    _main(sys.argv[1:])
