"""Heterogeneous crossbar batches (xbar_tiles_*, TileBatch) on a GPU.

Every crossbar's currents are compared with the oracle's (per-vector relative error
<= 1e-10), for both ways of solving a class: one workgroup per crossbar (blocks and
vector splits the tuner chooses among) and the plan path's kernels batched over the
class (condensation, twisted block Gauss-Jordan factor, currents-only sweep), on
ragged shapes: m = 1, n not a multiple of 64 (70, 130, 300), B not a multiple of 16,
class sizes that are not multiples of the 8 XCDs.  Also: a bad conductance spoils
only its own crossbar, a captured graph replays the eager bits, the whole
heterogeneous tiles workload matches stored oracle currents class by class, and the
tuning cache decides the configuration.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import GOLDEN, TOL_FP64, log, rel_err

pytestmark = pytest.mark.gpu

R = (1.5, 3.0, 40.0, 60.0)


def _class(m, n, count, B, seed):
    rng = np.random.default_rng(seed)
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (count, m, n)))
    V = rng.uniform(0.0, 0.5, (count, B, m))
    return G, V


def _run(classes, data, configs=None, streams=None, r=R):
    import torch

    import paper_2410_19993_amd as xb
    Gs = [torch.from_numpy(G).cuda() for G, _ in data]
    Vs = [torch.from_numpy(V).cuda() for _, V in data]
    with xb.TileBatch(classes, *r, configs=configs, streams=streams) as tb:
        Is = tb.run(Gs, Vs)
        torch.cuda.synchronize()
        return [I.cpu().numpy() for I in Is], tb.configs


def _check(classes, data, out, r=R, skip=()):
    worst = 0.0
    for k, ((m, n, count, B), (G, V)) in enumerate(zip(classes, data)):
        for t in range(count):
            if (k, t) in skip:
                continue
            ref = oracle.solve(G[t], V[t], *r).currents
            e = float(rel_err(out[k][t], ref).max())
            worst = max(worst, e)
            assert np.all(np.isfinite(out[k][t])) and e <= TOL_FP64, (m, n, t, e)
    return worst


PIPE_CASES = [(40, 70, 3, 20), (5, 130, 9, 33), (1, 100, 2, 5), (65, 64, 3, 16), (3, 300, 2, 17), (2, 1, 4, 3)]


def test_pipeline_classes_against_oracle():
    from paper_2410_19993_amd.tiles import TileConfig
    classes = PIPE_CASES
    data = [_class(*c, seed=300 + k) for k, c in enumerate(classes)]
    log(f"case pipeline classes {classes}")
    out, _ = _run(classes, data, configs=[TileConfig("pipeline")] * len(classes), streams=3)
    log(f"  max current rel err {_check(classes, data, out):.3e}")


@pytest.mark.parametrize("m,n", [(6, 130), (9, 260)])
def test_column_factor_matches_tile_factor_bits(m, n):
    """Nine crossbars with three or more 64-column blocks (eighteen or nine jobs per
    launch) are factored with one workgroup per column block of each job; a crossbar
    alone (one or two jobs) with one workgroup per tile.  Both form the same products
    in the same order, and the batched sweep runs the same arithmetic per vector, so
    every crossbar's currents agree bit for bit; the batch also meets the oracle."""
    from paper_2410_19993_amd.tiles import TileConfig
    G, V = _class(m, n, 9, 24, seed=350 + n)
    log(f"case column factor {m}x{n}, 9 crossbars")
    out, _ = _run([(m, n, 9, 24)], [(G, V)], configs=[TileConfig("pipeline")], streams=1)
    for t in range(9):
        one, _ = _run([(m, n, 1, 24)], [(G[t:t + 1], V[t:t + 1])], configs=[TileConfig("pipeline")], streams=1)
        assert np.array_equal(out[0][t], one[0][0]), t
    log(f"  bitwise equal; max current rel err {_check([(m, n, 9, 24)], [(G, V)], out):.3e}")


@pytest.mark.parametrize("m,n", [(6, 130), (7, 100)])
def test_large_batch_eliminates_every_pivot_tile(m, n):
    """Above 256 crossbars a class's pivot tiles are all eliminated (no Newton-Schulz
    slots): 300 crossbars with three (column workgroups) or two (tile workgroups)
    64-column blocks; sampled crossbars across the batch meet the oracle."""
    from paper_2410_19993_amd.tiles import TileConfig
    T, B = 300, 4
    G, V = _class(m, n, T, B, seed=371 + n)
    log(f"case large batch: {T} crossbars of {m}x{n}")
    out, _ = _run([(m, n, T, B)], [(G, V)], configs=[TileConfig("pipeline")], streams=1)
    assert np.all(np.isfinite(out[0]))
    worst = 0.0
    for t in (0, 1, 7, 8, 150, 298, 299):
        ref = oracle.solve(G[t], V[t], *R).currents
        worst = max(worst, float(rel_err(out[0][t], ref).max()))
    log(f"  sampled max current rel err {worst:.3e}")
    assert worst <= TOL_FP64


@pytest.mark.parametrize("method", ["one_wg", "pipeline"])
def test_reciprocal_classes_against_oracle(method):
    """Classes solved through their reciprocal problem (the turned, transposed crossbar
    driven by unit inputs, then I = V T): m < n, m = 1, n not a multiple of 16 or 64,
    n up to 256 unit inputs."""
    from paper_2410_19993_amd.tiles import TileConfig
    classes = [(12, 70, 3, 20), (5, 130, 4, 33), (1, 40, 2, 7), (33, 256, 2, 16), (40, 41, 3, 9)]
    data = [_class(*c, seed=800 + k) for k, c in enumerate(classes)]
    cfgs = [TileConfig(method, 0, 1, True) for _ in classes]
    log(f"case reciprocal classes through {method}: {classes}")
    out, _ = _run(classes, data, configs=cfgs, streams=3)
    log(f"  max current rel err {_check(classes, data, out):.3e}")


@pytest.mark.parametrize("block,split", [(0, 1), (64, 1), (32, 2), (64, 4), (16, 3)])
def test_one_wg_blocks_and_splits_against_oracle(block, split):
    from paper_2410_19993_amd.tiles import TileConfig
    classes = [(9, 12, 5, 37), (33, 16, 3, 256), (1, 7, 2, 9), (20, 30, 4, 100)]
    data = [_class(*c, seed=400 + k) for k, c in enumerate(classes)]
    cfgs = [TileConfig("one_wg", block if block >= n else 0, split) for (_, n, _, _) in classes]
    log(f"case one-workgroup classes, block {block}, split {split}")
    out, _ = _run(classes, data, configs=cfgs, streams=2)
    log(f"  max current rel err {_check(classes, data, out):.3e}")


def test_bad_conductance_spoils_only_its_crossbar():
    from paper_2410_19993_amd.tiles import TileConfig
    classes = [(12, 130, 4, 16), (12, 40, 4, 16), (10, 60, 3, 8)]
    data = [_class(*c, seed=500 + k) for k, c in enumerate(classes)]
    data[0][0][2][3, 7] = 0.0
    data[1][0][1][5, 9] = np.nan
    data[2][0][0][9, 59] = -1e-5
    log("case bad conductances in a pipeline, a one-workgroup and a reciprocal class")
    out, _ = _run(classes, data, configs=[TileConfig("pipeline"), TileConfig("one_wg"),
                                          TileConfig("one_wg", 0, 1, True)], streams=2)
    assert np.all(np.isnan(out[0][2])) and np.all(np.isnan(out[1][1])) and np.all(np.isnan(out[2][0]))
    _check(classes, data, out, skip={(0, 2), (1, 1), (2, 0)})


def test_tile_batch_graph_replays_eager_bits():
    import torch

    import paper_2410_19993_amd as xb
    from paper_2410_19993_amd.tiles import TileConfig
    classes = [(24, 140, 3, 32), (40, 64, 5, 48), (16, 32, 7, 64)]
    data = [_class(*c, seed=600 + k) for k, c in enumerate(classes)]
    Gs = [torch.from_numpy(G).cuda() for G, _ in data]
    Vs = [torch.from_numpy(V).cuda() for _, V in data]
    s = torch.cuda.Stream()
    cfgs = [TileConfig("pipeline"), TileConfig("one_wg", 64, 2), TileConfig("one_wg")]
    with xb.TileBatch(classes, *R, configs=cfgs, streams=3, stream=s) as tb:
        Is = [torch.empty((c, B, n), dtype=torch.float64, device="cuda") for (m, n, c, B) in classes]
        with torch.cuda.stream(s):
            tb.run(Gs, Vs, Is)
        s.synchronize()
        eager = [I.clone() for I in Is]
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            tb.run(Gs, Vs, Is)
        for rep in range(3):
            for I in Is:
                I.fill_(float("nan"))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            log(f"  replay {rep}")
            for k in range(len(classes)):
                assert torch.equal(Is[k], eager[k]), (rep, k)
            _ = torch.ones(1000, device="cuda").sum().item()        # eager work between replays
    out = [e.cpu().numpy() for e in eager]
    _check(classes, data, out)


def test_c4_workload_every_class_against_stored_oracle():
    """All 2048 crossbars of the heterogeneous tiles workload in one batch with the tuned
    configuration; the first crossbar of each of the 16 classes, all 256 vectors,
    against the stored oracle currents, and every crossbar's currents finite and
    non-negative (inputs >= 0)."""
    import torch

    import paper_2410_19993_amd as xb
    g = workloads.C4_GEOM
    r = (g["r_wl"], g["r_bl"], g["r_src"], g["r_sense"])
    tiles = workloads.c4()
    by_class = {}
    for t in tiles:
        by_class.setdefault((t.G.shape[0], t.G.shape[1], t.V.shape[0]), []).append(t)
    keys = sorted(by_class)
    classes = [(m, n, len(by_class[(m, n, B)]), B) for (m, n, B) in keys]
    Gs = [torch.from_numpy(np.stack([t.G for t in by_class[k]])).cuda() for k in keys]
    Vs = [torch.from_numpy(np.stack([t.V for t in by_class[k]])).cuda() for k in keys]
    gold = np.load(os.path.join(GOLDEN, "c4_class_currents.npz"))
    with xb.TileBatch(classes, *r) as tb:
        log(f"case c4 workload: {len(tiles)} crossbars, configs {[(c.method, c.block, c.split) for c in tb.configs]}")
        Is = tb.run(Gs, Vs)
        torch.cuda.synchronize()
    worst = 0.0
    for k, (m, n, B) in enumerate(keys):
        first = by_class[(m, n, B)][0]
        assert first.index == int(gold[f"t{m}x{n}"])
        I = Is[k].cpu().numpy()
        e = float(rel_err(I[0], gold[f"I{m}x{n}"]).max())
        worst = max(worst, e)
        log(f"  class {m}x{n}: first crossbar max rel err {e:.3e}")
        assert e <= TOL_FP64
        assert np.all(np.isfinite(I)) and I.min() >= 0.0
    log(f"  worst {worst:.3e}")


def test_tuning_cache_decides_the_configuration(tmp_path):
    import torch

    import paper_2410_19993_amd as xb
    from paper_2410_19993_amd import tiles as tl
    dev = tl.device_name()
    cache = {"format": 1, "devices": {dev: {"streams": 3, "classes": {
        "10x20x16": {"method": "one_wg", "block": 64, "split": 2},
        "10x90x16": {"method": "pipeline", "block": 0, "split": 1},
        "10x30x16": {"method": "one_wg", "block": 16, "split": 1}}}}}     # invalid: block < n
    path = tmp_path / "cache.json"
    path.write_text(json.dumps(cache))
    classes = [(10, 20, 2, 16), (10, 90, 2, 16), (10, 30, 2, 16), (10, 40, 2, 16)]
    with xb.TileBatch(classes, *R, cache_path=str(path)) as tb:
        assert tb.streams == 3
        assert tb.configs[0] == tl.TileConfig("one_wg", 64, 2) and tb.sources[0] == "cache"
        assert tb.configs[1] == tl.TileConfig("pipeline") and tb.sources[1] == "cache"
        assert tb.configs[2] == tl.default_config(10, 30) and tb.sources[2] == "default"
        assert tb.configs[3] == tl.default_config(10, 40) and tb.sources[3] == "default"
        data = [_class(*c, seed=700 + k) for k, c in enumerate(classes)]
        Is = tb.run([torch.from_numpy(G).cuda() for G, _ in data], [torch.from_numpy(V).cuda() for _, V in data])
        torch.cuda.synchronize()
        _check(classes, data, [I.cpu().numpy() for I in Is])
