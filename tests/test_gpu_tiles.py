"""GPU parity of the batched small-crossbar solver (xbar_tiles_currents).

Each crossbar of the batch is checked against the oracle's currents for that
crossbar alone (per-vector relative error <= 1e-10, the float64 tolerance), over
shapes that take each padded block size (16, 32, 64), ragged n, m = 1, B up to
256, and batches of several crossbars.
"""
import numpy as np
import pytest

import oracle
from tests.gpu_util import TOL_FP64, log, rel_err

pytestmark = pytest.mark.gpu


def _inputs(T, m, n, B, seed, binary=False):
    rng = np.random.default_rng(seed)
    G = np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), (T, m, n)))
    V = (rng.integers(0, 2, (T, B, m)) * 0.5) if binary else rng.uniform(0.0, 0.5, (T, B, m))
    return G, V


def _gpu(G, V, r):
    import torch

    import paper_2410_19993_amd as xb
    I = xb.tiles_currents(torch.from_numpy(G).cuda(), torch.from_numpy(V).cuda(), *r)
    torch.cuda.synchronize()
    return I.cpu().numpy()


@pytest.mark.parametrize("T,m,n,B,seed", [
    (1, 1, 1, 1, 71), (2, 1, 5, 3, 72), (3, 2, 3, 4, 73), (4, 7, 16, 17, 74), (2, 9, 20, 5, 75),
    (3, 33, 32, 64, 76), (2, 12, 64, 256, 77), (5, 64, 33, 8, 78), (2, 130, 48, 9, 79),
    (300, 4, 8, 2, 80)])
def test_tiles_match_oracle(T, m, n, B, seed):
    r = (2.5, 3.0, 40.0, 60.0)
    log(f"case tiles T={T} m={m} n={n} B={B}")
    G, V = _inputs(T, m, n, B, seed, binary=seed % 2 == 0)
    I = _gpu(G, V, r)
    assert I.shape == (T, B, n) and np.all(np.isfinite(I))
    worst = 0.0
    for t in range(T):
        ref = oracle.solve(G[t], V[t], *r).currents
        worst = max(worst, float(rel_err(I[t], ref).max()))
    log(f"  max current rel err {worst:.3e}")
    assert worst <= TOL_FP64


def test_tiles_bad_conductance_only_spoils_its_tile():
    r = (2.5, 2.5, 50.0, 50.0)
    G, V = _inputs(3, 6, 10, 4, 81)
    G[1, 2, 3] = -1e-5
    log("case tiles with a negative conductance in tile 1")
    I = _gpu(G, V, r)
    assert np.all(np.isnan(I[1]))
    for t in (0, 2):
        assert rel_err(I[t], oracle.solve(G[t], V[t], *r).currents).max() <= TOL_FP64


def test_tiles_agree_with_the_plan_path():
    """The one-launch tile solver and the plan-based solver on the same crossbar."""
    from tests.gpu_util import gpu_solve
    import workloads
    r = (1.5, 3.0, 40.0, 60.0)
    G, V = _inputs(1, 40, 64, 32, 82)
    log("case tiles vs plan path m=40 n=64 B=32")
    I = _gpu(G, V, r)[0]
    Ip, _, (st, _) = gpu_solve(G[0], V[0], workloads.Geometry(40, 64, *r), "fp64", node_voltages=False)
    assert st == 0
    assert rel_err(I, Ip).max() <= 1e-11


def test_c4_tiles_in_bench_configuration():
    """The heterogeneous tiles workload as the benchmark runs it: every (m_t, n_t) class with
    n_t <= 64 in one launch; the first two tiles of each class against the oracle (all 256
    input vectors for m_t <= 64, the first 32 otherwise)."""
    import torch

    import paper_2410_19993_amd as xb
    import workloads
    g = workloads.C4_GEOM
    r = (g["r_wl"], g["r_bl"], g["r_src"], g["r_sense"])
    classes = {}
    for t in workloads.c4(max_n=64):
        classes.setdefault(t.G.shape, []).append(t)
    worst = 0.0
    for (m, n), ts in sorted(classes.items()):
        log(f"case c4 class m={m} n={n}: {len(ts)} tiles")
        Gs = torch.from_numpy(np.stack([t.G for t in ts])).cuda()
        Vs = torch.from_numpy(np.stack([t.V for t in ts])).cuda()
        I = xb.tiles_currents(Gs, Vs, *r).cpu().numpy()
        assert np.all(np.isfinite(I))
        for k in range(2):
            rows = slice(None) if m <= 64 else slice(0, 32)
            ref = oracle.solve(ts[k].G, ts[k].V[rows], *r).currents
            worst = max(worst, float(rel_err(I[k][rows], ref).max()))
    log(f"  max current rel err {worst:.3e}")
    assert worst <= TOL_FP64


def test_tiles_in_a_captured_graph():
    """Launches of several classes on forked streams, captured into one HIP graph and replayed
    three times with eager work between the replays: every replay gives the eager bits."""
    import torch

    import paper_2410_19993_amd as xb
    r = (2.5, 2.5, 50.0, 50.0)
    shapes = [(3, 20, 16, 8), (2, 37, 40, 4), (4, 12, 64, 32)]
    data = []
    for k, (T, m, n, B) in enumerate(shapes):
        G, V = _inputs(T, m, n, B, 90 + k)
        data.append((torch.from_numpy(G).cuda(), torch.from_numpy(V).cuda(),
                     torch.empty((T, B, n), dtype=torch.float64, device="cuda")))
    eager = [xb.tiles_currents(Gd, Vd, *r).cpu().numpy() for Gd, Vd, _ in data]
    log("case tiles graph capture: 3 classes on 2 forked streams")
    side = [torch.cuda.Stream() for _ in range(2)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        main = torch.cuda.current_stream()
        fork = torch.cuda.Event()
        fork.record(main)
        for k, (Gd, Vd, Id) in enumerate(data):
            st = side[k % 2]
            st.wait_event(fork)
            xb.tiles_currents(Gd, Vd, *r, out=Id, stream=st)
        for st in side:
            done = torch.cuda.Event()
            done.record(st)
            main.wait_event(done)
    for rep in range(3):
        for _, _, Id in data:
            Id.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, (_, _, Id) in enumerate(data):
            assert np.array_equal(Id.cpu().numpy(), eager[k]), f"replay {rep}, class {k}"
        _ = torch.ones(1000, device="cuda").sum().item()        # eager work between replays
