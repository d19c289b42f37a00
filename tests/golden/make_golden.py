"""Write the stored expected values used by the GPU parity tests.

Every value written here comes from the CPU oracle (``oracle/``) run on the
seeded workloads of ``workloads/``; nothing is read from the GPU library.

    python tests/golden/make_golden.py c2          # 128x128, all 1024 input vectors
    python tests/golden/make_golden.py c3          # 512x512, seeded 256-vector subset, r in {1, 2.5, 5}
    python tests/golden/make_golden.py c4          # heterogeneous tiles: the first tile of each of
                                                   # the 16 (m_t, n_t) classes, all 256 vectors
    python tests/golden/make_golden.py rev         # a 32 x 700 crossbar (more columns than rows)

Outputs (float64 .npy/.npz next to this file):

* ``c2_currents.npy``            [1024][128]
* ``c3_r{r}_currents.npy``       [256][512]   rows = workloads.c3_subset()
* ``c3_r{r}_nodes.npz``          node voltages of the first 8 subset vectors at
                                 4096 seeded node indices (``idx``, ``v``)
* ``c4_class_currents.npz``      per (m_t, n_t) class: the index of the class's first tile
                                 in workloads.c4() (``t{m}x{n}``) and its currents
                                 [256][n_t] (``I{m}x{n}``)
* ``rev_32x700_b3.npz``           a 32 x 700 crossbar (workloads.random_crossbar(32, 700, 3, 41),
                                 2.5-ohm segments): currents [3][700] (``I``) and node
                                 voltages [3][44800] (``v``)
* ``manifest.json``              oracle diagnostics and timings per file
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402


def _manifest_update(key, info):
    path = os.path.join(HERE, "manifest.json")
    man = json.load(open(path)) if os.path.exists(path) else {}
    man[key] = info
    with open(path, "w") as f:
        json.dump(man, f, indent=1, sort_keys=True)


def make_c2():
    wl = workloads.c2()
    t = time.time()
    res = oracle.solve_workload(wl)
    np.save(os.path.join(HERE, "c2_currents.npy"), res.currents)
    _manifest_update("c2_currents.npy", {
        "workload": wl.name, "rows": "all", "refine": 2, "seconds": time.time() - t,
        "residual_inf_A": res.residual_inf, "corrections": res.correction_norms,
        "min_pivot": res.min_pivot})


def make_c3(rs=workloads.C3_R):
    sub = workloads.c3_subset()
    for r in rs:
        wl = workloads.c3(r=r)
        t = time.time()
        res = oracle.solve_workload(wl, rows=sub)
        tag = f"c3_r{r:g}"
        np.save(os.path.join(HERE, f"{tag}_currents.npy"), res.currents)
        idx = np.sort(np.random.default_rng(4242).choice(res.node_v.shape[1], 4096, replace=False))
        np.savez(os.path.join(HERE, f"{tag}_nodes.npz"), idx=idx, v=res.node_v[:8, idx])
        _manifest_update(f"{tag}_currents.npy", {
            "workload": wl.name, "rows": "workloads.c3_subset()", "refine": 2,
            "seconds": time.time() - t, "residual_inf_A": res.residual_inf,
            "corrections": res.correction_norms, "min_pivot": res.min_pivot})
        print(tag, "done", time.time() - t, flush=True)
        del res


def make_c4():
    g = workloads.C4_GEOM
    r = (g["r_wl"], g["r_bl"], g["r_src"], g["r_sense"])
    first = {}
    for t in workloads.c4():
        first.setdefault(t.G.shape, t)
    out, info = {}, {}
    for (m, n), t in sorted(first.items()):
        t0 = time.time()
        res = oracle.solve(t.G, t.V, *r)
        out[f"t{m}x{n}"] = np.array(t.index)
        out[f"I{m}x{n}"] = res.currents
        info[f"{m}x{n}"] = {"tile": t.index, "seconds": time.time() - t0, "residual_inf_A": res.residual_inf,
                           "min_pivot": res.min_pivot}
        print(f"c4 {m}x{n} tile {t.index}: {time.time() - t0:.1f} s", flush=True)
    np.savez(os.path.join(HERE, "c4_class_currents.npz"), **out)
    _manifest_update("c4_class_currents.npz", {"workload": "c4 (seed 1004), first tile of each class",
                                               "vectors": 256, "refine": 2, "classes": info})


def make_rev():
    wl = workloads.random_crossbar(32, 700, 3, 41)
    t = time.time()
    res = oracle.solve_workload(wl)
    np.savez(os.path.join(HERE, "rev_32x700_b3.npz"), I=res.currents, v=res.node_v)
    _manifest_update("rev_32x700_b3.npz", {
        "workload": wl.name, "refine": 2, "seconds": time.time() - t, "residual_inf_A": res.residual_inf,
        "corrections": res.correction_norms, "min_pivot": res.min_pivot})


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2", "c3", "c4", "rev"]
    if "c2" in which:
        make_c2()
    if "c3" in which:
        rs = [float(x) for x in which[which.index("c3") + 1:] if x[0].isdigit()] or list(workloads.C3_R)
        make_c3(rs)
    if "c4" in which:
        make_c4()
    if "rev" in which:
        make_rev()
