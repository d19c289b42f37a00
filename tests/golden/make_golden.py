"""Write the stored expected values used by the GPU parity tests.

Every value written here comes from the CPU oracle (``oracle/``) run on the
seeded workloads of ``workloads/``; nothing is read from the GPU library.

    python tests/golden/make_golden.py c2          # 128x128, all 1024 input vectors
    python tests/golden/make_golden.py c3          # 512x512, seeded 256-vector subset, r in {1, 2.5, 5}

Outputs (float64 .npy/.npz next to this file):

* ``c2_currents.npy``            [1024][128]
* ``c3_r{r}_currents.npy``       [256][512]   rows = workloads.c3_subset()
* ``c3_r{r}_nodes.npz``          node voltages of the first 8 subset vectors at
                                 4096 seeded node indices (``idx``, ``v``)
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


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2", "c3"]
    if "c2" in which:
        make_c2()
    if "c3" in which:
        rs = [float(x) for x in which[which.index("c3") + 1:]] or list(workloads.C3_R)
        make_c3(rs)
