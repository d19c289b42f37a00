"""Seeded synthetic crossbar workloads.

This module only draws random inputs; it holds none of the solver's
arithmetic, so both the CPU oracle and the GPU path can take their inputs
from it without sharing any part of the method.

The paper (Sec. III.A) generates random conductances and input voltages with
unstated distributions and 5-ohm parasitics.  The workloads below stand in
for those random crossbars with stated distributions:

* ``c1``: 16x16, G ~ U[1e-6, 1e-4] S, 1-ohm segments, 50-ohm source and
  sense resistors, 8 input vectors ~ U[0, 0.5] V.
* ``c2``: 128x128, G log-uniform on [1e-6, 1e-4] S, 2.5-ohm segments,
  50/50 ohm, 1024 input vectors ~ U[0, 0.5] V.
* ``c3``: 512x512, G log-uniform, segment resistance in {1, 2.5, 5} ohm
  (one G and V shared by the three), 50/50 ohm, 4096 input vectors.
* ``c4``: 2048 heterogeneous tiles (the partitioned crossbars of Sec. III.C at
  scale): m_t, n_t in {32, 64, 128, 256}, signed weights mapped to
  differential column pairs, 256 input vectors each, binarized or uniform.

All arrays are float64, drawn with ``numpy.random.default_rng(seed)`` (PCG64)
in the order listed in each function.  ``G`` is [m][n] (row = word line,
column = bit line), ``V`` is [B][m] (one input vector per row).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

G_MIN = 1e-6
G_MAX = 1e-4


@dataclass(frozen=True)
class Geometry:
    """Wire and terminal resistances of a crossbar, in ohms."""

    m: int
    n: int
    r_wl: float
    r_bl: float
    r_src: float = 50.0
    r_sense: float = 50.0


@dataclass
class Workload:
    name: str
    geom: Geometry
    G: np.ndarray          # [m][n] siemens
    V: np.ndarray          # [B][m] volts
    extra: dict = field(default_factory=dict)

    @property
    def B(self) -> int:
        return int(self.V.shape[0])


def log_uniform(rng: np.random.Generator, shape, lo=G_MIN, hi=G_MAX) -> np.ndarray:
    return np.exp(rng.uniform(np.log(lo), np.log(hi), shape))


def c1(seed: int = 1001) -> Workload:
    rng = np.random.default_rng(seed)
    G = rng.uniform(G_MIN, G_MAX, (16, 16))
    V = rng.uniform(0.0, 0.5, (8, 16))
    return Workload("c1_16x16_b8", Geometry(16, 16, 1.0, 1.0, 50.0, 50.0), G, V)


def c2(seed: int = 1002, batch: int = 1024) -> Workload:
    rng = np.random.default_rng(seed)
    G = log_uniform(rng, (128, 128))
    V = rng.uniform(0.0, 0.5, (1024, 128))[:batch]
    return Workload("c2_128x128_b1024", Geometry(128, 128, 2.5, 2.5, 50.0, 50.0), G, V)


C3_R = (1.0, 2.5, 5.0)


def c3(r: float = 2.5, seed: int = 1003, batch: int = 4096) -> Workload:
    """512x512 crossbar; the same G and V serve every segment resistance."""
    if r not in C3_R:
        raise ValueError(f"c3 segment resistance must be one of {C3_R}")
    rng = np.random.default_rng(seed)
    G = log_uniform(rng, (512, 512))
    V = rng.uniform(0.0, 0.5, (4096, 512))[:batch]
    return Workload(f"c3_512x512_b4096_r{r:g}", Geometry(512, 512, r, r, 50.0, 50.0), G, V,
                    extra={"subset": c3_subset()})


def c3_subset(k: int = 256) -> np.ndarray:
    """Sorted indices of the seeded 256-vector subset of the c3 batch."""
    return np.sort(np.random.default_rng(2003).choice(4096, k, replace=False))


def random_crossbar(m: int, n: int, B: int, seed: int, r_wl: float = 2.5,
                    r_bl: float | None = None, r_src: float = 50.0,
                    r_sense: float = 50.0, g_dist: str = "log") -> Workload:
    """Generic seeded crossbar used by the parity tests at other shapes."""
    rng = np.random.default_rng(seed)
    if g_dist == "log":
        G = log_uniform(rng, (m, n))
    else:
        G = rng.uniform(G_MIN, G_MAX, (m, n))
    V = rng.uniform(0.0, 0.5, (B, m))
    rb = r_wl if r_bl is None else r_bl
    return Workload(f"rand_{m}x{n}_b{B}_s{seed}", Geometry(m, n, r_wl, rb, r_src, r_sense), G, V)


C4_SIZES = (32, 64, 128, 256)


@dataclass
class Tile:
    index: int
    G: np.ndarray          # [m_t][n_t] siemens, columns (2k, 2k+1) = (G+, G-) of weight column k
    V: np.ndarray          # [256][m_t] volts


def c4(seed: int = 1004, tiles: int = 2048, max_n: int | None = None) -> list:
    """Heterogeneous tiles, drawn in this order for each tile t: m_t and n_t, each
    C4_SIZES[integers(4)]; W ~ N(0, 0.05) of shape m_t x (n_t / 2), clipped to
    +-0.15; G+ = G_MIN + (G_MAX - G_MIN) max(W, 0) / 0.15 and G- the same for -W,
    interleaved as columns (2k, 2k+1); V of shape 256 x m_t, in {0, 0.5} with
    probability 1/2 each for even t, U[0, 0.5] for odd t.  Wires: r = 2.5 ohm,
    50-ohm source and sense resistors (``C4_GEOM``).  Every tile's draws are
    made; with ``max_n`` only the tiles with n_t <= max_n are returned."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(tiles):
        m = C4_SIZES[int(rng.integers(4))]
        n = C4_SIZES[int(rng.integers(4))]
        W = np.clip(rng.normal(0.0, 0.05, (m, n // 2)), -0.15, 0.15)
        G = np.empty((m, n))
        G[:, 0::2] = G_MIN + (G_MAX - G_MIN) * np.maximum(W, 0.0) / 0.15
        G[:, 1::2] = G_MIN + (G_MAX - G_MIN) * np.maximum(-W, 0.0) / 0.15
        if t % 2 == 0:
            V = rng.integers(0, 2, (256, m)).astype(np.float64) * 0.5
        else:
            V = rng.uniform(0.0, 0.5, (256, m))
        if max_n is None or n <= max_n:
            out.append(Tile(t, G, V))
    return out


C4_GEOM = dict(r_wl=2.5, r_bl=2.5, r_src=50.0, r_sense=50.0)
