"""Crossbar netlist: the circuit of the paper's Sec. II.A, as a plain resistor list.

Circuit (paper Fig. 1 and the notation list of Sec. II.A; readings of the
garbled passages are listed in the module ``oracle`` docstring):

* m word lines (rows, index i) and n bit lines (columns, index j), 0-based
  here, 1-based in the paper.
* Two voltage nodes per crosspoint: the word-line side WL(i,j) and the
  bit-line side BL(i,j) of device D(i,j).  Node numbering follows the
  interleaved unknown order of Sec. II.B: WL(i,j) -> 2(i*n+j),
  BL(i,j) -> 2(i*n+j)+1.
* Resistors (3*m*n in total, as Sec. II.A counts):
    - source link: ideal source V_i -> WL(i,0), conductance g_src
      (Eq. 5 places a word-line segment there; the paper's model is
      r_src = r_wl);
    - word-line segments WL(i,j) - WL(i,j+1), conductance g_wl;
    - devices WL(i,j) - BL(i,j), conductance G[i][j];
    - bit-line segments BL(i,j) - BL(i+1,j), conductance g_bl;
    - sense terminations BL(m-1,j) - ground, conductance g_sense (the
      paper's model is r_sense = r_bl).
* Output j is the current through the termination of bit line j
  (Sec. II, first paragraph), positive into the sense resistor.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

GROUND = -1


@dataclass
class Netlist:
    m: int
    n: int
    # two-terminal resistors between nodes (b may be GROUND)
    a: np.ndarray      # int64 [R]
    b: np.ndarray      # int64 [R]
    g: np.ndarray      # float64 [R], siemens
    kind: np.ndarray   # int8 [R]: 1 WL segment, 2 device, 3 BL segment, 4 sense
    # resistors from an ideal source V_i to a node
    src_node: np.ndarray  # int64 [m]
    src_row: np.ndarray   # int64 [m], which input V_i drives it
    src_g: np.ndarray     # float64 [m]

    @property
    def num_nodes(self) -> int:
        return 2 * self.m * self.n

    @property
    def num_resistors(self) -> int:
        return int(self.g.size + self.src_g.size)


KIND_WL, KIND_DEVICE, KIND_BL, KIND_SENSE = 1, 2, 3, 4


def wl_node(i, j, n):
    return 2 * (i * n + j)


def bl_node(i, j, n):
    return 2 * (i * n + j) + 1


def build_netlist(G: np.ndarray, r_wl: float, r_bl: float, r_src: float,
                  r_sense: float) -> Netlist:
    G = np.asarray(G, dtype=np.float64)
    m, n = G.shape
    g_wl, g_bl, g_src, g_sense = 1.0 / r_wl, 1.0 / r_bl, 1.0 / r_src, 1.0 / r_sense
    A, Bn, Gv, K = [], [], [], []

    ii, jj = np.meshgrid(np.arange(m), np.arange(n - 1), indexing="ij")
    A.append(wl_node(ii, jj, n).ravel()); Bn.append(wl_node(ii, jj + 1, n).ravel())
    Gv.append(np.full(ii.size, g_wl)); K.append(np.full(ii.size, KIND_WL))

    ii, jj = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    A.append(wl_node(ii, jj, n).ravel()); Bn.append(bl_node(ii, jj, n).ravel())
    Gv.append(G.ravel().copy()); K.append(np.full(ii.size, KIND_DEVICE))

    ii, jj = np.meshgrid(np.arange(m - 1), np.arange(n), indexing="ij")
    A.append(bl_node(ii, jj, n).ravel()); Bn.append(bl_node(ii + 1, jj, n).ravel())
    Gv.append(np.full(ii.size, g_bl)); K.append(np.full(ii.size, KIND_BL))

    jj = np.arange(n)
    A.append(bl_node(m - 1, jj, n)); Bn.append(np.full(n, GROUND))
    Gv.append(np.full(n, g_sense)); K.append(np.full(n, KIND_SENSE))

    rows = np.arange(m)
    return Netlist(
        m=m, n=n,
        a=np.concatenate(A).astype(np.int64), b=np.concatenate(Bn).astype(np.int64),
        g=np.concatenate(Gv).astype(np.float64), kind=np.concatenate(K).astype(np.int8),
        src_node=wl_node(rows, 0, n).astype(np.int64), src_row=rows.astype(np.int64),
        src_g=np.full(m, g_src),
    )


def sense_nodes(m: int, n: int) -> np.ndarray:
    return bl_node(m - 1, np.arange(n), n)
