"""Plain CPU oracle for the memristive-crossbar nodal solve (TEST INFRASTRUCTURE).

This package is the slow, obviously correct reference that the GPU library
is checked against.  It is test infrastructure only: the GPU library never
imports, links or calls it, and it shares no code, headers, tables or
constants with the GPU path.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark use it.

What it computes (paper Sec. II): the node voltages v of the nodal equations
G v = I of an m x n crossbar with word-line and bit-line wire resistance
(Eqs. 1-7), by banded LU decomposition without row exchanges followed by
forward and back substitution (Sec. II.C), and the bit-line termination
currents.  Arithmetic is float64; the KCL residual used for refinement is
accumulated in long double.

Readings taken where the paper is garbled or silent:

* The word-line source is reached through a resistor r_src (Eq. 5 shows a
  word-line segment there; the paper's own model is r_src = r_wl).
* Bit lines terminate at the last row (i = m) through r_sense to 0 V; the
  output current is positive into the sense resistor (the paper's model is
  r_sense = r_bl).
* Eq. 6's coupling term "s(-G_D(i,j))" is -G_ij; Eq. 7 holds for every
  column j.
* The nonzero count printed as a product in Sec. II is read as the sum
  m(4n-2) + n(4m-2) = 8mn - 2m - 2n.
* The injection vector has m nonzeros (one per word line), not "all but n".
* Devices are linear conductances; precision is float64.

Parity status: every function here is pinned by the CPU tests
(tests/test_oracle_*.py) against closed forms, exact rational solves,
LAPACK solves, circuit invariants and the paper's printed stamps.
"""
from .netlist import Netlist, build_netlist, sense_nodes, wl_node, bl_node, GROUND  # noqa: F401
from .solve import (OracleResult, assemble_band, band_to_dense, half_bandwidth,  # noqa: F401
                    injections, kcl_residual_ld, lu_factor, lu_solve, solve, solve_workload)
from . import diagnostics  # noqa: F401
