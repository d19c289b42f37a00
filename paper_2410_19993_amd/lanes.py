"""Many crossbars of mixed shapes through concurrent plans ("lanes").

The paper splits a large array into smaller crossbars that are solved one by one
(Sec. III.C).  The plan path solves one crossbar per call, and for crossbars of
128 to 256 lines its launches are small (a factor chain of m/2 rows on
(n_p/32)^2 workgroups), so one crossbar at a time leaves most of the GPU idle.
A PlanLanes object runs `lanes` host threads, each with a HIP stream of its own
and one plan per (m, n) shape, that take the crossbars in order of decreasing
size until none is left.  Plans share no state, and each plan waits only on its
own stream when its factorization reads the schedule state back, so the lanes'
kernels overlap on the device.  A plan clears its device-side error flags at
every assembly, so each lane reads its plan's status after every crossbar it
solves; `status` keeps one code per crossbar.  All arithmetic runs in the
library's kernels.
"""
from __future__ import annotations

import threading

from . import Plan, XbarError, _check_tensor, _lib


def _torch():
    import torch
    return torch


class PlanLanes:
    """Output currents of many crossbars of any shapes, `lanes` plans at a time.

    r_wl, r_bl, r_src, r_sense: the geometry's resistances (ohm), shared by every
    crossbar.  Plans are created on first use of a shape in a lane and kept until
    close(), so repeated calls reuse them."""

    def __init__(self, r_wl: float, r_bl: float, r_src: float = 50.0, r_sense: float = 50.0,
                 lanes: int = 2, max_batch: int = 256, precision: str = "fp64"):
        torch = _torch()
        if lanes < 1:
            raise ValueError("lanes must be >= 1")
        self.r = (float(r_wl), float(r_bl), float(r_src), float(r_sense))
        self.max_batch = int(max_batch)
        self.precision = precision
        self._lanes = [{"stream": torch.cuda.Stream(), "plans": {}} for _ in range(int(lanes))]

    @property
    def lanes(self) -> int:
        return len(self._lanes)

    def _plan(self, lane, m, n):
        p = lane["plans"].get((m, n))
        if p is None:
            # each crossbar of a lane is a new conductance map on the same plan: the factor
            # reads its schedule back and falls back to Gauss-Jordan if it must
            p = Plan(m, n, *self.r, precision=self.precision, max_batch=self.max_batch, stream=lane["stream"],
                     factor_method="checked")
            lane["plans"][(m, n)] = p
        return p

    def currents(self, Gs, Vs, outs=None):
        """Gs[k] [m_k][n_k], Vs[k] [B_k][m_k] (B_k <= max_batch) float64 CUDA/HIP tensors
        written on the current stream; returns outs[k] [B_k][n_k], ready on the current
        stream.  Raises the first error any lane met, after every lane has stopped.
        Device-side failures of single crossbars (a conductance that is not finite and
        positive, a pivot that is not) do not raise here: `status[k]` holds each
        crossbar's code (XBAR_OK = 0) and check() raises for them."""
        torch = _torch()
        T = len(Gs)
        if len(Vs) != T or (outs is not None and len(outs) != T):
            raise ValueError("Gs, Vs and outs must have the same length")
        shapes = []
        for k in range(T):
            m, n = (int(x) for x in Gs[k].shape)
            B = int(Vs[k].shape[0])
            if not 1 <= B <= self.max_batch:
                raise ValueError(f"crossbar {k}: batch {B} outside [1, {self.max_batch}]")
            _check_tensor(f"Gs[{k}]", Gs[k], (m, n))
            _check_tensor(f"Vs[{k}]", Vs[k], (B, m))
            shapes.append((m, n, B))
        if outs is None:
            outs = [torch.empty((B, n), dtype=torch.float64, device="cuda") for m, n, B in shapes]
        for k, (m, n, B) in enumerate(shapes):
            _check_tensor(f"outs[{k}]", outs[k], (B, n))
        if T == 0:
            return outs

        cur = torch.cuda.current_stream()
        ready = torch.cuda.Event()
        ready.record(cur)
        for lane in self._lanes:
            lane["stream"].wait_event(ready)
        order = iter(sorted(range(T), key=lambda k: (-shapes[k][0] * shapes[k][1], k)))
        lock = threading.Lock()
        errors = []
        self.status = [None] * T

        def work(lane):
            try:
                while True:
                    with lock:
                        if errors:
                            return
                        k = next(order, None)
                    if k is None:
                        return
                    m, n, _ = shapes[k]
                    p = self._plan(lane, m, n)
                    p.assemble(Gs[k])
                    p.factor()
                    p.solve_batch(Vs[k], None)
                    p.currents(outs[k])
                    self.status[k] = p.info()[0]        # before the next assembly clears it
            except BaseException as e:          # handed to the caller below
                with lock:
                    errors.append(e)

        threads = [threading.Thread(target=work, args=(lane,)) for lane in self._lanes[1:]]
        for t in threads:
            t.start()
        work(self._lanes[0])
        for t in threads:
            t.join()
        for lane in self._lanes:
            done = torch.cuda.Event()
            done.record(lane["stream"])
            cur.wait_event(done)
        if errors:
            raise errors[0]
        return outs

    def failed(self) -> list:
        """Indices of the crossbars of the last currents() call whose solve failed on
        the device."""
        return [k for k, st in enumerate(getattr(self, "status", [])) if st is not None and st != _lib.XBAR_OK]

    def check(self) -> None:
        """Raise XbarError if any crossbar of the last currents() call failed on the
        device; the message names the crossbars."""
        bad = self.failed()
        if bad:
            st = self.status[bad[0]]
            raise XbarError(f"PlanLanes crossbars {bad[:8]}{' ...' if len(bad) > 8 else ''}", st)

    def close(self) -> None:
        for lane in self._lanes:
            for p in lane["plans"].values():
                p.close()
            lane["plans"].clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
