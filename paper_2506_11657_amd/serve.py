"""Request loop for forward and adjoint TEM solves on one GPU.

Requests (a grid, a conductivity model, 1-4 loops, receivers; forward or
adjoint) arrive over time.  A scheduler admits a request when its device
footprint fits in the HBM budget and a slot is free; every admitted request
runs on its own library context in a worker thread (the C calls release the
GIL), and a request that arrives while others run is admitted as soon as
memory and a slot free up.  All requests share one pole/residue set (the
channels are the same).

With batched=True (continuous batching) every request's context is attached
to one solve engine of the library: the multi-shift solves of all admitted
requests (their loop sources and adjoint receiver rows) advance together in
batched launches, one seed stencil and one seed update launch per iteration
for all of them and one shift-block and block-update launch per 64
iterations for all their poles, replayed as HIP graphs; a request joins the
batch at the next 64-iteration boundary after it is admitted and leaves it
when its shifts have converged.  The library sends only the solves of grids
too small to fill the device to the engine; larger ones (64^3 and up on
MI355X) run their own launches, as they do without an engine.  Without it,
each request replays its own solver graphs on its own streams and the
requests overlap on the device.

Each request's arithmetic is independent of the others (its own buffers,
fixed-order reductions whose order does not depend on the batch), so its
result is bitwise the same alone or in any mix.
"""
from __future__ import annotations

import os
import sys
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import tem


def footprint_bytes(nx, ny, nz, J, n_src, kind, block=64, n_rx=1, concurrent=4):
    """Device bytes a request needs (the library's allocations for it):
    operator arrays; one solver workspace per concurrent multi-shift solve
    (residual ring of `block` vectors, 3x that with overlapped updates, the
    seed's p and q in two slots each, right-hand side, per-shift p_j, 4 MiB of
    partial sums and 2 MiB of solver state); the solutions y_j of every concurrent source (of every source for the
    adjoint, which keeps them); the residual and contraction scratch; for the
    adjoint, its right-hand sides per concurrent receiver row and its COCG
    vectors."""
    n3 = 3 * (nx + 1) * (ny + 1) * (nz + 1)
    vec = 16 * n3 * J                      # J complex node-padded vectors
    ops = 8 * n3 * 3 + 8 * nx * ny * nz
    conc = min(n_src, concurrent)
    slots = conc
    if kind == "adjoint":
        slots = max(slots, min(n_rx, concurrent))
    ring = 3 * block if os.environ.get("TEM_OVERLAP") == "1" else block   # 3 blocks with overlapped updates
    slot = 8 * n3 * (ring + 6) + vec + (6 << 20)
    keep = vec * (n_src if kind == "adjoint" else conc)
    scratch = vec + 24 * n3
    adj = 0
    if kind == "adjoint":
        adj = vec * (min(n_rx, concurrent) + 5) + 8 * n3
    return ops + slots * slot + keep + scratch + adj


@dataclass
class Request:
    rid: int
    kind: str                    # "forward" or "adjoint"
    workload: object             # tem_workloads.Workload
    arrival: float = 0.0         # seconds after the trace start
    d_obs: np.ndarray = None     # adjoint: observed data (n_src, T, n_rx)
    footprint: int = 0
    # results
    admitted: float = None
    finished: float = None
    data: np.ndarray = None
    grad: np.ndarray = None
    stats: dict = field(default_factory=dict)
    error: str = None
    precision: int = 0           # 1: FP32 search directions + FP64 refinement (not batched)

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


class Server:
    def __init__(self, xi, c, device=0, hbm_budget=64 << 30, max_active=4, rtol=0.0, verbose=False,
                 batched=False, max_jobs=0):
        self.verbose = verbose
        self.engine = tem.Engine(device, max_jobs) if batched else None
        self.xi, self.c = np.asarray(xi), np.asarray(c)
        self.device = device
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.rtol = rtol
        self._lock = threading.Condition()
        self._used = 0
        self._active = 0
        self._threads = []

    def _run(self, req: Request, t0: float):
        wl = req.workload
        ctx = None
        try:
            ctx = tem.Context(wl.hx, wl.hy, wl.hz, wl.k_s, device=self.device)
            if self.engine is not None:
                ctx.attach(self.engine)
            ctx.set_conductivity(wl.sigma)
            keep = req.kind == "adjoint"
            data, st = ctx.forward(wl.loops, wl.receivers, self.xi, self.c, keep_solutions=keep,
                                   rtol=self.rtol if req.precision == 0 else 0.0, precision=req.precision)
            req.data = data
            req.stats["forward"] = {"iterations": st["iterations"], "unknown_updates": st["unknown_updates"]}
            if keep:
                w = data - req.d_obs
                grad, sa = ctx.adjoint(w)
                req.grad = grad
                req.stats["adjoint"] = {"iterations": sa["iterations"], "unknown_updates": sa["unknown_updates"]}
        except Exception as e:  # reported per request; the loop keeps serving
            req.error = repr(e)
        finally:
            if ctx is not None:
                ctx.close()
            req.finished = time.perf_counter() - t0
            if self.verbose:
                wl = req.workload
                print("request %d (%s, %dx%dx%d, %d loops) done at %.2f s, latency %.2f s%s"
                      % (req.rid, req.kind, len(wl.hx), len(wl.hy), len(wl.hz), len(wl.loops), req.finished,
                         req.latency, "" if req.error is None else " ERROR " + req.error),
                      file=sys.stderr, flush=True)
            with self._lock:
                self._used -= req.footprint
                self._active -= 1
                self._lock.notify_all()

    def run(self, requests, realtime=True):
        """Serve the requests in arrival order; with realtime, a request is not
        admitted before its arrival time.  Returns the requests with results
        and timestamps (seconds from the start)."""
        J = len(self.xi)
        for r in requests:
            wl = r.workload
            r.footprint = footprint_bytes(len(wl.hx), len(wl.hy), len(wl.hz), J, len(wl.loops), r.kind,
                                          n_rx=len(wl.receivers))
            if r.footprint > self.budget:
                r.error = "TEM_ENOMEM: request footprint %d exceeds the budget %d" % (r.footprint, self.budget)
        t0 = time.perf_counter()
        for r in sorted(requests, key=lambda q: q.arrival):
            if r.error:
                r.finished = r.arrival
                continue
            if realtime:
                wait = r.arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
            with self._lock:
                while self._active >= self.max_active or self._used + r.footprint > self.budget:
                    self._lock.wait()
                self._active += 1
                self._used += r.footprint
            r.admitted = time.perf_counter() - t0
            th = threading.Thread(target=self._run, args=(r, t0), daemon=True)
            th.start()
            self._threads.append(th)
        for th in self._threads:
            th.join()
        self._threads = []
        return requests

    def close(self):
        if self.engine is not None:
            self.engine.close()
            self.engine = None


def summarize(requests, wall):
    done = [r for r in requests if r.error is None and r.finished is not None]
    lat = np.array([r.latency for r in done]) if done else np.zeros(1)
    upd = sum(r.stats.get("forward", {}).get("unknown_updates", 0.0) +
              r.stats.get("adjoint", {}).get("unknown_updates", 0.0) for r in done)
    return {"completed": len(done), "failed": len(requests) - len(done),
            "models_per_s": len(done) / wall if wall > 0 else 0.0,
            "unknown_updates_per_s": upd / wall if wall > 0 else 0.0,
            "p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
            "makespan_s": wall,
            # per request: (arrival, admitted, finished) in seconds from the start
            "requests": [(r.rid, r.kind, len(r.workload.hx), len(r.workload.loops), r.arrival, r.admitted, r.finished)
                         for r in requests]}
