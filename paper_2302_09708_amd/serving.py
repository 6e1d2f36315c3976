"""Continuous-batching request loop for CheFSI solves on one GPU.

Requests (a Hamiltonian, a block width Ns, a degree and an iteration count)
arrive over time and queue in arrival order.  When a slot is free, the request at
the head of the queue is opened: its potentials and projectors are uploaded (its
library handle is created) and its exact device footprint becomes known (the
orbital block X, the library workspace for its Ns, and the handle's own arrays).
It is admitted, first come first served, as soon as its footprint fits in what
the admitted requests leave of the HBM budget; every admitted request runs its
whole solve on its own HIP stream from its own host thread, so solves of
different sizes overlap on the device.  Only the head of the queue holds device
memory while it waits, so the device holds at most the budget plus the arrays of
one waiting handle.  Latency is completion minus arrival.

The scheduling (``Scheduler``) is independent of the GPU: it calls an
``open(request) -> (state, footprint)`` and a ``run(state) -> output`` supplied
by the caller.  ``gpu_ops`` supplies the library-backed pair.
"""
from __future__ import annotations

import dataclasses
import math
import threading
import time
from typing import Any, Callable, Dict, List, Optional, Tuple

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    prob: Any                 # inputs.Problem
    ns: int
    degree: int
    n_iter: int
    x_seed: int
    arrival: float            # seconds after the start of the stream
    x0: Optional[np.ndarray] = None  # (ns, Nd) starting block; None: seeded N(0,1) drawn on the device


@dataclasses.dataclass
class Result:
    rid: int
    output: Any
    arrival: float
    admitted: float
    finished: float
    footprint: int
    slot: int
    error: Optional[str] = None   # set (and output None) when the solve failed

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of n requests from a Poisson process of the given rate (1/s)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def nearest_rank(values, p: float) -> float:
    """p-th percentile by the nearest-rank rule (p in (0, 100])."""
    v = np.sort(np.asarray(values, dtype=np.float64))
    if v.size == 0:
        raise ValueError("no values")
    k = max(1, int(math.ceil(p / 100.0 * v.size)))
    return float(v[k - 1])


def summarize(results: List[Result]) -> Dict[str, float]:
    lat = [r.latency for r in results]
    failed = sum(1 for r in results if r.error is not None)
    t_first = min(r.arrival for r in results)
    t_last = max(r.finished for r in results)
    return {"requests": len(results), "p50_s": nearest_rank(lat, 50), "p99_s": nearest_rank(lat, 99),
            "mean_s": float(np.mean(lat)), "makespan_s": t_last - t_first,
            "solves_per_s": (len(results) - failed) / (t_last - t_first), "failed": failed}


class AdmissionError(RuntimeError):
    pass


class Scheduler:
    """First-come-first-served admission by free slot and HBM footprint.

    open_fn(request) -> (state, footprint_bytes) runs on the scheduling thread when the
    request is at the head of the queue and a slot is free (so at most one opened request
    waits for room); run_fn(state, slot) -> output runs on the slot's worker thread;
    close_fn(state) releases what open_fn acquired.  A request whose footprint
    exceeds the whole budget is refused with AdmissionError.  With fail_fast the first
    exception of a solve stops the loop and is raised; otherwise the request's Result
    carries the error and the loop goes on."""

    def __init__(self, budget_bytes: int, slots: int, open_fn: Callable, run_fn: Callable,
                 close_fn: Optional[Callable] = None, clock=time.perf_counter, fail_fast: bool = True):
        if slots < 1 or budget_bytes <= 0:
            raise ValueError("need at least one slot and a positive budget")
        self.budget = int(budget_bytes)
        self.slots = slots
        self.open_fn, self.run_fn, self.close_fn = open_fn, run_fn, close_fn
        self.clock = clock
        self.fail_fast = fail_fast
        self.peak_bytes = 0
        self.peak_active = 0

    def run(self, requests: List[Request]) -> List[Result]:
        order = sorted(requests, key=lambda r: (r.arrival, r.rid))
        cv = threading.Condition()
        free_slots = list(range(self.slots))
        used = 0
        results: List[Result] = []
        errors: List[BaseException] = []
        arrived: List[Request] = []  # arrived, not opened yet (arrival order)
        head: Optional[Tuple[Request, Any, int]] = None  # opened, waiting for room
        workers: List[threading.Thread] = []
        t0 = self.clock()

        def worker(req: Request, state, fp: int, slot: int, t_arr: float, t_adm: float):
            nonlocal used
            try:
                out = self.run_fn(state, slot)
                t_end = self.clock() - t0
                res = Result(req.rid, out, t_arr, t_adm, t_end, fp, slot)
            except BaseException as e:
                if self.fail_fast:  # surfaced to the caller after the drain
                    res = None
                    errors.append(e)
                else:
                    res = Result(req.rid, None, t_arr, t_adm, self.clock() - t0, fp, slot, error=repr(e))
            finally:
                if self.close_fn is not None:
                    try:
                        self.close_fn(state)
                    except BaseException as e:
                        errors.append(e)
            with cv:
                used -= fp
                free_slots.append(slot)
                if res is not None:
                    results.append(res)
                cv.notify_all()

        nxt = 0
        try:
            while True:
                now = self.clock() - t0
                while nxt < len(order) and order[nxt].arrival <= now:
                    arrived.append(order[nxt])
                    nxt += 1
                with cv:
                    slot_free = bool(free_slots)
                if head is None and arrived and slot_free and not errors:
                    # open the head of the queue (upload its Hamiltonian, learn its footprint)
                    req = arrived.pop(0)
                    state, fp = self.open_fn(req)
                    head = (req, state, int(fp))
                    if fp > self.budget:
                        head = None
                        if self.close_fn is not None:
                            self.close_fn(state)
                        raise AdmissionError(f"request {req.rid} needs {fp} bytes, budget {self.budget}")
                with cv:
                    if head is not None and free_slots and used + head[2] <= self.budget and not errors:
                        req, state, fp = head
                        head = None
                        slot = free_slots.pop(0)
                        used += fp
                        self.peak_bytes = max(self.peak_bytes, used)
                        self.peak_active = max(self.peak_active, self.slots - len(free_slots))
                        th = threading.Thread(target=worker,
                                              args=(req, state, fp, slot, req.arrival, self.clock() - t0),
                                              daemon=True)
                        workers.append(th)
                        th.start()
                        continue
                    if errors:
                        break
                    if nxt >= len(order) and not arrived and head is None and len(free_slots) == self.slots:
                        break
                    if head is None and arrived and free_slots:
                        continue
                    # wait for a finished solve (room, a slot) or the next arrival
                    wait = None if nxt >= len(order) else max(0.0, order[nxt].arrival - (self.clock() - t0))
                    cv.wait(timeout=wait if wait is not None else 1.0)
        finally:
            for th in workers:
                th.join()
            if head is not None and self.close_fn is not None:  # opened, never admitted
                self.close_fn(head[1])
        if errors:
            raise errors[0]
        return sorted(results, key=lambda r: r.rid)


def gpu_ops(precision: int, device: int = 0):
    """open/run/close callables that solve requests with the HIP library.

    open: creates the request's handle (uploads Veff and projectors), returns the
    exact footprint X + workspace + handle arrays.  run: allocates X and the
    workspace on the slot's stream, draws or copies X0, runs the solve (mixed:
    n_iter - 1 steps + the FP64 refinement) and returns the Ritz values."""
    import torch
    from paper_2302_09708_amd import chefsi as cs

    streams: Dict[int, Any] = {}
    elem = 8 if precision == cs.FP64 else 4
    dtype = torch.float64 if precision == cs.FP64 else torch.float32

    def open_fn(req: Request):
        torch.cuda.set_device(device)
        h = cs.Handle(req.prob, precision=precision, max_ns=req.ns)
        fp = req.prob.nd * req.ns * elem + h.chefsi_workspace_bytes(req.ns) + h.device_bytes()
        return (req, h), fp

    def run_fn(state, slot: int):
        req, h = state
        torch.cuda.set_device(device)
        if slot not in streams:
            streams[slot] = torch.cuda.Stream(device=device)
        s = streams[slot]
        with torch.cuda.stream(s):
            ws = torch.empty(h.chefsi_workspace_bytes(req.ns), dtype=torch.uint8, device=f"cuda:{device}")
            if req.x0 is not None:
                X = torch.from_numpy(np.ascontiguousarray(req.x0)).to(device=f"cuda:{device}", dtype=dtype,
                                                                      non_blocking=False)
            else:
                g = torch.Generator(device=f"cuda:{device}")
                g.manual_seed(int(req.x_seed))
                X = torch.randn((req.ns, req.prob.nd), generator=g, device=f"cuda:{device}", dtype=dtype)
            ritz, _, _ = h.solve(X, req.ns, req.degree, req.n_iter, ws, stream=s)
            s.synchronize()
            del X, ws
        return ritz

    def close_fn(state):
        _, h = state
        h.close()

    return open_fn, run_fn, close_fn
