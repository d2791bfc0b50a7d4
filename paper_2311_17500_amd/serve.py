"""Continuous-batching request loop for space-time solves on one GPU.

Requests (a problem description each) arrive over time.  The loop admits them
in arrival order as soon as a solver slot is free and the request's device
footprint (``st_iga_workspace_bytes`` plus its solution vectors) fits the HBM
budget; admitted requests run concurrently, each in its own library context on
its slot's HIP stream, so their kernels overlap on the device while earlier
requests are still in flight.  A finished request frees its slot and memory
for the next one.  Each context is independent and every reduction has a fixed
order, so a request's result does not depend on what else is running.

All arithmetic happens in the HIP library; this module only schedules.
"""
from __future__ import annotations

import dataclasses
import threading
import time
from collections import deque
from typing import List, Optional

import numpy as np

from . import binding


@dataclasses.dataclass
class Record:
    index: int
    arrival: float            # seconds since the start of the stream
    admitted: float = 0.0
    finished: float = 0.0
    dof: int = 0
    footprint: int = 0
    outer_iters: int = 0
    krylov: int = 0
    status: str = "pending"
    shape: tuple = ()         # (degree, space elements, time elements): requests that could share launches
    u: Optional[np.ndarray] = None

    @property
    def latency(self):
        return self.finished - self.arrival


class Server:
    def __init__(self, device="cuda:0", slots: int = 6, hbm_budget: Optional[int] = None,
                 keep_results: bool = False, **options):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.slots = slots
        if hbm_budget is None:
            free, total = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(0.7 * free)
        self.budget = hbm_budget
        self.options = options
        self.keep_results = keep_results
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]

    def footprint(self, prob) -> int:
        """HBM bytes a request holds while admitted (workspace + u, w), cached
        per mesh shape (the workspace does not depend on sigma or the stimulus)."""
        key = (prob.d, prob.p_s, prob.p_t, tuple(prob.nel_s), prob.nel_t)
        if not hasattr(self, "_fp_cache"):
            self._fp_cache = {}
        if key not in self._fp_cache:
            self._fp_cache[key] = binding.workspace_bytes(prob, **self.options) + 2 * prob.dof * 8 + (1 << 20)
        return self._fp_cache[key]

    def _solve(self, slot: int, prob, rec: Record, t0: float):
        torch = self.torch
        stream = self.streams[slot]
        S = None
        try:
            with torch.cuda.device(self.device):
                S = binding.Solver(prob, device=self.device, stream=stream, **self.options)
                u, w, rep = S.solve()
                rec.outer_iters, rec.krylov = rep.outer_iters, rep.krylov_total
                if self.keep_results:
                    rec.u = u.cpu().numpy()
                del u, w
                stream.synchronize()
            rec.status = "ok"
        except Exception as e:   # any failure is recorded; the slot is given back by the caller
            rec.status = f"{type(e).__name__}: {e}"
        finally:
            if S is not None:
                try:
                    S.close()
                except Exception as e:
                    if rec.status == "ok":
                        rec.status = f"close failed: {e}"
            rec.finished = time.perf_counter() - t0

    def run(self, requests) -> List[Record]:
        """requests: iterable of (arrival_seconds, problem).  Blocks until all finish."""
        reqs = list(requests)
        recs = [Record(i, float(t), dof=p.dof, footprint=self.footprint(p),
                       shape=(p.p_s, p.p_t, tuple(p.nel_s), p.nel_t)) for i, (t, p) in enumerate(reqs)]
        for r in recs:
            if r.footprint > self.budget:
                raise ValueError(f"request {r.index} needs {r.footprint} bytes, budget {self.budget}")
        lock = threading.Condition()
        used = [0]
        free_slots = deque(range(self.slots))
        threads = []
        t0 = time.perf_counter()

        def worker(slot, prob, rec):
            try:
                self._solve(slot, prob, rec, t0)
            finally:
                with lock:
                    used[0] -= rec.footprint
                    free_slots.append(slot)
                    lock.notify_all()

        for (t_arr, prob), rec in zip(reqs, recs):
            now = time.perf_counter() - t0
            if t_arr > now:
                time.sleep(t_arr - now)
            with lock:
                while not free_slots or used[0] + rec.footprint > self.budget:
                    lock.wait()
                slot = free_slots.popleft()
                used[0] += rec.footprint
                rec.admitted = time.perf_counter() - t0
            th = threading.Thread(target=worker, args=(slot, prob, rec), daemon=True)
            th.start()
            threads.append(th)
        for th in threads:
            th.join()
        return recs


def overlap_stats(recs: List[Record]) -> dict:
    """At each admission: how many other requests were in flight, and how many
    of those had the same shape (degree, mesh), i.e. work a launch shared
    across requests could have grouped with it."""
    others, same = [], []
    for r in recs:
        live = [q for q in recs if q is not r and q.admitted <= r.admitted < q.finished]
        others.append(len(live))
        same.append(sum(1 for q in live if q.shape == r.shape))
    if not recs:
        return {}
    return {"in_flight_at_admission_mean": float(np.mean(others)),
            "same_shape_in_flight_mean": float(np.mean(same)),
            "admissions_with_same_shape_partner": float(np.mean([s > 0 for s in same])),
            "distinct_shapes": len({r.shape for r in recs})}


def summarize(recs: List[Record]) -> dict:
    ok = [r for r in recs if r.status == "ok"]
    lat = np.array([r.latency for r in ok]) if ok else np.array([np.nan])
    makespan = max(r.finished for r in recs) - min(r.arrival for r in recs)
    return {"requests": len(recs), "completed": len(ok),
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(np.mean(lat)), "makespan_s": float(makespan),
            "dof_per_s": float(sum(r.dof for r in ok) / makespan) if makespan > 0 else None,
            "outer_iters_mean": float(np.mean([r.outer_iters for r in ok])) if ok else None,
            "krylov_mean": float(np.mean([r.krylov for r in ok])) if ok else None,
            "failures": [r.status for r in recs if r.status != "ok"][:5], **overlap_stats(recs)}
