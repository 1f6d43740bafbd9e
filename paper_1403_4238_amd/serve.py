"""Continuous-batching serving loop for object-removal jobs.

Jobs arrive over time (e.g. a Poisson process).  A job is admitted when a
batch slot is free and its device footprint (the workspace its context needs)
fits the memory budget; it is then created on a side stream and attached to
the running batch between two batch steps.  Every batch step advances every
attached unfinished job by G fill iterations in one persistent, graph-replayed
launch sequence, so jobs that arrive while others run share the device with
them.  Finished jobs are read back, detached and their memory released,
which may admit queued jobs.  Latency is completion time minus arrival time.

The loop talks to an engine object; ``GpuEngine`` drives libinpaint through
the binding, ``FakeEngine`` (tests) simulates iteration counts on the CPU.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable

import numpy as np


@dataclasses.dataclass
class JobRecord:
    index: int
    name: str
    arrival_s: float
    footprint: int
    admit_s: float | None = None
    done_s: float | None = None
    iterations: int = 0
    evals: int = 0
    status: str = "queued"          # queued | running | done | rejected | failed
    error: str = ""
    result: object = None

    @property
    def latency_s(self) -> float | None:
        return None if self.done_s is None else self.done_s - self.arrival_s


class Server:
    """Admission by footprint + slot, continuous batching, latency stats."""

    def __init__(self, engine, budget_bytes: int, capacity: int, graph_iters: int = 8,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
                 keep_results: bool = True):
        if capacity < 1 or budget_bytes <= 0 or graph_iters < 1:
            raise ValueError("capacity, budget and graph_iters must be positive")
        self.engine = engine
        self.budget = int(budget_bytes)
        self.capacity = int(capacity)
        self.G = int(graph_iters)
        self.clock = clock
        self.sleep = sleep
        self.keep_results = keep_results
        self.used = 0
        self.peak_used = 0
        self.peak_active = 0
        self.steps = 0

    def run(self, jobs) -> list[JobRecord]:
        """Serves ``jobs`` (objects with .arrival_s) to completion."""
        eng = self.engine
        recs = [JobRecord(i, getattr(j, "name", str(i)), float(j.arrival_s), int(eng.footprint(j)))
                for i, j in enumerate(jobs)]
        order = sorted(range(len(jobs)), key=lambda i: (recs[i].arrival_s, i))
        t0 = self.clock()
        nxt = 0
        queue: list[int] = []
        active: dict[int, object] = {}
        while nxt < len(order) or queue or active:
            now = self.clock() - t0
            while nxt < len(order) and recs[order[nxt]].arrival_s <= now:
                i = order[nxt]
                nxt += 1
                if recs[i].footprint > self.budget:
                    recs[i].status, recs[i].error = "rejected", "footprint exceeds the memory budget"
                    recs[i].done_s = now
                    continue
                queue.append(i)
            # admit in arrival order while a slot and memory are free
            while queue and len(active) < self.capacity and self.used + recs[queue[0]].footprint <= self.budget:
                i = queue.pop(0)
                try:
                    h = eng.admit(jobs[i])
                except Exception as e:  # invalid job: report it, keep serving the rest
                    recs[i].status, recs[i].error = "failed", str(e)
                    recs[i].done_s = self.clock() - t0
                    continue
                active[i] = h
                self.used += recs[i].footprint
                recs[i].admit_s = self.clock() - t0
                recs[i].status = "running"
            self.peak_used = max(self.peak_used, self.used)
            self.peak_active = max(self.peak_active, len(active))
            if active:
                eng.step(self.G)
                self.steps += 1
                now = self.clock() - t0
                for i in [i for i, h in active.items() if eng.finished(h)]:
                    h = active.pop(i)
                    r = recs[i]
                    try:
                        res = eng.collect(h)
                        r.iterations, r.evals = res.get("iterations", 0), res.get("evals", 0)
                        r.result = res if self.keep_results else None
                        r.status = "done"
                    except Exception as e:
                        r.status, r.error = "failed", str(e)
                    finally:
                        eng.release(h)
                    r.done_s = now
                    self.used -= r.footprint
            elif nxt < len(order):
                wait = recs[order[nxt]].arrival_s - (self.clock() - t0)
                if wait > 0:
                    self.sleep(min(wait, 0.05))
        return recs


def summarize(recs: list[JobRecord]) -> dict:
    done = [r for r in recs if r.status == "done"]
    lat = np.array([r.latency_s for r in done], dtype=np.float64)
    if not len(done):
        return {"completed": 0, "rejected": sum(r.status == "rejected" for r in recs),
                "failed": sum(r.status == "failed" for r in recs)}
    span = max(r.done_s for r in done) - min(r.arrival_s for r in recs)
    evals = sum(r.evals for r in done)
    return {
        "completed": len(done),
        "rejected": sum(r.status == "rejected" for r in recs),
        "failed": sum(r.status == "failed" for r in recs),
        "p50_latency_ms": round(1000 * float(np.percentile(lat, 50)), 3),
        "p99_latency_ms": round(1000 * float(np.percentile(lat, 99)), 3),
        "mean_latency_ms": round(1000 * float(lat.mean()), 3),
        "jobs_per_s": round(len(done) / span, 3) if span > 0 else None,
        "patch_evals_per_s": round(evals / span, 1) if span > 0 else None,
        "span_s": round(span, 4),
    }


class FakeEngine:
    """CPU stand-in with the engine interface: each job needs a scripted
    number of iterations and has a scripted footprint; a step advances every
    admitted job by G iterations and costs ``step_cost_s`` of (fake) time."""

    def __init__(self, iterations: Callable, footprint: Callable, clock=None, step_cost_s: float = 0.0,
                 fail_on: Callable | None = None):
        self.iterations = iterations
        self._footprint = footprint
        self.step_cost_s = step_cost_s
        self.clock = clock
        self.fail_on = fail_on
        self.live: dict[int, list] = {}
        self.max_live = 0
        self.released = 0
        self._next = 0

    def footprint(self, job) -> int:
        return self._footprint(job)

    def admit(self, job):
        if self.fail_on and self.fail_on(job):
            raise ValueError("invalid job")
        h = self._next
        self._next += 1
        self.live[h] = [job, 0, int(self.iterations(job))]
        self.max_live = max(self.max_live, len(self.live))
        return h

    def step(self, G: int) -> int:
        for st in self.live.values():
            st[1] = min(st[1] + G, st[2])
        if self.clock is not None:
            self.clock.advance(self.step_cost_s)
        return sum(1 for st in self.live.values() if st[1] < st[2])

    def finished(self, h) -> bool:
        st = self.live[h]
        return st[1] >= st[2]

    def collect(self, h) -> dict:
        job, done, need = self.live[h]
        return {"iterations": done, "evals": done, "job": job}

    def release(self, h):
        del self.live[h]
        self.released += 1


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self) -> float:
        return self.t

    def advance(self, dt: float):
        self.t += dt

    def sleep(self, dt: float):
        self.t += dt


class GpuEngine:
    """libinpaint through the binding: one Batch, contexts created on a side
    stream, their torch workspaces freed on release."""

    def __init__(self, capacity: int, graph_iters: int = 8, autotune: bool = True, tune_cache: str | None = None,
                 log: bool = True):
        import torch

        from . import binding as B
        self.B = B
        self.torch = torch
        self.stream = torch.cuda.current_stream()
        self.side = torch.cuda.Stream()
        self.batch = B.Batch(capacity, graph_iters, autotune, tune_cache, stream=self.stream)
        self.log = log

    def footprint(self, job) -> int:
        p = self.B.make_params(job.patch_radius, job.search_mode, job.alpha, job.rect,
                               log_capacity=int(np.count_nonzero(job.mask)) if self.log else 0)
        return self.B.inpaint_workspace_bytes(job.width, job.height, p)

    def admit(self, job):
        with self.torch.cuda.stream(self.side):
            ctx = self.B.Inpainter(job.rgb, job.mask, job.patch_radius, job.search_mode, job.alpha, job.rect,
                                   log_capacity=int(np.count_nonzero(job.mask)) if self.log else 0,
                                   stream=self.side)
        self.batch.attach(ctx)
        return ctx

    def step(self, G: int) -> int:
        return self.batch.step(G)

    def finished(self, ctx) -> bool:
        st = self.batch.status(ctx)
        if st == 3:
            return True            # collect() raises for it
        return st == 2

    def collect(self, ctx) -> dict:
        if self.batch.status(ctx) == 3:
            raise RuntimeError("device error in this job")
        it, _ = ctx.progress()
        _, cands = ctx.search_info()
        out = {"iterations": it, "evals": it * cands, "image": ctx.read_image()}
        if self.log:
            out["log"] = ctx.read_log(0, it)
        return out

    def release(self, ctx):
        self.batch.detach(ctx)
        ctx.close()
        ctx.workspace = None
