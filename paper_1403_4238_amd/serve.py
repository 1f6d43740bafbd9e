"""Continuous-batching serving loop for object-removal jobs.

Jobs arrive over time (e.g. a Poisson process).  A job is admitted when a
batch slot is free and its device footprint (the workspace its context needs)
fits the memory budget: both are reserved at once, and the job's context is
prepared (upload and initialisation) on a worker thread with its own stream
while the loop keeps stepping the running jobs.  A prepared job is attached to
the running batch between two batch steps, in arrival order, once the engine
has room for it (an engine may gate this: ``GpuEngine(tiles_per_group=N)``
attaches a job only while every search work-group of the batched persistent
dispatch would hold at most N tiles; a job arriving at an empty batch always
starts).  Every batch step advances every attached unfinished job by G fill
iterations, so jobs that arrive while others run share the device with them.
Finished jobs are read back, detached and their memory released, which may
admit queued jobs.  Latency is completion time minus arrival time.

The loop talks to an engine object; ``GpuEngine`` drives libinpaint through
the binding, ``FakeEngine`` (tests) simulates iteration counts on the CPU.
An engine with ``prepare`` / ``attach`` is admitted asynchronously (when the
server has workers); otherwise ``admit`` runs on the loop.
"""
from __future__ import annotations

import concurrent.futures as cf
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
                 keep_results: bool = True, workers: int = 0):
        if capacity < 1 or budget_bytes <= 0 or graph_iters < 1 or workers < 0:
            raise ValueError("capacity, budget and graph_iters must be positive")
        self.workers = workers if hasattr(engine, "prepare") else 0
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
        if self.workers:
            with cf.ThreadPoolExecutor(self.workers, thread_name_prefix="admit") as pool:
                return self._run(jobs, pool)
        return self._run(jobs, None)

    def _run(self, jobs, pool) -> list[JobRecord]:
        eng = self.engine
        recs = [JobRecord(i, getattr(j, "name", str(i)), float(j.arrival_s), int(eng.footprint(j)))
                for i, j in enumerate(jobs)]
        order = sorted(range(len(jobs)), key=lambda i: (recs[i].arrival_s, i))
        t0 = self.clock()
        nxt = 0
        queue: list[int] = []
        preparing: dict[int, cf.Future] = {}   # admitted, context being prepared off the loop
        ready: list[tuple[int, object]] = []   # prepared, waiting for room in the batch
        active: dict[int, object] = {}
        room = getattr(eng, "room", None)

        def fail(i, e):
            recs[i].status, recs[i].error = "failed", str(e)
            recs[i].done_s = self.clock() - t0
            self.used -= recs[i].footprint

        while nxt < len(order) or queue or preparing or ready or active:
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
            while (queue and len(active) + len(preparing) + len(ready) < self.capacity
                   and self.used + recs[queue[0]].footprint <= self.budget):
                i = queue.pop(0)
                self.used += recs[i].footprint
                recs[i].status = "admitted"
                if pool is not None:
                    preparing[i] = pool.submit(eng.prepare, jobs[i])
                    continue
                try:
                    if room is None:
                        active[i] = eng.admit(jobs[i])
                    else:
                        ready.append((i, eng.prepare(jobs[i])))
                        continue
                except Exception as e:  # invalid job: report it, keep serving the rest
                    fail(i, e)
                    continue
                recs[i].admit_s = self.clock() - t0
                recs[i].status = "running"
            for i in [i for i, f in preparing.items() if f.done()]:
                f = preparing.pop(i)
                try:
                    ready.append((i, f.result()))
                except Exception as e:
                    fail(i, e)
            # prepared jobs join the batch between two steps, in arrival
            # order, while the engine has room for them (always when the
            # batch is empty); a job without room holds back the later ones
            ready.sort(key=lambda ip: (recs[ip[0]].arrival_s, ip[0]))
            while ready and (not active or room is None or room(ready[0][1])):
                i, prepared = ready.pop(0)
                try:
                    active[i] = eng.attach(prepared)
                except Exception as e:
                    fail(i, e)
                    continue
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
            elif preparing:
                cf.wait(list(preparing.values()), timeout=0.05, return_when=cf.FIRST_COMPLETED)
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
                 fail_on: Callable | None = None, room: Callable | None = None):
        self.iterations = iterations
        # room(running jobs, job) -> bool: the batch has room for job
        self.room = None if room is None else (lambda job: room([st[0] for st in self.live.values()], job))
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

    def prepare(self, job):
        if self.fail_on and self.fail_on(job):
            raise ValueError("invalid job")
        return job

    def attach(self, job):
        h = self._next
        self._next += 1
        self.live[h] = [job, 0, int(self.iterations(job))]
        self.max_live = max(self.max_live, len(self.live))
        return h

    def admit(self, job):
        return self.attach(self.prepare(job))

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
    """libinpaint through the binding: one Batch (the batched persistent
    form unless ``form`` says otherwise); contexts are prepared on a side
    stream of the calling thread (a server worker, so the loop keeps stepping
    meanwhile) and attached between steps while the batch has room for
    their search tiles, at most ``tiles_per_group`` per search work-group
    (``Batch.room``; 0: whenever a slot is free); their torch workspaces are
    freed on release."""

    def __init__(self, capacity: int, graph_iters: int = 8, autotune: bool = True, tune_cache: str | None = None,
                 log: bool = True, path: str = "mfma", form: str = "persistent", tiles_per_group: int = 0):
        import threading

        import torch

        from . import binding as B
        self.B = B
        self.torch = torch
        self.stream = torch.cuda.current_stream()
        self.device = torch.cuda.current_device()
        self._local = threading.local()
        self.batch = B.Batch(capacity, graph_iters, autotune, tune_cache, stream=self.stream, form=form)
        self.log = log
        self.path = path
        self.tiles_per_group = tiles_per_group
        if not tiles_per_group:
            self.room = None   # attach whenever a slot is free

    def _side(self):
        s = getattr(self._local, "stream", None)
        if s is None:
            self.torch.cuda.set_device(self.device)
            s = self._local.stream = self.torch.cuda.Stream()
        return s

    def _path_id(self, job):
        # the int8-MFMA search serves patches up to 13x13
        return self.B.PATH_MFMA if self.path == "mfma" and job.patch_radius <= 6 else self.B.PATH_SIMT

    def footprint(self, job) -> int:
        p = self.B.make_params(job.patch_radius, job.search_mode, job.alpha, job.rect, path=self._path_id(job),
                               log_capacity=int(np.count_nonzero(job.mask)) if self.log else 0)
        return self.B.inpaint_workspace_bytes(job.width, job.height, p)

    def prepare(self, job):
        side = self._side()
        with self.torch.cuda.stream(side):
            ctx = self.B.Inpainter(job.rgb, job.mask, job.patch_radius, job.search_mode, job.alpha, job.rect,
                                   log_capacity=int(np.count_nonzero(job.mask)) if self.log else 0,
                                   stream=side, path=self._path_id(job))
        return ctx

    def room(self, ctx) -> bool:
        return self.batch.room(ctx, self.tiles_per_group)

    def attach(self, ctx):
        self.batch.attach(ctx)
        return ctx

    def admit(self, job):
        return self.attach(self.prepare(job))

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
