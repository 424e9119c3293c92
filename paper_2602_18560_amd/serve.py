"""Continuous-batching service of subtraction jobs on one GPU.

Jobs (a catalog in pinned host memory, or population-model hyperparameters
and a seed to draw it on the GPU, plus its run configuration) are queued in
arrival order.  A job is admitted into the shared gbsub batch as soon as a
slot is free and its device footprint (catalog + workspace) fits the byte
budget; admission copies the catalog host-to-device, runs its preparation and
adds it to every following loop launch.  All running jobs advance together,
``chunk`` loop bodies per graph launch; a job that settles is retired (its
results land in its context) and its memory returns to the budget.  Every
step of the method runs in the library's kernels; this module only schedules.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import gbsub as G
from .autotune import grid_class


@dataclass
class Request:
    index: int
    arrival_s: float
    A: object            # pinned host tensors, fp32 (id: int32 view of uint32); None: drawn on the GPU
    f: object
    fdot: object
    ids: object
    run: object          # inputs.RunConfig
    n: int = 0           # sources (read from A when it is given)
    model: object = None  # gbsub.PopulationStruct of a catalog drawn at admission
    seed: int = 0


def model_request(job) -> Request:
    """Request of an inputs.ModelJob: its catalog is drawn on the GPU at
    admission (no host catalog, no host-to-device copy)."""
    return Request(job.index, job.arrival_s, None, None, None, None, run=job.run, n=job.n,
                   model=G.population(**job.model), seed=job.seed)


@dataclass
class Completion:
    index: int
    status: int
    summary: G.Summary
    n_sources: int
    arrival_s: float
    admit_s: float
    done_s: float
    context: G.Context = field(repr=False, default=None)

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def pin_catalog(cat):
    """Pinned host tensors of a host catalog (done ahead of a job's arrival)."""
    import torch

    def p(a, dt):
        t = torch.empty(a.shape[0], dtype=dt, pin_memory=True)
        t.numpy()[:] = a
        return t
    return (p(cat.A.astype(np.float32), torch.float32), p(cat.f.astype(np.float32), torch.float32),
            p(cat.fdot.astype(np.float32), torch.float32),
            p(cat.id.astype(np.uint32).view(np.int32), torch.int32))


class Server:
    """One GPU, one stream, one batch of up to ``max_slots`` running jobs."""

    def __init__(self, max_slots: int = 64, budget_bytes: float = 200 * 2**30, chunk: int = 4,
                 keep_contexts: bool = False, schedules=None, keep_jobs=()):
        import torch
        self.torch = torch
        self.stream = torch.cuda.Stream()
        self.batch = G.Batch(max_slots)
        self.max_slots = max_slots
        self.budget = float(budget_bytes)
        self.chunk = int(chunk)
        self.keep = keep_contexts
        self.keep_jobs = set(keep_jobs)   # job indices whose contexts (results) are kept
        # schedule (tile size, split budget) per grid class, e.g. from autotune.tune_batch
        self.schedules = dict(schedules or {})
        self.queue: deque[Request] = deque()
        self.live = {}               # slot -> (request, ctx, device catalog, bytes, admit time)
        self.used = 0.0
        self.h2d_events = []         # (start, end, bytes) per admitted job
        self.t0 = None

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def start(self):
        self.t0 = time.perf_counter()

    def submit(self, req: Request):
        if req.A is not None:
            req.n = int(req.A.shape[0])
        self.queue.append(req)

    def footprint(self, ctx: G.Context, n: int) -> int:
        return ctx.workspace_size(n) + 256 + 16 * n

    def _admit_ready(self, now: float):
        torch = self.torch
        while self.queue and self.queue[0].arrival_s <= now and len(self.live) < self.max_slots:
            req = self.queue[0]
            sch = self.schedules.get(grid_class(req.run), {})
            ctx = G.Context(G.config_from_run(req.run, **sch))
            need = self.footprint(ctx, req.n)
            if self.live and self.used + need > self.budget:
                ctx.close()
                return                      # first in, first served: wait for memory
            self.queue.popleft()
            with torch.cuda.stream(self.stream):
                if req.A is None:          # drawn on the GPU, on the serving stream
                    dev = [torch.empty(req.n, dtype=dt, device="cuda") for dt in
                           (torch.float32, torch.float32, torch.float32, torch.int32)]
                    G.generate(req.model, req.seed, req.n, out=G.DeviceCatalog(*dev), stream=self.stream)
                else:
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record(self.stream)
                    dev = [torch.empty(req.n, dtype=x.dtype, device="cuda") for x in
                           (req.A, req.f, req.fdot, req.ids)]
                    for d, h in zip(dev, (req.A, req.f, req.fdot, req.ids)):
                        d.copy_(h, non_blocking=True)
                    b.record(self.stream)
                    self.h2d_events.append((a, b, 16 * req.n))
                ws = torch.empty(ctx.workspace_size(req.n) + 256, dtype=torch.uint8, device="cuda")
            ctx.workspace = ws          # the results live there: the context keeps it
            dc = G.DeviceCatalog(*dev)
            k = self.batch.admit(ctx, dc, ws=ws, stream=self.stream)
            self.live[k] = (req, ctx, dc, need, self.now())
            self.used += need

    def pump(self) -> list[Completion]:
        """Admit what has arrived and fits, run one chunk of loop bodies,
        retire what settled.  Returns the jobs completed by this call."""
        self._admit_ready(self.now())
        if not self.live:
            return []
        self.batch.step(self.chunk, self.stream)
        state, _ = self.batch.poll(self.stream)
        out = []
        for k in [k for k in self.live if state[k] != G.SLOT_RUNNING]:
            req, ctx, dc, need, t_adm = self.live.pop(k)
            st, s = self.batch.retire(k, self.stream)
            keep = self.keep or req.index in self.keep_jobs
            out.append(Completion(req.index, st, s, req.n, req.arrival_s, t_adm, self.now(),
                                  ctx if keep else None))
            if not keep:
                ctx.close()
            self.used -= need
        return out

    def idle(self) -> bool:
        return not self.live and not self.queue

    def next_arrival(self):
        return self.queue[0].arrival_s if self.queue else None

    def h2d_stats(self):
        """(total bytes, total ms) of the host-to-device catalog copies."""
        self.torch.cuda.synchronize()
        ms = sum(a.elapsed_time(b) for a, b, _ in self.h2d_events)
        return sum(n for _, _, n in self.h2d_events), ms

    def close(self):
        for k in list(self.live):
            self.live.pop(k)[1].close()
        self.batch.close()


def serve(requests, max_slots=64, budget_bytes=200 * 2**30, chunk=4, keep_contexts=False, schedules=None,
          keep_jobs=(), progress=None):
    """Runs every request to completion in wall-clock time (arrivals are
    honoured: the server idles until the next one is due).  Returns the
    completions in completion order and the server (for its statistics).
    ``progress(n_done, n_total)``, if given, is called every 100 completions."""
    srv = Server(max_slots, budget_bytes, chunk, keep_contexts, schedules, keep_jobs)
    for r in sorted(requests, key=lambda r: r.arrival_s):
        srv.submit(r)
    done = []
    srv.start()
    while not srv.idle():
        if not srv.live:
            nxt = srv.next_arrival()
            wait = nxt - srv.now()
            if wait > 0:
                time.sleep(min(wait, 0.05))
        before = len(done)
        done.extend(srv.pump())
        if progress and len(done) // 100 > before // 100:
            progress(len(done), len(requests))
    return done, srv
