"""Served form: a request loop over the batched C ABI.

Requests (each a mesh, order, precision, parameters and a step count) arrive
over time.  The loop keeps the batch stepping (gb_batch_run, asynchronous,
a few steps at a time while requests wait for admission, up to the next
completion otherwise) while a worker thread does the host-side setup on a
separate stream:

  * the mesh of every arrived request (connectivity, trace map, upload);
  * for the requests admitted in arrival order -- a request is taken while
    its device footprint (gb_solver_footprint + gb_mesh_footprint) fits the
    free part of the budget, and one that does not fit waits, and so does
    every request behind it -- the solver and its initial state;
  * the final state of the requests that completed;

at each step boundary the loop retires the requests that reached their step
count (gb_batch_poll; latency = completion - arrival) and adds the prepared
ones to the batch (gb_batch_add).

A request's state stays on the device from admission to completion.  This
module only marshals arguments and keeps the books; every step of every
request runs in libgb.so.
"""
from __future__ import annotations

import math
import os
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

from . import _lib as L
from .session import equilibrium_moments, initial_offset, motion_params


@dataclass
class Request:
    index: int
    arrival: float                  # seconds after the start of serve()
    case: object                    # a workloads Case
    nsteps: int
    precision: int = L.GB_FP32
    keep_state: bool = False        # copy the final state to the host
    # filled in by the server
    bytes: int = 0
    dof: int = 0
    t_admit: float = math.nan
    t_done: float = math.nan
    state: np.ndarray | None = None
    t_final: float = math.nan
    steps_done: int = 0
    rejected: bool = False
    error: str | None = None        # latched device error reported at completion
    _mesh: object = None
    _solver: object = None
    _params: object = None


def admit_fifo(queue_bytes, free_bytes: int) -> int:
    """Number of requests admitted from the head of a FIFO queue whose
    footprints are queue_bytes, given free_bytes: stops at the first request
    that does not fit (no overtaking)."""
    n = 0
    for b in queue_bytes:
        if b > free_bytes:
            break
        free_bytes -= b
        n += 1
    return n


def latency_summary(latencies) -> dict:
    """p50 / p99 / max / mean of a list of latencies (seconds), nearest-rank
    percentiles."""
    x = np.sort(np.asarray(latencies, float))
    if x.size == 0:
        return {"n": 0, "p50": None, "p99": None, "max": None, "mean": None}

    def pct(p):
        k = max(1, int(math.ceil(p / 100.0 * x.size)))
        return float(x[k - 1])

    return {"n": int(x.size), "p50": pct(50), "p99": pct(99), "max": float(x[-1]), "mean": float(x.mean())}


def case_params(case, precision):
    """gb_params for a case: physical constants, and for cases with far-field
    faces the free-stream equilibrium and the sponge layer."""
    q_inf = sponge = None
    if "u" in case.extra and case.face_tag is not None:
        u = case.extra["u"]
        q_inf = equilibrium_moments(case.dim, np.array(1.0), [np.array(v) for v in u], case.c)
    if "sponge" in case.extra:
        sponge = case.extra["sponge"]
    return L.make_params(case.c, case.tau, precision, q_inf=q_inf, sponge=sponge)


def set_initial_state(case, mesh, solver):
    """The case's initial state (equilibrium of its macroscopic fields at the
    mesh's nodes), formed by the library on the device."""
    X = L.gb_mesh_nodes(mesh, case.dim)
    rho, u = case.macroscopic(X)
    NF = 6 if case.dim == 2 else 10
    L.gb_state_set_equilibrium(solver, rho, np.stack(u, axis=1), initial_offset(case, NF))


class Server:
    """One batch on one device, with a separate context (stream) for request
    setup so that building and uploading a new request does not wait for the
    batch's queued steps.  Both streams are non-blocking streams of the
    library's own HIP runtime."""

    def __init__(self, budget_bytes: int, device: int = 0, steps_per_launch: int = 5, autotune: bool = True,
                 tune_cache: str | None = None, concurrency: int = 1, max_steps_per_launch: int = 0,
                 setup_workers: int = 4):
        self.streams = [L.gb_stream_create(device), L.gb_stream_create(device)]
        self.run_ctx = L.gb_ctx_create(device, self.streams[0])
        self.setup_ctx = L.gb_ctx_create(device, self.streams[1])
        self.batch = L.gb_batch_create(self.run_ctx, budget_bytes)
        L.gb_batch_set_autotune(self.batch, autotune)
        if concurrency > 1:
            L.gb_batch_set_concurrency(self.batch, concurrency)
        self.budget = int(budget_bytes)
        self.steps_per_launch = int(steps_per_launch)
        # when no request is waiting, the batch runs up to the next completion
        # (at most this many steps, in multiples of 8) between step boundaries
        self.max_steps_per_launch = int(max_steps_per_launch)
        self.classes = []
        # host threads building request meshes (connectivity) at once
        self.setup_workers = max(1, int(setup_workers))
        # launch tiles from earlier runs (gb_tune_cache_*), saved again at close
        self.tune_cache = tune_cache
        if tune_cache and os.path.exists(tune_cache):
            L.gb_tune_cache_load(tune_cache)

    # -------------------------------------------------------------- requests
    def _prepare(self, r: Request):
        c = r.case
        r._mesh = L.gb_mesh_create(self.setup_ctx, c.dim, c.N, c.vx, c.etov, c.period, c.face_tag)
        kind, p = motion_params(c.motion)
        L.gb_set_motion(r._mesh, kind, p)
        r._params = case_params(c, r.precision)
        r.bytes = L.gb_solver_footprint(r._mesh, r._params) + L.gb_mesh_footprint(r._mesh)
        K, Np, NF, _, _ = L.gb_mesh_sizes(r._mesh)
        r.dof = K * Np * NF

    def _stage(self, r: Request):
        """Solver and initial state of an admitted request (setup stream)."""
        r._solver = L.gb_solver_create(r._mesh, r._params)
        set_initial_state(r.case, r._mesh, r._solver)

    def _finish(self, r: Request):
        shape = None
        if r.keep_state:
            K, Np, NF, _, _ = L.gb_mesh_sizes(r._mesh)
            shape = (K, NF, Np)
        try:
            q, t, step = L.gb_state_get(r._solver, shape)
            r.t_final, r.steps_done, r.state = t, step, q
        except L.GbError as ex:
            # a latched error (non-physical state, inverted element) fails
            # this request only
            r.error = str(ex)
        self._release(r)

    def _release(self, r: Request):
        if r._solver is not None:
            L.gb_solver_destroy(r._solver)
            r._solver = None
        if r._mesh is not None:
            L.gb_mesh_destroy(r._mesh)
            r._mesh = None

    # -------------------------------------------------------------- loop
    def serve(self, requests, clock=time.perf_counter, sleep=time.sleep) -> dict:
        pend = deque(sorted(requests, key=lambda q: q.arrival))
        queue: deque = deque()          # arrived, in arrival order (setup of the mesh submitted)
        staged: list = []               # admitted, solver setup submitted, not yet in the batch
        active: dict = {}
        remaining: dict = {}            # ticket -> steps still to run
        finished = []
        prep, stg, fin = {}, {}, []     # futures of the host-side setup work
        # Host-side setup runs on worker threads on the setup context's
        # stream, so the stepping loop keeps the GPU fed meanwhile: mesh
        # builds (host connectivity, the longest part) on several threads,
        # solver creation, initial state and final-state download in order on
        # one.
        pool = ThreadPoolExecutor(max_workers=1)
        mesh_pool = ThreadPoolExecutor(max_workers=self.setup_workers)
        t0 = clock()

        def intake():
            now = clock() - t0
            while pend and pend[0].arrival <= now:
                r = pend.popleft()
                queue.append(r)
                prep[id(r)] = mesh_pool.submit(self._prepare, r)
            _, used, _ = L.gb_batch_info(self.batch)
            free = self.budget - used - sum(r.bytes for r in staged)
            # arrival order, no overtaking: stop at the first request whose
            # mesh is not ready yet or whose footprint does not fit
            while queue and prep[id(queue[0])].done():
                r = queue[0]
                prep[id(r)].result()
                if r.bytes > free:
                    break
                queue.popleft()
                free -= r.bytes
                r.t_admit = clock() - t0
                stg[id(r)] = pool.submit(self._stage, r)
                staged.append(r)

        def join_staged(block: bool):
            while staged and (block or stg[id(staged[0])].done()):
                r = staged.pop(0)
                stg.pop(id(r)).result()
                block = False
                try:
                    tk = L.gb_batch_add(self.batch, r._solver, r.case.dt, r.nsteps)
                    active[tk] = r
                    remaining[tk] = r.nsteps
                except L.GbError as ex:
                    # a request the batch cannot take (a shape the batched
                    # kernel is not built for, a full table) fails on its own
                    r.error = str(ex)
                    r.t_done = clock() - t0
                    fin.append(pool.submit(self._release, r))
                    finished.append(r)

        try:
            while pend or queue or staged or active:
                intake()
                join_staged(block=False)
                if not active:
                    if staged:
                        join_staged(block=True)
                    elif queue:
                        r = queue[0]
                        prep[id(r)].result()
                        _, used, _ = L.gb_batch_info(self.batch)
                        if r.bytes > self.budget - used:
                            # nothing running and the head does not fit: it never will
                            queue.popleft()
                            r.rejected = True
                            fin.append(pool.submit(self._release, r))
                            finished.append(r)
                    elif pend:
                        sleep(max(0.0, pend[0].arrival - (clock() - t0)))
                    continue
                n = self.steps_per_launch
                if self.max_steps_per_launch > n and not pend and not queue and not staged:
                    # nobody waits for admission: run to the next completion
                    n = max(n, min(min(remaining.values()), self.max_steps_per_launch))
                    if n >= 8:
                        n -= n % 8
                L.gb_batch_run(self.batch, n)
                for tk in remaining:
                    remaining[tk] = max(0, remaining[tk] - n)
                if not self.classes:
                    self.classes = [L.gb_batch_class_info(self.batch, i)
                                    for i in range(L.gb_batch_class_count(self.batch))]
                intake()                     # overlaps the steps just enqueued
                for ticket in L.gb_batch_poll(self.batch, len(active)):
                    remaining.pop(ticket, None)
                    r = active.pop(ticket)
                    r.t_done = clock() - t0
                    fin.append(pool.submit(self._finish, r))
                    finished.append(r)
        finally:
            mesh_pool.shutdown(wait=True)
            pool.shutdown(wait=True)
        for f in fin:
            f.result()
        done = [r for r in finished if not r.rejected and r.error is None]
        lat = [r.t_done - r.arrival for r in done]
        work = sum(4.0 * r.dof * r.nsteps for r in done)
        first = min((r.arrival for r in done), default=0.0)
        last = max((r.t_done for r in done), default=0.0)
        span = max(last - first, 1e-12)
        return {"requests": len(requests), "completed": len(done),
                "rejected": sum(r.rejected for r in finished),
                "failed": sum(r.error is not None for r in finished),
                "latency_s": latency_summary(lat),
                "wait_s": latency_summary([r.t_admit - r.arrival for r in done]),
                "makespan_s": span, "dof_stages": work, "gdof_stage_s": work / span / 1e9,
                "classes": self.classes}

    def close(self):
        if self.batch:
            if self.tune_cache:
                L.gb_tune_cache_save(self.tune_cache)
            L.gb_batch_destroy(self.batch)
            self.batch = None
            L.gb_ctx_destroy(self.setup_ctx)
            L.gb_ctx_destroy(self.run_ctx)
            for st in self.streams:
                L.gb_stream_destroy(st)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serial_rate(req: Request, device: int = 0, steps: int = 20, warmup: int = 3) -> float:
    """Seconds per step of the request solved alone (graph replay of the
    single-mesh path), from `steps` timed steps after `warmup`."""
    ctx = L.gb_ctx_create(device, 0)
    c = req.case
    mesh = L.gb_mesh_create(ctx, c.dim, c.N, c.vx, c.etov, c.period, c.face_tag)
    try:
        kind, p = motion_params(c.motion)
        L.gb_set_motion(mesh, kind, p)
        s = L.gb_solver_create(mesh, case_params(c, req.precision))
        try:
            set_initial_state(c, mesh, s)
            L.gb_sark_step_graph(s, c.dt, warmup)
            L.gb_ctx_synchronize(ctx)
            t0 = time.perf_counter()
            L.gb_sark_step_graph(s, c.dt, steps)
            L.gb_ctx_synchronize(ctx)
            return (time.perf_counter() - t0) / steps
        finally:
            L.gb_solver_destroy(s)
    finally:
        L.gb_mesh_destroy(mesh)
        L.gb_ctx_destroy(ctx)
