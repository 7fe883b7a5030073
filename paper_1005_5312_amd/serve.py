"""Request loop for rate solves: continuous batching with HBM admission.

Requests arrive at any time (`Server.submit`, thread safe) and are served by
a scheduler thread:

* a request names a *scene* (sources and gas of one snapshot); the source
  tree and the gas grid of a scene are built once and stay resident in HBM
  while requests use them (least recently used scenes are evicted when the
  budget needs room);
* scene builds run on a builder thread with a context (HIP stream) of its
  own, so a build never holds up the dispatch of requests whose scenes are
  already resident; a request waits for its scene's build, then joins the
  ready requests;
* admission is by memory: a request is admitted when the bytes it needs (its
  scene if not resident, plus its rate call; `start_estimate_bytes`) fit in
  the budget next to everything in flight; otherwise it waits, in arrival
  order (no request overtakes an older one that fits);
* continuous batching: at every scheduler turn the ready requests are packed
  into one batched rate call on a free slot (one HIP stream per slot), so
  requests that arrive while others run join the next batch and batches on
  different slots overlap on the GPU;
* failures stay with their request: requests are checked when submitted (a
  malformed one fails at once); a batch that fails anyway (a device-side
  input error, a launch error) is split and its requests are run one by one,
  so only the bad ones fail; a failed scene build fails the requests waiting
  for that scene; every failure releases what the request had reserved;
* a request's latency is measured from `submit` to its result being on the
  host.

Results do not depend on what a request is batched with: every target's rate
is computed from its own interaction list in a fixed order (tested bit for
bit).  The policy is written against a small executor interface so it can be
tested on the CPU with a fake executor and a fake clock.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import threading
import time
from concurrent.futures import Future
from typing import Any, Callable, Optional

import numpy as np

PRECISIONS = ("fp32c", "fp64")


@dataclasses.dataclass
class Scene:
    """Sources and gas of one snapshot (host arrays, as in workloads.Workload).
    self_src: for scenes whose particles are also sources, each particle's own
    source index (used by requests for every particle of the scene)."""
    key: Any
    box: Any                 # binding.Box
    src_xyz: np.ndarray
    src_lum: np.ndarray
    gas_xyz: np.ndarray
    gas_h: np.ndarray
    gas_nhi: np.ndarray
    grid_log2: int
    self_src: Optional[np.ndarray] = None

    @property
    def n_src(self):
        return int(self.src_xyz.shape[1])

    @property
    def n_gas(self):
        return int(self.gas_xyz.shape[1])


@dataclasses.dataclass
class Request:
    """Rates of the targets tgt_xyz [3, n] in a scene; tgt_xyz = None asks for
    every gas particle of the scene (with the scene's self_src), whose
    positions stay on the device with the scene."""
    scene: Scene
    tgt_xyz: Optional[np.ndarray] = None
    self_src: Optional[np.ndarray] = None
    theta: float = 1.0
    sigma: float = 6.3e-18
    prec: str = "fp32c"
    # filled by the server
    rid: int = -1
    t_submit: float = 0.0
    t_done: float = 0.0
    future: Optional[Future] = None
    solo: bool = False       # run alone (its batch failed once)
    cold: bool = False       # waited for its scene's build

    @property
    def n_t(self):
        return self.scene.n_gas if self.tgt_xyz is None else int(self.tgt_xyz.shape[1])


def validate_request(req: Request) -> None:
    """Raises ValueError for a request the library would refuse: unknown
    precision, theta or sigma negative or not finite, targets of the wrong
    shape, not finite or outside the scene's box, own-source indices out of
    range.  (The library checks the same on the device; this catches them
    before a batch is packed.)"""
    if req.prec not in PRECISIONS:
        raise ValueError(f"unknown precision {req.prec!r}")
    for name in ("theta", "sigma"):
        v = getattr(req, name)
        if not (isinstance(v, (int, float)) and math.isfinite(v) and v >= 0):
            raise ValueError(f"{name} must be finite and >= 0, got {v!r}")
    if req.tgt_xyz is None:
        if req.self_src is not None:
            raise ValueError("self_src is taken from the scene when tgt_xyz is None")
        return
    t = req.tgt_xyz
    if not isinstance(t, np.ndarray) or t.ndim != 2 or t.shape[0] != 3:
        raise ValueError("tgt_xyz must be a (3, n) array")
    if not np.all(np.isfinite(t)):
        raise ValueError("target positions are not finite")
    box = req.scene.box
    if box is not None and t.shape[1] > 0:
        lo = np.asarray(box.lo, dtype=np.float64)[:, None]
        if np.any(t < lo) or np.any(t > lo + float(box.size)):
            raise ValueError("a target lies outside the scene's box")
    if req.self_src is not None:
        s = np.asarray(req.self_src)
        if s.shape != (t.shape[1],) or not np.issubdtype(s.dtype, np.integer):
            raise ValueError("self_src must hold one integer per target")
        if s.size and (s.min() < -1 or s.max() >= req.scene.n_src):
            raise ValueError("self_src index out of range")


class Executor:
    """What the scheduler needs from the device.  build_scene and free_scene
    are called from the builder thread, the others from the scheduler."""

    n_slots = 1

    def scene_bytes(self, scene: Scene) -> int:
        raise NotImplementedError

    def request_bytes(self, req: Request) -> int:
        raise NotImplementedError

    def build_scene(self, scene: Scene) -> Any:
        raise NotImplementedError

    def free_scene(self, handle: Any) -> None:
        raise NotImplementedError

    def forget_scene(self, key: Any) -> None:
        """Drops what the executor keeps for a scene that is about to be freed
        (called from the scheduler thread first)."""

    def launch(self, slot: int, batch: list, scenes: dict) -> Any:
        raise NotImplementedError

    def done(self, token: Any) -> bool:
        raise NotImplementedError

    def results(self, token: Any) -> list:
        raise NotImplementedError


class GpuExecutor(Executor):
    """libstart on one GPU: one Context (HIP stream) per slot, and one more
    for the builder thread, on which scenes are built (tree and grid at the
    same time, start_build_scene) and from which every slot uses them (a build
    returns only when its data is on the device).  A scene's gas positions
    and own-source indices stay on the device with it, for requests that ask
    for every particle; other targets are uploaded through a pinned staging
    buffer per slot, asynchronously on the slot's stream.

    With plans (the default), a request for every particle of a scene is
    served from a rate plan of that slot (start_rates_plan_*: staged once,
    then replayed from a HIP graph), kept while the scene is resident; other
    requests of a batch share one batched call.

    Without autotune the library picks the tile size from the call's size.
    With autotune, the first batch of each size class (total targets and
    largest source count, each rounded up to a power of two) up to 2^17
    targets on a slot is run through start_autotune_rates, which computes it
    with several tile sizes and keeps the fastest for that class; later
    batches of the class use it (results do not depend on it).  This tunes on
    the request path, so the first batch of a class is slow."""

    TUNE_MAX_CLASS = 17

    def __init__(self, device: int = 0, n_slots: int = 2, autotune: bool = False, plans: bool = True):
        import torch

        from . import binding
        self.torch = torch
        self.binding = binding
        self.n_slots = n_slots
        self.ctxs = [binding.Context(device) for _ in range(n_slots)]
        self.build_ctx = binding.Context(device)
        self.dev = self.ctxs[0].device
        self.autotune = autotune
        self.tuned = [set() for _ in range(n_slots)]
        self.stage = [None] * n_slots    # pinned staging of targets per slot
        self.plans = plans
        self.plan_cache = [dict() for _ in range(n_slots)]   # (scene key, prec, theta, sigma) -> (plan, out)
        # A plan's creation captures its slot stream into a HIP graph; device
        # memory freed (or the device synchronised) by another thread during
        # the capture would invalidate it.  Builds and frees, which run on
        # the builder thread, and plan creation and release therefore hold
        # this lock (taken with no scheduler lock held by its other users).
        self.mm_lock = threading.Lock()

    def _est(self, n_t, n_s, n_gas, grid_log2, prec):
        return self.binding.estimate_bytes(n_t, n_s, n_gas, grid_log2, prec)

    def scene_bytes(self, scene):
        # tree, grid and the resident particle positions and own sources, and
        # the rate plans of the slots (staging, sorted targets, output)
        plans = self.n_slots * (self._est(scene.n_gas, 0, 0, 0, "fp64") + scene.n_gas * 8) if self.plans else 0
        return self._est(0, scene.n_src, scene.n_gas, scene.grid_log2, "fp64") + scene.n_gas * (24 + 8) + plans

    def request_bytes(self, req):
        # targets on the device, output, and the rate call's scratch
        return self._est(req.n_t, 0, 0, 0, req.prec) + req.n_t * (24 + 8 + 8)

    def build_scene(self, scene):
        t = self.torch
        c = self.build_ctx
        d = lambda a: t.from_numpy(np.ascontiguousarray(a)).to(self.dev)  # noqa: E731
        with self.mm_lock:
            with t.cuda.stream(c.stream):
                gas = d(scene.gas_xyz)
                ss = None if scene.self_src is None else d(np.asarray(scene.self_src, dtype=np.int64))
                tree, grid = c.build_scene(scene.box, d(scene.src_xyz), d(scene.src_lum), gas, d(scene.gas_h),
                                           d(scene.gas_nhi), scene.grid_log2)
            c.stream.synchronize()
        return tree, grid, gas, ss

    def free_scene(self, handle):
        tree, grid = handle[0], handle[1]
        with self.mm_lock:
            tree.free()
            grid.free()

    def forget_scene(self, key):
        with self.mm_lock:
            for slot, cache in enumerate(self.plan_cache):
                for k in [k for k in cache if k[0] == key]:
                    cache.pop(k)[0].free()

    def launch(self, slot, batch, scenes):
        t = self.torch
        ctx = self.ctxs[slot]
        items = []
        outs = [None] * len(batch)
        with t.cuda.stream(ctx.stream):
            uploads = [r for r in batch if r.tgt_xyz is not None]
            total_up = sum(3 * r.n_t for r in uploads)
            buf = self.stage[slot]
            if uploads and (buf is None or buf.numel() < total_up):
                buf = t.empty(max(total_up, 1 << 16), dtype=t.float64, pin_memory=True)
                self.stage[slot] = buf
            at = 0
            batched = []
            for k, r in enumerate(batch):
                tree, grid, gas, gss = scenes[r.scene.key]
                dt = t.float64 if r.prec == "fp64" else t.float32
                if r.tgt_xyz is None and self.plans:
                    key = (r.scene.key, r.prec, float(r.theta), float(r.sigma))
                    entry = self.plan_cache[slot].get(key)
                    if entry is None:   # created (and run once) on first use
                        out = t.empty(r.n_t, dtype=dt, device=self.dev)
                        with self.mm_lock:
                            plan = ctx.rates_plan([dict(tree=tree, grid=grid, tgt_xyz=gas, self_src=gss,
                                                        theta=r.theta, sigma=r.sigma, prec=r.prec, out=out)])
                        self.plan_cache[slot][key] = (plan, out)
                    else:
                        plan, out = entry
                        plan.launch()
                    outs[k] = out.to("cpu", non_blocking=True)
                    continue
                if r.tgt_xyz is None:
                    xyz, ss = gas, gss
                else:
                    m = 3 * r.n_t
                    host = buf[at: at + m]
                    host.numpy()[:] = np.ascontiguousarray(r.tgt_xyz, dtype=np.float64).reshape(-1)
                    xyz = host.to(self.dev, non_blocking=True).view(3, r.n_t)
                    at += m
                    ss = None if r.self_src is None else \
                        t.from_numpy(np.ascontiguousarray(r.self_src, dtype=np.int64)).to(self.dev)
                out = t.empty(r.n_t, dtype=dt, device=self.dev)
                items.append(dict(tree=tree, grid=grid, tgt_xyz=xyz, self_src=ss, theta=r.theta, sigma=r.sigma,
                                  prec=r.prec, out=out))
                batched.append(k)
            if items:
                total = sum(batch[k].n_t for k in batched)
                n_src = max(batch[k].scene.n_src for k in batched)
                key = (max(0, (total - 1).bit_length()), max(0, (n_src - 1).bit_length()))
                if self.autotune and key[0] <= self.TUNE_MAX_CLASS and key not in self.tuned[slot]:
                    ctx.autotune_rates(items, reps=2)
                    self.tuned[slot].add(key)
                else:
                    ctx.compute_rates_batched(items)
                for k, it in zip(batched, items):
                    outs[k] = it["out"].to("cpu", non_blocking=True)
            ev = t.cuda.Event()
            ev.record(ctx.stream)
        return (ctx, ev, items, outs)

    def done(self, token):
        return token[1].query()

    def results(self, token):
        ctx, ev, items, outs = token
        ctx.synchronize()   # raises on device-side input errors
        ev.synchronize()
        return [o.numpy() for o in outs]


_BUILDING = object()   # a scene whose build is queued or running


class Server:
    """Continuous-batching rate server (see the module docstring)."""

    def __init__(self, executor: Executor, hbm_budget: int, max_batch: int = 64,
                 clock: Callable[[], float] = time.perf_counter, idle_wait: float = 0.0005):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_batch = max_batch
        self.clock = clock
        self.idle_wait = idle_wait
        self.lock = threading.Condition()
        self.pending: collections.deque = collections.deque()   # arrival order
        self.waiting: dict = collections.defaultdict(list)      # scene key -> admitted, scene building
        self.ready: list = []          # admitted, scene resident, waiting for a slot
        self.inflight: dict = {}       # slot -> (token, batch)
        self.scenes: collections.OrderedDict = collections.OrderedDict()   # key -> handle or _BUILDING (LRU)
        self.scene_cost: dict = {}
        self.scene_users: collections.Counter = collections.Counter()
        self.used = 0                  # bytes: resident scenes + admitted requests
        self.builds = 0                # scene builds queued
        self.evictions = 0             # resident scenes freed for room
        self.next_id = 0
        self.completed: list = []
        self.errors: list = []
        self.stop_flag = False
        self.builder_stop = False
        self.thread: Optional[threading.Thread] = None
        self.builder: Optional[threading.Thread] = None
        self.jobs: collections.deque = collections.deque()      # ("build", scene) / ("free", handle)
        self.jobs_cv = threading.Condition()
        self.builds_done: collections.deque = collections.deque()   # (key, handle, error)

    # ------------------------------------------------------------ client ---
    def submit(self, req: Request) -> Future:
        """Queues a request; returns its future.  A malformed request gets a
        future that has already failed (ValueError); one larger than the whole
        budget raises ValueError."""
        need = self.ex.request_bytes(req)
        if req.scene.key not in self.scenes:
            need += self.ex.scene_bytes(req.scene)
        if need > self.budget:
            raise ValueError(f"request needs {need} bytes, more than the whole budget {self.budget}")
        try:
            validate_request(req)
            bad = None
        except ValueError as e:
            bad = e
        with self.lock:
            req.rid = self.next_id
            self.next_id += 1
            req.t_submit = self.clock()
            req.future = Future()
            if bad is not None:
                req.t_done = req.t_submit
                self.errors.append((req.rid, bad))
                req.future.set_exception(bad)
                return req.future
            self.pending.append(req)
            self.lock.notify()
        return req.future

    def start(self):
        self.builder = threading.Thread(target=self._build_loop, daemon=True)
        self.builder.start()
        self.thread = threading.Thread(target=self.run, daemon=True)
        self.thread.start()
        return self

    def stop(self, wait: bool = True):
        """Stops once every submitted request has completed (the builder
        thread last: the scheduler may still need builds)."""
        with self.lock:
            self.stop_flag = True
            self.lock.notify()
        if not wait:
            return
        if self.thread is not None:
            self.thread.join()
        with self.jobs_cv:
            self.builder_stop = True
            self.jobs_cv.notify()
        if self.builder is not None:
            self.builder.join()

    def close(self):
        """Stops the server and frees every resident scene."""
        self.stop()
        with self.lock:
            for key in list(self.scenes.keys()):
                self.ex.forget_scene(key)
            handles = [h for h in self.scenes.values() if h is not _BUILDING]
            self.scenes.clear()
            self.scene_cost.clear()
        for h in handles:
            self.ex.free_scene(h)
        self.used = sum(self.ex.request_bytes(r) for r in self.ready)

    def drain(self, timeout: float = 600.0):
        """Waits until every submitted request has completed."""
        t0 = time.perf_counter()
        while True:
            with self.lock:
                if self._idle():
                    return
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError("server did not drain")
            time.sleep(0.001)

    def _idle(self):
        return not self.pending and not self.ready and not self.inflight and not any(self.waiting.values())

    # ----------------------------------------------------------- builder ---
    def _queue_job(self, job):
        with self.jobs_cv:
            self.jobs.append(job)
            self.jobs_cv.notify()

    def _run_job(self, job):
        kind, arg = job
        if kind == "free":
            try:
                self.ex.free_scene(arg)
            except Exception as e:   # nothing waits for a free: record it
                self.errors.append((None, e))
            return
        try:
            handle, err = self.ex.build_scene(arg), None
        except Exception as e:
            handle, err = None, e
        with self.lock:
            self.builds_done.append((arg.key, handle, err))
            self.lock.notify()

    def _build_loop(self):
        while True:
            with self.jobs_cv:
                while not self.jobs and not self.builder_stop:
                    self.jobs_cv.wait(timeout=0.05)
                if not self.jobs:
                    return
                job = self.jobs.popleft()
            self._run_job(job)

    def _pump_jobs(self):
        """Without a builder thread (step() driven directly, as in tests) the
        queued builds and frees run here, at the start of a turn."""
        if self.builder is not None:
            return
        while True:
            with self.jobs_cv:
                if not self.jobs:
                    return
                job = self.jobs.popleft()
            self._run_job(job)

    # --------------------------------------------------------- scheduler ---
    def _release(self, r, err):
        """A request fails: its reservation is returned and its future set."""
        r.t_done = self.clock()
        self.used -= self.ex.request_bytes(r)
        self.scene_users[r.scene.key] -= 1
        self.errors.append((r.rid, err))
        r.future.set_exception(err)
        self.completed.append(r)

    def _finish_builds(self):
        while self.builds_done:
            key, handle, err = self.builds_done.popleft()
            reqs = self.waiting.pop(key, [])
            if err is None:
                self.scenes[key] = handle
                self.ready.extend(reqs)
                continue
            # the build failed: the scene is dropped with its reservation and
            # the requests that waited for it fail
            self.scenes.pop(key, None)
            self.used -= self.scene_cost.pop(key, 0)
            for r in reqs:
                self._release(r, err)

    def _admit(self):
        """Moves requests from pending to ready (or to the wait for their
        scene's build) while they fit, oldest first."""
        while self.pending:
            r = self.pending[0]
            need = self.ex.request_bytes(r)
            scene_new = r.scene.key not in self.scenes
            if scene_new:
                need += self.ex.scene_bytes(r.scene)
            if self.used + need > self.budget:
                if not self._evict(self.used + need - self.budget):
                    return   # the oldest waits; nobody overtakes it
                continue
            self.pending.popleft()
            key = r.scene.key
            if scene_new:
                self.scenes[key] = _BUILDING
                self.scene_cost[key] = self.ex.scene_bytes(r.scene)
                self.used += self.scene_cost[key]
                self._queue_job(("build", r.scene))
                self.builds += 1
            self.scenes.move_to_end(key)
            self.scene_users[key] += 1
            self.used += self.ex.request_bytes(r)
            if self.scenes[key] is _BUILDING:
                r.cold = True
                self.waiting[key].append(r)
            else:
                self.ready.append(r)

    def _evict(self, nbytes: int) -> bool:
        """Frees unused resident scenes (least recently used first)."""
        freed = 0
        for key in list(self.scenes.keys()):
            if freed >= nbytes:
                break
            if self.scene_users[key] > 0 or self.scenes[key] is _BUILDING:
                continue
            self.ex.forget_scene(key)
            self._queue_job(("free", self.scenes.pop(key)))
            self.evictions += 1
            cost = self.scene_cost.pop(key)
            self.used -= cost
            freed += cost
        return freed >= nbytes

    def _next_batch(self):
        if self.ready[0].solo:
            return [self.ready.pop(0)]
        k = 0
        while k < len(self.ready) and k < self.max_batch and not self.ready[k].solo:
            k += 1
        batch = self.ready[:k]
        del self.ready[:k]
        return batch

    def _split_or_fail(self, batch, err):
        """A failed batch: each request is tried again on its own (ahead of
        the others, in order); a request that failed alone fails."""
        if len(batch) > 1:
            for r in batch:
                r.solo = True
            self.ready[:0] = batch
            return
        self._release(batch[0], err)

    def _launch(self):
        for slot in range(self.ex.n_slots):
            if not self.ready:
                return
            if slot in self.inflight:
                continue
            batch = self._next_batch()
            try:
                token = self.ex.launch(slot, batch, self.scenes)
            except Exception as e:
                self._split_or_fail(batch, e)
                continue
            self.inflight[slot] = (token, batch)

    def _complete(self):
        for slot in list(self.inflight.keys()):
            token, batch = self.inflight[slot]
            try:
                if not self.ex.done(token):
                    continue
                outs = self.ex.results(token)
                err = None
            except Exception as e:
                outs, err = None, e
            del self.inflight[slot]
            if err is not None:
                self._split_or_fail(batch, err)
                continue
            now = self.clock()
            for r, o in zip(batch, outs):
                r.t_done = now
                self.used -= self.ex.request_bytes(r)
                self.scene_users[r.scene.key] -= 1
                r.future.set_result(o)
                self.completed.append(r)

    def step(self):
        """One scheduler turn (also driven directly by tests, where the builds
        that the turn queues run inline before its launches)."""
        self._pump_jobs()
        with self.lock:
            self._finish_builds()
            self._complete()
            self._admit()
        self._pump_jobs()
        with self.lock:
            self._finish_builds()
            self._launch()

    def run(self):
        while True:
            with self.lock:
                if self.stop_flag and self._idle():
                    return
                if not self.pending and not self.ready and not self.inflight and not self.builds_done:
                    self.lock.wait(timeout=0.01)
            self.step()
            with self.lock:
                busy = bool(self.inflight)
            if busy:
                time.sleep(self.idle_wait)

    # ----------------------------------------------------------- metrics ---
    def latency_stats(self):
        ok = [r for r in self.completed if r.t_done > 0 and r.future.exception() is None]
        lat = np.array([r.t_done - r.t_submit for r in ok])
        if lat.size == 0:
            return {}
        n_t = sum(r.n_t for r in ok)
        span = max(r.t_done for r in ok) - min(r.t_submit for r in ok)
        out = {"requests": int(lat.size), "failed": len(self.completed) - len(ok),
               "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
               "mean_ms": float(lat.mean() * 1e3),
               "targets_per_s": float(n_t / span) if span > 0 else None, "span_s": float(span)}
        for name, sel in (("warm", [not r.cold for r in ok]), ("cold", [r.cold for r in ok])):
            v = lat[np.array(sel, dtype=bool)]
            if v.size:
                out[name] = {"requests": int(v.size), "p50_ms": float(np.percentile(v, 50) * 1e3),
                             "p99_ms": float(np.percentile(v, 99) * 1e3)}
        return out
