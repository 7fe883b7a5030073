"""Request loop for rate solves: continuous batching with HBM admission.

Requests arrive at any time (`Server.submit`, thread safe) and are served by
a scheduler thread:

* a request names a *scene* (sources and gas of one snapshot); the source
  tree and the gas grid of a scene are built once and stay resident in HBM
  while requests use them (least recently used scenes are evicted when the
  budget needs room);
* admission is by memory: a request is admitted when the bytes it needs (its
  scene if not resident, plus its rate call; `start_estimate_bytes`) fit in
  the budget next to everything in flight; otherwise it waits, in arrival
  order (no request overtakes an older one that fits);
* continuous batching: at every scheduler turn the admitted requests whose
  scenes are ready are packed into one batched rate call on a free slot (one
  HIP stream per slot), so requests that arrive while others run join the next
  batch and batches on different slots overlap on the GPU;
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
import threading
import time
from concurrent.futures import Future
from typing import Any, Callable, Optional

import numpy as np


@dataclasses.dataclass
class Scene:
    """Sources and gas of one snapshot (host arrays, as in workloads.Workload)."""
    key: Any
    box: Any                 # binding.Box
    src_xyz: np.ndarray
    src_lum: np.ndarray
    gas_xyz: np.ndarray
    gas_h: np.ndarray
    gas_nhi: np.ndarray
    grid_log2: int

    @property
    def n_src(self):
        return int(self.src_xyz.shape[1])

    @property
    def n_gas(self):
        return int(self.gas_xyz.shape[1])


@dataclasses.dataclass
class Request:
    scene: Scene
    tgt_xyz: np.ndarray
    self_src: Optional[np.ndarray] = None
    theta: float = 1.0
    sigma: float = 6.3e-18
    prec: str = "fp32c"
    # filled by the server
    rid: int = -1
    t_submit: float = 0.0
    t_done: float = 0.0
    future: Optional[Future] = None

    @property
    def n_t(self):
        return int(self.tgt_xyz.shape[1])


class Executor:
    """What the scheduler needs from the device."""

    n_slots = 1

    def scene_bytes(self, scene: Scene) -> int:
        raise NotImplementedError

    def request_bytes(self, req: Request) -> int:
        raise NotImplementedError

    def build_scene(self, scene: Scene) -> Any:
        raise NotImplementedError

    def free_scene(self, handle: Any) -> None:
        raise NotImplementedError

    def launch(self, slot: int, batch: list, scenes: dict) -> Any:
        raise NotImplementedError

    def done(self, token: Any) -> bool:
        raise NotImplementedError

    def results(self, token: Any) -> list:
        raise NotImplementedError


class GpuExecutor(Executor):
    """libstart on one GPU: one Context (HIP stream) per slot; scenes are
    built on slot 0's context and used from every slot (builds synchronise).

    Without autotune the library picks the tile size from the call's size.
    With autotune, the first batch of each size class (total targets and
    largest source count, each rounded up to a power of two) up to 2^17
    targets on a slot is run through
    start_autotune_rates, which computes it with several tile sizes and keeps
    the fastest for that class; later batches of the class use it (results
    do not depend on it).  This tunes on the request path, so the first
    batch of a class is slow."""

    TUNE_MAX_CLASS = 17

    def __init__(self, device: int = 0, n_slots: int = 2, autotune: bool = False):
        import torch

        from . import binding
        self.torch = torch
        self.binding = binding
        self.n_slots = n_slots
        self.ctxs = [binding.Context(device) for _ in range(n_slots)]
        self.dev = self.ctxs[0].device
        self.autotune = autotune
        self.tuned = [set() for _ in range(n_slots)]

    def _est(self, n_t, n_s, n_gas, grid_log2, prec):
        return self.binding.estimate_bytes(n_t, n_s, n_gas, grid_log2, prec)

    def scene_bytes(self, scene):
        return self._est(0, scene.n_src, scene.n_gas, scene.grid_log2, "fp64")

    def request_bytes(self, req):
        # targets on the device, output, and the rate call's scratch
        return self._est(req.n_t, 0, 0, 0, req.prec) + req.n_t * (24 + 8 + 8)

    def build_scene(self, scene):
        t = self.torch
        c = self.ctxs[0]
        d = lambda a: t.from_numpy(np.ascontiguousarray(a)).to(self.dev)  # noqa: E731
        tree = c.build_source_tree(scene.box, d(scene.src_xyz), d(scene.src_lum))
        grid = c.build_gas_grid(scene.box, d(scene.gas_xyz), d(scene.gas_h), d(scene.gas_nhi), scene.grid_log2)
        return tree, grid

    def free_scene(self, handle):
        tree, grid = handle
        tree.free()
        grid.free()

    def launch(self, slot, batch, scenes):
        t = self.torch
        ctx = self.ctxs[slot]
        items = []
        with t.cuda.stream(ctx.stream):
            for r in batch:
                tree, grid = scenes[r.scene.key]
                dt = t.float64 if r.prec == "fp64" else t.float32
                xyz = t.from_numpy(np.ascontiguousarray(r.tgt_xyz)).to(self.dev, non_blocking=False)
                ss = None if r.self_src is None else t.from_numpy(np.ascontiguousarray(r.self_src)).to(self.dev)
                out = t.empty(r.n_t, dtype=dt, device=self.dev)
                items.append(dict(tree=tree, grid=grid, tgt_xyz=xyz, self_src=ss, theta=r.theta, sigma=r.sigma,
                                  prec=r.prec, out=out))
            total = sum(r.n_t for r in batch)
            n_src = max(r.scene.n_src for r in batch)
            key = (max(0, (total - 1).bit_length()), max(0, (n_src - 1).bit_length()))
            if self.autotune and key[0] <= self.TUNE_MAX_CLASS and key not in self.tuned[slot]:
                ctx.autotune_rates(items, reps=2)
                self.tuned[slot].add(key)
            else:
                ctx.compute_rates_batched(items)
            ev = t.cuda.Event()
            ev.record(ctx.stream)
        return (ctx, ev, items)

    def done(self, token):
        return token[1].query()

    def results(self, token):
        ctx, ev, items = token
        ctx.synchronize()   # raises on device-side input errors
        return [it["out"].cpu().numpy() for it in items]


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
        self.ready: list = []          # admitted, waiting for a slot
        self.inflight: dict = {}       # slot -> (token, batch, bytes)
        self.scenes: collections.OrderedDict = collections.OrderedDict()   # key -> handle (LRU)
        self.scene_cost: dict = {}
        self.scene_users: collections.Counter = collections.Counter()
        self.used = 0                  # bytes: resident scenes + admitted requests
        self.next_id = 0
        self.completed: list = []
        self.errors: list = []
        self.stop_flag = False
        self.thread: Optional[threading.Thread] = None

    # ------------------------------------------------------------ client ---
    def submit(self, req: Request) -> Future:
        need = self.ex.request_bytes(req)
        if req.scene.key not in self.scenes:
            need += self.ex.scene_bytes(req.scene)
        if need > self.budget:
            raise ValueError(f"request needs {need} bytes, more than the whole budget {self.budget}")
        with self.lock:
            req.rid = self.next_id
            self.next_id += 1
            req.t_submit = self.clock()
            req.future = Future()
            self.pending.append(req)
            self.lock.notify()
        return req.future

    def start(self):
        self.thread = threading.Thread(target=self.run, daemon=True)
        self.thread.start()
        return self

    def stop(self, wait: bool = True):
        with self.lock:
            self.stop_flag = True
            self.lock.notify()
        if wait and self.thread is not None:
            self.thread.join()

    def drain(self, timeout: float = 600.0):
        """Waits until every submitted request has completed."""
        t0 = time.perf_counter()
        while True:
            with self.lock:
                if not self.pending and not self.ready and not self.inflight:
                    return
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError("server did not drain")
            time.sleep(0.001)

    # --------------------------------------------------------- scheduler ---
    def _admit(self):
        """Moves requests from pending to ready while they fit, oldest first."""
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
            if scene_new:
                self.scenes[r.scene.key] = self.ex.build_scene(r.scene)
                self.scene_cost[r.scene.key] = self.ex.scene_bytes(r.scene)
                self.used += self.scene_cost[r.scene.key]
            self.scenes.move_to_end(r.scene.key)
            self.scene_users[r.scene.key] += 1
            self.used += self.ex.request_bytes(r)
            self.ready.append(r)

    def _evict(self, nbytes: int) -> bool:
        """Frees unused resident scenes (least recently used first)."""
        freed = 0
        for key in list(self.scenes.keys()):
            if freed >= nbytes:
                break
            if self.scene_users[key] > 0:
                continue
            self.ex.free_scene(self.scenes.pop(key))
            cost = self.scene_cost.pop(key)
            self.used -= cost
            freed += cost
        return freed >= nbytes

    def _launch(self):
        for slot in range(self.ex.n_slots):
            if not self.ready:
                return
            if slot in self.inflight:
                continue
            batch = self.ready[: self.max_batch]
            del self.ready[: len(batch)]
            token = self.ex.launch(slot, batch, self.scenes)
            self.inflight[slot] = (token, batch)

    def _complete(self):
        for slot in list(self.inflight.keys()):
            token, batch = self.inflight[slot]
            if not self.ex.done(token):
                continue
            del self.inflight[slot]
            try:
                outs = self.ex.results(token)
                err = None
            except Exception as e:   # a failing batch fails its requests only
                outs, err = [None] * len(batch), e
            now = self.clock()
            for r, o in zip(batch, outs):
                r.t_done = now
                self.used -= self.ex.request_bytes(r)
                self.scene_users[r.scene.key] -= 1
                if err is None:
                    r.future.set_result(o)
                else:
                    self.errors.append((r.rid, err))
                    r.future.set_exception(err)
                self.completed.append(r)

    def step(self):
        """One scheduler turn (also driven directly by tests)."""
        with self.lock:
            self._complete()
            self._admit()
            self._launch()

    def run(self):
        while True:
            with self.lock:
                if self.stop_flag and not self.pending and not self.ready and not self.inflight:
                    return
                if not self.pending and not self.ready and not self.inflight:
                    self.lock.wait(timeout=0.01)
            self.step()
            with self.lock:
                busy = bool(self.inflight)
            if busy:
                time.sleep(self.idle_wait)

    # ----------------------------------------------------------- metrics ---
    def latency_stats(self):
        lat = np.array([r.t_done - r.t_submit for r in self.completed if r.t_done > 0])
        if lat.size == 0:
            return {}
        n_t = sum(r.n_t for r in self.completed)
        span = max(r.t_done for r in self.completed) - min(r.t_submit for r in self.completed)
        return {"requests": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
                "targets_per_s": float(n_t / span) if span > 0 else None, "span_s": float(span)}
