#!/usr/bin/env python3
"""Throughput of the START photoionization-rate path on one MI355X.

One step = the whole hot path over one synthetic snapshot, inputs resident
in HBM: source octree (Morton keys, radix sort, cells, virtual-source
moments), neutral-hydrogen grid, target ordering, and the tree walk with ray
marches that produces Gamma for every particle.  value = particles / step time.

Also measured in the same run: the rate call alone with tree and grid
resident (FP32C and FP64), the walk kernel's duration from HIP events on the
library's stream (roofline: the algorithmic byte model against the HBM peak,
the bound and issue fractions from the committed counter summaries), the
CPU FP64 oracle on the whole workload (cpu_baseline), and the other
configurations: batching and rate plans, the served request mix, the
opening-angle sweep, the shadowing configuration, the equilibrium loops,
H2 photodissociation and the upstream-particle chain.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload diffuse]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CUS, CLOCK_HZ = 256, 2.4e9          # MI355X compute units and peak engine clock
METRIC = "particle-rate evals/s at θ_crit=1 (FP32 vs FP64 GPU); serve p50/p99 latency"
WORKLOAD_TEXT = {
    "diffuse": "diffuse recombination: N_p = 2^20 emitting SPH particles + central 1e50/s star "
               "(N_s = 2^20 + 1), HII sphere r = 0.3 box, theta_crit = 1, G = 128",
    "shadow": "shadowing: N_p = 2^21 emitters + 1e50/s star, 16 clumps (200x, r = 0.05 box), theta_crit = 1, G = 128",
    "clumpy": "clumpy: N_p = 2^18 lognormal medium, N_s = 1024 log-uniform sources, theta_crit = 1, G = 64",
    "small": "small: N_p = 4096 uniform neutral medium, N_s = 16, theta_crit = 1, G = 16",
}
# algorithmic bytes per target (FP32C and FP64): target position + Gamma,
# per opening test (cell key|level 8 B + subtree link 4 B), per entry
# (centre + luminosity), per grid cell crossed (one density value)
BYTES = {"fp32c": dict(base=24 + 4, test=12, entry=16, cell=4),
         "fp64": dict(base=24 + 8, test=12, entry=32, cell=8)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(counters, prec):
    b = BYTES[prec]
    c = counters.sum(axis=0).astype(np.float64)
    n = counters.shape[0]
    return b["base"] * n + b["test"] * c[0] + b["entry"] * c[1] + b["cell"] * c[2]


def source_sha():
    """Hash of the sources the rate kernel is compiled from (a profile taken
    on other sources no longer describes it)."""
    h = hashlib.sha256()
    for name in ("internal.h", "rates.hip"):
        with open(os.path.join(ROOT, "paper_1005_5312_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload, prec, sha):
    """HBM bytes per walk launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"rates_kernel_{prec}_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha") != sha:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def counters_from_profiles(workload, prec, sha):
    """SQ and L1 counters per walk launch from the committed rocprofv3 summary,
    if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"rates_kernel_{prec}_{workload}_sq_tcp_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha") != sha:
        return None
    try:
        return {k: float(v) for k, v in vals.items() if not k.endswith("source_sha")}
    except ValueError:
        return None


def cpu_baseline(w):
    """The CPU FP64 oracle on this host, on the whole benchmark workload: tree,
    grid and the rates of every target, on the threads this process is given
    (OMP_NUM_THREADS when set, else every core in its affinity mask)."""
    from oracle import oracle as O
    n_aff = len(os.sched_getaffinity(0))
    threads = n_aff
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        threads = min(threads, int(env))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    box = O.make_box(w.box_lo, w.box_size, w.length_unit_cm)
    t0 = time.perf_counter()
    tree = O.Tree(box, w.src_xyz, w.src_lum)
    t1 = time.perf_counter()
    grid = O.grid(box, w.gas_xyz, w.gas_h, w.gas_nhi, w.grid_log2)
    t2 = time.perf_counter()
    O.rates(tree, w.grid_log2, grid, w.tgt_xyz, w.self_src, 1.0, w.sigma, nthreads=threads)
    t3 = time.perf_counter()
    step = t3 - t0
    return {"value": w.n_tgt / step, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole workload: FP64 oracle, {threads} threads, tree ({t1 - t0:.2f} s), grid "
                      f"({t2 - t1:.2f} s) and the rates of all {w.n_tgt} targets ({t3 - t2:.2f} s) = {step:.1f} s",
            "rates_only_evals_per_s": w.n_tgt / (t3 - t2), "cpu_model": model, "nproc": os.cpu_count(),
            "affinity_cpus": n_aff, "omp_num_threads_env": env or None}


def make_scene_pool(n, seed, lo_log2=14, hi_log2=17):
    """Scenes shaped like the served workload: N_p log-uniform, N_s in
    {1, 64, N_p}, medium from one of the small / clumpy / diffuse generators."""
    from paper_1005_5312_amd import serve
    from paper_1005_5312_amd import workloads as W
    rng = np.random.default_rng(seed)
    pool = []
    for k in range(n):
        n_p = int(round(2 ** rng.uniform(lo_log2, hi_log2)))
        kind = ("small", "clumpy", "diffuse")[k % 3]
        ns_kind = ("one", "64", "all")[(k // 3) % 3]
        s = int(rng.integers(1 << 30))
        if kind == "diffuse":
            w = W.make_diffuse(seed=s, n_gas=n_p)
            if ns_kind != "all":   # keep the star plus a few emitters
                m = 1 if ns_kind == "one" else 64
                keep = np.concatenate([rng.choice(n_p, size=m - 1, replace=False), [n_p]]) if m > 1 else [n_p]
                w.src_xyz = np.ascontiguousarray(w.src_xyz[:, keep])
                w.src_lum = np.ascontiguousarray(w.src_lum[keep])
                w.self_src = None
        else:
            n_s = 1 if ns_kind == "one" else (64 if ns_kind == "64" else n_p)
            w = (W.make_small if kind == "small" else W.make_clumpy)(seed=s, n_gas=n_p, n_src=n_s)
        box_t = tuple(float(v) for v in w.box_lo)
        from paper_1005_5312_amd import Box
        pool.append((serve.Scene(("scene", k), Box(box_t, float(w.box_size), float(w.length_unit_cm)), w.src_xyz,
                                 w.src_lum, w.gas_xyz, w.gas_h, w.gas_nhi, w.grid_log2), w))
    return pool


def make_serve_pool(n_scenes, seed, lo_log2=14, hi_log2=21):
    """Scenes of the served mix: N_p = round(2^U[lo, hi]) particles, N_s drawn
    from {1, 64, N_p}, the medium from the small / clumpy / diffuse generators
    (uniform choices), every particle a target.  Diffuse scenes with N_s = N_p
    keep all emitters (and the star; own sources excluded), with N_s = 1 or 64
    the star and 63 emitters."""
    from paper_1005_5312_amd import Box, serve
    from paper_1005_5312_amd import workloads as W
    rng = np.random.default_rng(seed)
    pool = []
    for k in range(n_scenes):
        n_p = int(round(2 ** rng.uniform(lo_log2, hi_log2)))
        kind = ("small", "clumpy", "diffuse")[int(rng.integers(3))]
        ns_kind = ("one", "64", "all")[int(rng.integers(3))]
        s = int(rng.integers(1 << 30))
        if kind == "diffuse":
            w = W.make_diffuse(seed=s, n_gas=n_p)
            if ns_kind != "all":
                m = 1 if ns_kind == "one" else 64
                keep = np.concatenate([rng.choice(n_p, size=m - 1, replace=False), [n_p]]) if m > 1 else [n_p]
                w.src_xyz = np.ascontiguousarray(w.src_xyz[:, keep])
                w.src_lum = np.ascontiguousarray(w.src_lum[keep])
                w.self_src = None
        else:
            n_s = 1 if ns_kind == "one" else (64 if ns_kind == "64" else n_p)
            w = (W.make_small if kind == "small" else W.make_clumpy)(seed=s, n_gas=n_p, n_src=n_s)
        box = Box(tuple(float(v) for v in w.box_lo), float(w.box_size), float(w.length_unit_cm))
        pool.append(serve.Scene(("scene", k, kind, ns_kind), box, w.src_xyz, w.src_lum, w.gas_xyz, w.gas_h,
                                w.gas_nhi, w.grid_log2, self_src=w.self_src))
    return pool


def serve_bench(rates, window_s=15.0, max_requests=2000, n_scenes=32, seed=5, autotune=False, log_fn=None):
    """The served workload: Poisson arrivals at each rate in `rates` (requests
    per second), each request the rates of every particle of a scene drawn
    uniformly from a pool of n_scenes (make_serve_pool), FP32C, theta = 1.
    Every rate starts with no scene resident; the HBM budget holds the whole
    pool, so a scene is built on its first request and stays resident (those
    first requests are reported as "cold").  Requests per rate: min(
    max_requests, rate x window_s).  Latency from submit to the result on the
    host.  One more run at the lowest rate with a budget of half the pool
    shows the cost of evicting and rebuilding scenes."""
    import threading
    from paper_1005_5312_amd import serve
    t_pool = time.perf_counter()
    pool = make_serve_pool(n_scenes, seed)
    t_pool = time.perf_counter() - t_pool
    ex = serve.GpuExecutor(0, n_slots=2, autotune=autotune)
    sb = [ex.scene_bytes(sc) for sc in pool]
    rb = [ex.request_bytes(serve.Request(sc, None)) for sc in pool]
    budget = int(1.25 * (sum(sb) + 32 * max(rb)))
    small_budget = int(max(1.2 * (max(sb) + 4 * max(rb)), 0.5 * sum(sb)))
    rng = np.random.default_rng(seed + 1)

    def run(lam, bud):
        n_req = int(min(max_requests, max(20, round(lam * window_s))))
        if log_fn:
            log_fn(f"[bench] serving: Poisson arrivals at {lam}/s, {n_req} requests, budget {bud / 2**30:.2f} GiB")
        srv = serve.Server(ex, hbm_budget=bud, max_batch=32).start()
        gaps = rng.exponential(1.0 / lam, n_req)
        picks = rng.integers(0, len(pool), n_req)
        futs = []

        def client():
            t0 = time.perf_counter()
            at = 0.0
            for g, k in zip(gaps, picks):
                at += g
                d = t0 + at - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                futs.append(srv.submit(serve.Request(pool[k], None, theta=1.0, sigma=6.3e-18, prec="fp32c")))

        th = threading.Thread(target=client)
        th.start()
        th.join()
        errors = []
        for f in futs:
            try:
                f.result(timeout=600)
            except Exception as e:   # a failed request is counted, not fatal to the run
                errors.append(repr(e))
        srv.drain()
        srv.close()
        st = srv.latency_stats()
        rps = st["requests"] / st["span_s"] if st.get("span_s") else None
        st.update({"arrival_rate_per_s": lam, "requests_asked": n_req, "requests_per_s": rps,
                   "saturated": bool(rps is not None and rps < 0.9 * lam),
                   "scene_builds": srv.builds, "scene_evictions": srv.evictions, "hbm_budget_bytes": bud,
                   "failed_requests": len(errors), "first_error": errors[0] if errors else None})
        return st

    out = [run(lam, budget) for lam in rates]
    evict = run(min(rates), small_budget) if rates else None
    sizes = sorted(sc.n_gas for sc in pool)
    return {"workload": f"{n_scenes} scenes, N_p = round(2^U[14,21]) ({sizes[0]}-{sizes[-1]}), N_s from "
                        "{1, 64, N_p}, medium from the small / clumpy / diffuse generators; every particle a "
                        "target; FP32C, theta = 1; each request draws its scene uniformly",
            "pool_scene_bytes": int(sum(sb)), "pool_targets": int(sum(sizes)), "pool_build_host_s": t_pool,
            "slots": 2, "max_batch": 32, "autotuned_tiles": autotune, "by_rate": out,
            "half_pool_budget": evict}


def batch_bench(n_inst=256, n_p=1 << 14, seed=9, reps=3):
    """n_inst instances of n_p targets in one batched call vs one call each."""
    import torch
    import paper_1005_5312_amd as S
    pool = make_scene_pool(8, seed, lo_log2=14, hi_log2=14)
    ctx = S.Context(0)
    dev = torch.device("cuda", 0)
    built = []
    for sc, w in pool:
        d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
        tree = ctx.build_source_tree(sc.box, d(w.src_xyz), d(w.src_lum))
        grid = ctx.build_gas_grid(sc.box, d(w.gas_xyz), d(w.gas_h), d(w.gas_nhi), w.grid_log2)
        built.append((tree, grid, d(w.tgt_xyz), None if w.self_src is None else d(w.self_src), w))
    items = []
    for k in range(n_inst):
        tree, grid, tgt, ss, w = built[k % len(built)]
        items.append(dict(tree=tree, grid=grid, tgt_xyz=tgt, self_src=ss, theta=1.0, sigma=w.sigma, prec="fp32c",
                          out=torch.empty(w.n_tgt, dtype=torch.float32, device=dev)))
    ctx.compute_rates_batched(items)
    ctx.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.compute_rates_batched(items)
    ctx.synchronize()
    t_batched = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        for it in items:
            ctx.compute_rates_raw(it["tree"], it["grid"], it["tgt_xyz"], it["self_src"], 1.0, it["sigma"], "fp32c",
                                  it["out"])
    ctx.synchronize()
    t_single = (time.perf_counter() - t0) / reps
    # autotuned tiles: the whole batch, and one instance (its own size class)
    best_batch, _ = ctx.autotune_rates(items, reps=3)
    best_single, _ = ctx.autotune_rates(items[:1], reps=5)
    ctx.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.compute_rates_batched(items)
    ctx.synchronize()
    t_batched_tuned = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        for it in items:
            ctx.compute_rates_raw(it["tree"], it["grid"], it["tgt_xyz"], it["self_src"], 1.0, it["sigma"], "fp32c",
                                  it["out"])
    ctx.synchronize()
    t_single_tuned = (time.perf_counter() - t0) / reps
    n_total = sum(it["tgt_xyz"].shape[1] for it in items)
    # the same batch staged once and replayed from a HIP graph (a rate plan),
    # and one instance alone, plain call against its plan
    plan = ctx.rates_plan(items)
    ctx.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.launch()
    ctx.synchronize()
    t_plan = (time.perf_counter() - t0) / reps
    plan.free()
    one = items[:1]
    plan1 = ctx.rates_plan(one)
    k1 = 50
    ctx.synchronize()
    t0 = time.perf_counter()
    for _ in range(k1):
        ctx.compute_rates_batched(one)
    ctx.synchronize()
    t_one = (time.perf_counter() - t0) / k1
    t0 = time.perf_counter()
    for _ in range(k1):
        plan1.launch()
    ctx.synchronize()
    t_one_plan = (time.perf_counter() - t0) / k1
    plan1.free()
    # the same batch in plain FP64 (same lists and rays, FP64 grid and sums)
    items64 = [dict(it, prec="fp64", out=torch.empty(it["out"].numel(), dtype=torch.float64, device=dev))
               for it in items]
    ctx.compute_rates_batched(items64)
    ctx.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.compute_rates_batched(items64)
    ctx.synchronize()
    t_batched64 = (time.perf_counter() - t0) / reps
    for tree, grid, *_ in built:
        tree.free()
        grid.free()
    ctx.close()
    return {"instances": n_inst, "targets_each": n_p, "batched_ms": t_batched * 1e3,
            "one_call_each_ms": t_single * 1e3, "batched_evals_per_s": n_total / t_batched,
            "one_call_each_evals_per_s": n_total / t_single,
            "batched_fp64_ms": t_batched64 * 1e3, "batched_fp64_evals_per_s": n_total / t_batched64,
            "autotuned": {"batch_tile_targets": best_batch, "batched_ms": t_batched_tuned * 1e3,
                          "batched_evals_per_s": n_total / t_batched_tuned,
                          "single_tile_targets": best_single, "one_call_each_ms": t_single_tuned * 1e3,
                          "one_call_each_evals_per_s": n_total / t_single_tuned},
            "default_tiles": "from the call size: about total targets / 4096, a power of two in [1, 64]",
            "plan_replay": {"batched_ms": t_plan * 1e3, "one_instance_call_ms": t_one * 1e3,
                            "one_instance_plan_ms": t_one_plan * 1e3,
                            "what": "the batch (and one 2^14 instance) staged once and its rate kernels replayed "
                                    "from a HIP graph, against the plain call (host staging, target sort, launch)"}}


def equilibrium_bench(n_gas=1 << 21, grid_log2=7, tol=1e-4, max_iter=200):
    """Photoionisation equilibrium around one source (Test 4 setting) by the
    library's fixed-point loop, in both precisions: iterations, time, and the
    ionised radius against the Stromgren radius of eq. (17)."""
    import torch
    import paper_1005_5312_amd as S
    from paper_1005_5312_amd import workloads as W
    e = W.make_stromgren(n_gas=n_gas, grid_log2=grid_log2)
    w = e.work
    ctx = S.Context(0)
    dev = torch.device("cuda", 0)
    box = S.Box(tuple(float(v) for v in w.box_lo), float(w.box_size), float(w.length_unit_cm))
    tree = ctx.build_source_tree(box, torch.from_numpy(w.src_xyz).to(dev), torch.from_numpy(w.src_lum).to(dev))
    xyz = torch.from_numpy(w.gas_xyz).to(dev)
    h = torch.from_numpy(w.gas_h).to(dev)
    nh = torch.from_numpy(e.n_h).to(dev)
    x0 = torch.from_numpy(e.x_init).to(dev)
    out = {"workload": f"Test 4: one 5e48 photons/s source at the centre of a {w.box_size} kpc box, "
                       f"uniform n_H = 1e-3, {n_gas} particles, G = {1 << grid_log2}",
           "stromgren_radius_kpc": e.stromgren_radius_cm(1e-3) / W.KPC_CM}
    for prec in ("fp32c", "fp64"):
        ctx.ionization_equilibrium(tree, xyz, h, nh, x0, grid_log2, 1.0, w.sigma, e.alpha_b, prec, 2, 0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, gam, it, ch = ctx.ionization_equilibrium(tree, xyz, h, nh, x0, grid_log2, 1.0, w.sigma, e.alpha_b, prec,
                                                    max_iter, tol)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        xn, gn = x.cpu().numpy(), gam.cpu().numpy().astype(np.float64)
        # radius of the sphere with the ionised volume sum (1 - x) V, and the
        # photoionisations per second sum x n_H Gamma V over the source rate
        r_ion = (3.0 * float(np.sum((1.0 - xn) * e.volume_cm3)) / (4.0 * np.pi)) ** (1.0 / 3.0)
        ph = float(np.sum(xn * e.n_h * gn * e.volume_cm3)) / float(w.src_lum.sum())
        out[prec] = {"iterations": it, "last_change": ch, "ms_total": dt * 1e3, "ms_per_iteration": dt * 1e3 / it,
                     "particle_updates_per_s": n_gas * it / dt, "ionised_radius_kpc": r_ion / W.KPC_CM,
                     "photoionisations_over_source_rate": ph}
        log(f"[bench] equilibrium {prec}: {it} iterations, {dt * 1e3:.1f} ms")
    tree.free()
    # with the transfer of recombination photons (every particle an emitter,
    # the tree rebuilt every iteration), against on the spot, at 2^18 / G = 64
    e2 = W.make_stromgren(n_gas=1 << 18, grid_log2=6)
    w2 = e2.work
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xd, _, itd, chd = ctx.diffuse_equilibrium(box, w2.gas_xyz, w2.gas_h, e2.n_h, e2.volume_cm3, w2.src_xyz,
                                              w2.src_lum, e2.x_init, 6, 1.0, w2.sigma, 4.18e-13, 1.58e-13, "fp32c",
                                              max_iter, 1e-3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tree2 = ctx.build_source_tree(box, torch.from_numpy(w2.src_xyz).to(dev), torch.from_numpy(w2.src_lum).to(dev))
    xo, _, ito, _ = ctx.ionization_equilibrium(tree2, w2.gas_xyz, w2.gas_h, e2.n_h, e2.x_init, 6, 1.0, w2.sigma,
                                               e2.alpha_b, "fp32c", max_iter, 1e-3)
    tree2.free()
    rad = lambda x: (3.0 * float(np.sum((1.0 - x.cpu().numpy()) * e2.volume_cm3)) / (4.0 * np.pi)) ** (1 / 3) \
        / W.KPC_CM  # noqa: E731
    out["with_recombination_photons"] = {
        "workload": f"{1 << 18} particles, G = 64, every particle an emitter (alpha_1 = 1.58e-13), FP32C",
        "iterations": itd, "last_change": chd, "ms_total": dt * 1e3, "ms_per_iteration": dt * 1e3 / itd,
        "ionised_radius_kpc": rad(xd), "on_the_spot_ionised_radius_kpc": rad(xo), "on_the_spot_iterations": ito}
    log(f"[bench] equilibrium with recombination photons: {itd} iterations, {dt * 1e3:.1f} ms")
    ctx.close()
    return out


def k_ion_bench(ctx, w, gamma32, reps=200):
    """The per-particle terms of the transfer of recombination photons on the
    benchmark workload: emission and k_self (eqs. 19, 28, 30) and the total
    k_ion of eq. (25) from the FP32C rates.  The C-ABI is called directly on
    preallocated buffers, event-timed on the library stream, against the HBM
    peak (the kernels stream 40 B and 36 B per particle)."""
    import ctypes
    import torch
    from paper_1005_5312_amd import binding as B
    dev = torch.device("cuda", 0)
    n = w.n_gas
    nh = torch.full((n,), 1e-3, dtype=torch.float64, device=dev)
    x = torch.from_numpy(np.ascontiguousarray(w.gas_nhi / 1e-3)).to(dev)
    vol = torch.full((n,), (w.box_size * w.length_unit_cm) ** 3 / n, dtype=torch.float64, device=dev)
    lum = torch.empty(n, dtype=torch.float64, device=dev)
    ks = torch.empty(n, dtype=torch.float64, device=dev)
    kion = torch.empty(n, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    L = B.lib()
    calls = (
        ("recombination_emission", 40,
         lambda: L.start_recombination_emission(ctx._h, n, p(nh), p(x), p(vol), w.sigma, 1.58e-13, p(lum), p(ks))),
        ("total_ionization", 36,
         lambda: L.start_total_ionization(ctx._h, n, p(nh), p(x), p(gamma32), B.FP32C, p(ks), p(kion))))
    out = {}
    for name, nbytes, fn in calls:
        assert fn() == 0
        ctx.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(reps):
            fn()
        e1.record(ctx.stream)
        ctx.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = nbytes * n / (ms * 1e-3) / 1e9
        out[name] = {"ms": ms, "bytes_per_particle": nbytes, "achieved_GBs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
    return out


def lw_bench(n_gas=1 << 20, n_src=1024, reps=5):
    """H2 photodissociation rates (Appendix B) for every particle of a 2^20
    lognormal medium lit by 1024 Lyman-Werner sources at theta = 1."""
    import torch
    import paper_1005_5312_amd as S
    from paper_1005_5312_amd import workloads as W
    w = W.make_lw(n_gas=n_gas, n_src=n_src)
    ctx = S.Context(0)
    dev = torch.device("cuda", 0)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    box = S.Box(tuple(float(v) for v in w.box_lo), float(w.box_size), float(w.length_unit_cm))
    tree = ctx.build_source_tree(box, d(w.src_xyz), d(w.src_lum))
    grid = ctx.build_gas_grid(box, d(w.gas_xyz), d(w.gas_h), d(w.gas_nh2), w.grid_log2)
    tgt = d(w.tgt_xyz)
    out = {"workload": f"{n_gas} particles, lognormal n_H, H2 fraction 10^U[-7,-3], {n_src} sources, "
                       f"G = {1 << w.grid_log2}, theta = 1"}
    for prec in ("fp32c", "fp64"):
        ctx.compute_dissociation_rates(tree, grid, tgt, None, 1.0, prec)
        ctx.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(reps):
            ctx.compute_dissociation_rates(tree, grid, tgt, None, 1.0, prec)
        e1.record(ctx.stream)
        ctx.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[prec] = {"ms_per_call": ms, "evals_per_s": n_gas / (ms * 1e-3)}
        log(f"[bench] H2 dissociation {prec}: {ms:.3f} ms/call")
    tree.free()
    grid.free()
    ctx.close()
    return out


def upstream_bench(reps=3):
    """Rates with the upstream-particle chain optical depths (section 2.2.1)
    on the clumpy medium (2^18 particles, 1024 sources, theta = 1), against
    the ray-integrated rates of the same lists."""
    import torch
    import paper_1005_5312_amd as S
    from paper_1005_5312_amd import workloads as W
    w = W.make_clumpy()
    ctx = S.Context(0)
    dev = torch.device("cuda", 0)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    box = S.Box(tuple(float(v) for v in w.box_lo), float(w.box_size), float(w.length_unit_cm))
    tree = ctx.build_source_tree(box, d(w.src_xyz), d(w.src_lum))
    grid = ctx.build_gas_grid(box, d(w.gas_xyz), d(w.gas_h), d(w.gas_nhi), w.grid_log2)
    xyz, h, nhi = d(w.gas_xyz), d(w.gas_h), d(w.gas_nhi)
    g, offs, _, roots = ctx.compute_rates_upstream(tree, grid, xyz, h, nhi, None, 1.0, w.sigma, structure=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g = ctx.compute_rates_upstream(tree, grid, xyz, h, nhi, None, 1.0, w.sigma)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    ray = ctx.compute_rates(tree, grid, xyz, None, 1.0, w.sigma, "fp64")
    r = np.abs(np.log(g.cpu().numpy() / ray.cpu().numpy()))
    out = {"workload": f"{w.n_gas} particles (lognormal, i.i.d.), {w.n_src} sources, theta = 1",
           "ms_per_call": ms, "evals_per_s": w.n_gas / (ms * 1e-3), "pairs": int(offs[-1]),
           "pairs_integrated_along_ray": int(roots),
           "abs_ln_ratio_to_ray_integral": {"median": float(np.median(r)), "p90": float(np.percentile(r, 90))}}
    log(f"[bench] upstream chain: {ms:.1f} ms per call, {int(offs[-1])} pairs")
    tree.free()
    grid.free()
    ctx.close()
    return out


def _rel_stats(got, ref, floor=1e-30):
    """Relative-error statistics above the Gamma floor, and the largest
    absolute difference below it."""
    big = ref >= floor
    rel = np.abs(got[big] - ref[big]) / ref[big]
    small = np.abs(got[~big] - ref[~big])
    return {"n_above_floor": int(big.sum()), "median": float(np.median(rel)) if rel.size else 0.0,
            "p99": float(np.percentile(rel, 99)) if rel.size else 0.0,
            "p99_9": float(np.percentile(rel, 99.9)) if rel.size else 0.0,
            "max": float(rel.max()) if rel.size else 0.0,
            "max_abs_below_floor": float(small.max()) if small.size else 0.0}


def tree_error_bench(ctx, w, tree, grid, n_sample=1024, seed=23):
    """The tree approximation on the bench workload: theta = 1 in both
    precisions against theta = 0 (every source on its own: the exact sum
    over sources on the same grid), on a seeded sample of targets."""
    import torch
    from paper_1005_5312_amd import workloads as W
    dev = torch.device("cuda", 0)
    idx = W.sample_indices(w.n_tgt, n_sample, seed)
    tgt = torch.from_numpy(np.ascontiguousarray(w.tgt_xyz[:, idx])).to(dev)
    ss = None if w.self_src is None else torch.from_numpy(np.ascontiguousarray(w.self_src[idx])).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g0 = ctx.compute_rates(tree, grid, tgt, ss, 0.0, w.sigma, "fp64").cpu().numpy()
    ms0 = (time.perf_counter() - t0) * 1e3
    g64 = ctx.compute_rates(tree, grid, tgt, ss, 1.0, w.sigma, "fp64").cpu().numpy()
    g32 = ctx.compute_rates(tree, grid, tgt, ss, 1.0, w.sigma, "fp32c").cpu().numpy().astype(np.float64)
    log(f"[bench] theta 1 vs theta 0 on {n_sample} targets: fp64 median rel "
        f"{_rel_stats(g64, g0)['median']:.2e}")
    return {"sample_targets": n_sample, "theta0_ms": ms0, "fp64_theta1_vs_theta0": _rel_stats(g64, g0),
            "fp32c_theta1_vs_theta0": _rel_stats(g32, g0)}


def copy_bandwidth(reps=5):
    """Achievable HBM bandwidth on this device: a plain 1 GiB device-to-device
    copy (1 GiB read + 1 GiB written per copy), event-timed on the stream it
    runs on."""
    import torch
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2.0 * a.numel() * a.element_size() / (ms * 1e-3) / 1e9
    del a, b
    return gbs


def kernel_lum_bench(ctx, w, grid, theta, reps=3):
    """Kernel-weighted virtual-source luminosities (section 2.2.2, both SPH
    forms) on the benchmark tree: the call's wall time (synchronous: gather
    and validation, per-node chunk sums, FP32 copies), the member visits it
    makes (sum of the counts of the nodes of >= 2 sources), and the FP32C
    rate call on the weighted tree beside the plain one."""
    import torch
    from paper_1005_5312_amd import Box, LUM_KERNEL_MEAN, LUM_KERNEL_VOLUME, workloads as W
    dev = torch.device("cuda", 0)
    h, vol = W.source_kernel_inputs(w)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    sx, sl, hh, vv = d(w.src_xyz), d(w.src_lum), d(h), d(vol)
    tgt = d(w.tgt_xyz)
    ss = d(w.self_src) if w.self_src is not None else None
    box = Box(tuple(float(v) for v in w.box_lo), float(w.box_size), float(w.length_unit_cm))
    out = {"n_sources": w.n_src}
    plain = ctx.build_source_tree(box, sx, sl)
    g0 = ctx.compute_rates(plain, grid, tgt, ss, theta, w.sigma, prec="fp32c")
    ctx.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g0 = ctx.compute_rates(plain, grid, tgt, ss, theta, w.sigma, prec="fp32c")
    ctx.synchronize()
    out["rates_plain_ms"] = (time.perf_counter() - t0) * 1e3 / reps
    e = ctx.tree_export(plain)
    kind = e["geo"][:, 3] >> 8
    out["member_visits"] = int(e["link"][kind != 2, 2].sum())
    g0 = g0.double().cpu().numpy()
    plain.free()
    for form, name in ((LUM_KERNEL_MEAN, "mean"), (LUM_KERNEL_VOLUME, "volume")):
        tree = ctx.build_source_tree(box, sx, sl)
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            ctx.tree_kernel_luminosity(tree, form, hh, vv)
            best = min(best, (time.perf_counter() - t0) * 1e3)
        g = ctx.compute_rates(tree, grid, tgt, ss, theta, w.sigma, prec="fp32c")
        ctx.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g = ctx.compute_rates(tree, grid, tgt, ss, theta, w.sigma, prec="fp32c")
        ctx.synchronize()
        rms = (time.perf_counter() - t0) * 1e3 / reps
        g = g.double().cpu().numpy()
        ok = g0 > 0
        out[name] = {"call_ms": best, "member_visits_per_s": out["member_visits"] / (best * 1e-3),
                     "rates_ms": rms, "median_gamma_ratio_to_eq14": float(np.median(g[ok] / g0[ok]))}
        tree.free()
    return out


def shadow_bench(reps=3):
    """The shadowing configuration (2^21 emitting particles, a 1e50/s star,
    16 dense neutral clumps, theta = 1, G = 128): rate-call time in both
    precisions and the FP32C error against FP64 over every particle, in the
    clumps and outside them."""
    import torch
    import paper_1005_5312_amd as S
    from paper_1005_5312_amd import workloads as W
    w = W.make_shadow()
    ctx = S.Context(0)
    dev = torch.device("cuda", 0)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    box = S.Box(tuple(float(v) for v in w.box_lo), float(w.box_size), float(w.length_unit_cm))
    tree, grid = ctx.build_scene(box, d(w.src_xyz), d(w.src_lum), d(w.gas_xyz), d(w.gas_h), d(w.gas_nhi),
                                 w.grid_log2)
    tgt, ss = d(w.tgt_xyz), d(w.self_src)
    res = {}
    outs = {"fp64": torch.empty(w.n_tgt, dtype=torch.float64, device=dev),
            "fp32c": torch.empty(w.n_tgt, dtype=torch.float32, device=dev)}
    for prec, out in outs.items():
        ctx.compute_rates_raw(tree, grid, tgt, ss, 1.0, w.sigma, prec, out)
        ctx.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.compute_rates_raw(tree, grid, tgt, ss, 1.0, w.sigma, prec, out)
        ctx.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        res[prec] = {"ms_per_call": ms, "evals_per_s": w.n_tgt / (ms * 1e-3)}
    g64 = outs["fp64"].cpu().numpy()
    g32 = outs["fp32c"].cpu().numpy().astype(np.float64)
    clump = w.gas_nhi > 0.01
    res["fp32c_vs_fp64_all"] = _rel_stats(g32, g64)
    res["fp32c_vs_fp64_in_clumps"] = _rel_stats(g32[clump], g64[clump])
    res["fp32c_vs_fp64_outside"] = _rel_stats(g32[~clump], g64[~clump])
    res["workload"] = WORKLOAD_TEXT["shadow"]
    log(f"[bench] shadow: fp32c {res['fp32c']['ms_per_call']:.1f} ms, fp64 {res['fp64']['ms_per_call']:.1f} ms, "
        f"fp32c vs fp64 max rel {res['fp32c_vs_fp64_all']['max']:.2e}")
    tree.free()
    grid.free()
    ctx.close()
    return res


def theta_sweep_bench(thetas=(0.0, 0.3, 0.5, 0.8, 1.0), reps=3):
    """The clumpy medium (2^18 particles, 1024 sources with L = 10^U[47,50])
    over the opening angle: time per rate call in both precisions and the
    error against theta = 0, where every source is summed on its own (the
    exact sum over sources on the same grid), as median / p99 / max of the
    relative difference over all 2^18 particles."""
    import torch
    import paper_1005_5312_amd as S
    from paper_1005_5312_amd import workloads as W
    w = W.make_clumpy()
    ctx = S.Context(0)
    dev = torch.device("cuda", 0)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    box = S.Box(tuple(float(v) for v in w.box_lo), float(w.box_size), float(w.length_unit_cm))
    tree, grid = ctx.build_scene(box, d(w.src_xyz), d(w.src_lum), d(w.gas_xyz), d(w.gas_h), d(w.gas_nhi),
                                 w.grid_log2)
    tgt = d(w.tgt_xyz)
    outs = {"fp64": torch.empty(w.n_tgt, dtype=torch.float64, device=dev),
            "fp32c": torch.empty(w.n_tgt, dtype=torch.float32, device=dev)}
    ref = None
    rows = []
    for theta in thetas:
        row = {"theta": theta}
        for prec in ("fp64", "fp32c"):
            out = outs[prec]
            ctx.compute_rates_raw(tree, grid, tgt, None, theta, w.sigma, prec, out)
            ctx.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.compute_rates_raw(tree, grid, tgt, None, theta, w.sigma, prec, out)
            ctx.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps
            g = out.cpu().numpy().astype(np.float64)
            if ref is None:
                ref = g.copy()          # theta = 0, FP64: the exact sum over sources
            rel = np.abs(g - ref) / ref
            row[prec] = {"ms_per_call": ms, "evals_per_s": w.n_tgt / (ms * 1e-3),
                         "rel_err_vs_theta0_fp64": {"median": float(np.median(rel)),
                                                     "p99": float(np.percentile(rel, 99)),
                                                     "max": float(rel.max())}}
        log(f"[bench] theta {theta}: fp64 {row['fp64']['ms_per_call']:.2f} ms, fp32c "
            f"{row['fp32c']['ms_per_call']:.2f} ms, fp32c median rel err vs theta 0 "
            f"{row['fp32c']['rel_err_vs_theta0_fp64']['median']:.2e}")
        rows.append(row)
    tree.free()
    grid.free()
    ctx.close()
    return {"workload": f"{w.n_gas} particles (lognormal), {w.n_src} sources, G = {1 << w.grid_log2}",
            "sweep": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="diffuse", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--theta", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rates-only", action="store_true",
                    help="time only the rate call (profiling runs)")
    ap.add_argument("--upstream-only", action="store_true",
                    help="time only the upstream-particle chain on the clumpy medium (profiling runs)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving and batching measurements")
    ap.add_argument("--serve-rates", default="10,30,100,300,1000", help="Poisson arrival rates swept (requests/s)")
    ap.add_argument("--serve-window", type=float, default=15.0,
                    help="arrival window per rate (s): requests per rate = min(max, rate x window)")
    ap.add_argument("--serve-max-requests", type=int, default=2000, help="most requests per arrival rate")
    ap.add_argument("--serve-scenes", type=int, default=32, help="scenes in the served pool")
    ap.add_argument("--no-equilibrium", action="store_true", help="skip the equilibrium-loop measurement")
    ap.add_argument("--no-shadow", action="store_true", help="skip the 2^21-particle shadowing measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        log(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
            "the rate path would shard targets across GPUs, which is not built here.")
        sys.exit(2)

    import torch
    import paper_1005_5312_amd as S
    from paper_1005_5312_amd import workloads as W

    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        sys.exit(1)
    S.lib()   # fail loudly if the HIP library is missing
    def calibration_copy():
        # a plain 1 GiB device copy: the reference for the HBM byte counters
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.upstream_only:
        if args.copy_calibration:
            calibration_copy()
        print(json.dumps({"upstream_chain": upstream_bench(reps=max(1, args.steps))}), flush=True)
        return

    log(f"[bench] generating workload {args.workload}")
    w = W.make(args.workload)
    box = S.Box(tuple(float(v) for v in w.box_lo), float(w.box_size), float(w.length_unit_cm))
    dev = torch.device("cuda", 0)
    src_xyz = torch.from_numpy(w.src_xyz).to(dev)
    src_lum = torch.from_numpy(w.src_lum).to(dev)
    gas_xyz = torch.from_numpy(w.gas_xyz).to(dev)
    gas_h = torch.from_numpy(w.gas_h).to(dev)
    gas_nhi = torch.from_numpy(w.gas_nhi).to(dev)
    tgt = torch.from_numpy(np.ascontiguousarray(w.tgt_xyz)).to(dev)
    ss = None if w.self_src is None else torch.from_numpy(w.self_src).to(dev)
    out32 = torch.empty(w.n_tgt, dtype=torch.float32, device=dev)
    out64 = torch.empty(w.n_tgt, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    ctx = S.Context(0)
    stream = ctx.stream
    theta = args.theta

    def step():
        # tree and grid built at the same time (two streams), then the rates
        tree, grid = ctx.build_scene(box, src_xyz, src_lum, gas_xyz, gas_h, gas_nhi, w.grid_log2)
        ctx.compute_rates(tree, grid, tgt, ss, theta, w.sigma, "fp32c", out=out32)
        return tree, grid

    result = {}
    if not args.rates_only:
        log(f"[bench] warmup {args.warmup} full steps")
        for _ in range(args.warmup):
            t, g = step()
            ctx.synchronize()
            t.free()
            g.free()
        torch.cuda.synchronize()
        log(f"[bench] timing {args.steps} full steps")
        t0 = time.perf_counter()
        for _ in range(args.steps):
            t, g = step()
            t.free()
            g.free()
        ctx.synchronize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms_step = (t1 - t0) * 1e3 / max(args.steps, 1)
        result["ms_per_step"] = ms_step
        log(f"[bench] full step {ms_step:.3f} ms")

    # resident tree and grid: phase times and the rate call alone
    ta = time.perf_counter()
    tree = ctx.build_source_tree(box, src_xyz, src_lum)
    tb = time.perf_counter()
    grid = ctx.build_gas_grid(box, gas_xyz, gas_h, gas_nhi, w.grid_log2)
    tc = time.perf_counter()
    tree.free()
    grid.free()
    td = time.perf_counter()
    tree, grid = ctx.build_scene(box, src_xyz, src_lum, gas_xyz, gas_h, gas_nhi, w.grid_log2)
    te = time.perf_counter()
    rates = {}
    kern = {}
    for prec, out in (("fp32c", out32), ("fp64", out64)):
        for _ in range(max(1, args.warmup)):
            ctx.compute_rates(tree, grid, tgt, ss, theta, w.sigma, prec, out=out)
        ctx.synchronize()
        ctx.profile(True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            ctx.compute_rates_raw(tree, grid, tgt, ss, theta, w.sigma, prec, out)
        e1.record(stream)
        ctx.synchronize()
        ms = e0.elapsed_time(e1) / max(args.steps, 1)
        n, tot, mx = ctx.profile_read()
        ctx.profile(False)
        rates[prec] = {"ms_per_call": ms, "evals_per_s": w.n_tgt / (ms * 1e-3)}
        kern[prec] = {"launches": n, "avg_ms": tot / max(n, 1), "max_ms": mx}
        log(f"[bench] rates {prec}: {ms:.3f} ms/call, walk kernel avg {tot / max(n, 1):.3f} ms")

    if args.copy_calibration:
        calibration_copy()

    log("[bench] work counters")
    cnt = {p: ctx.rate_counters(tree, grid, tgt, ss, theta, p) for p in ("fp32c",)}
    c = cnt["fp32c"]
    sha = source_sha()
    alg = {p: algorithmic_bytes(c, p) for p in ("fp32c", "fp64")}
    prec = "fp32c"
    t_k = kern[prec]["avg_ms"] * 1e-3
    ach = alg[prec] / t_k / 1e9
    traffic = traffic_from_profiles(args.workload, prec, sha)
    cnt_p = counters_from_profiles(args.workload, prec, sha)
    # issue limits of the chip: one VALU wave-instruction per CU per cycle
    # (a wave64 instruction occupies one of the 4 SIMDs for 4 cycles)
    cyc = CUS * CLOCK_HZ * t_k
    valu_frac = cnt_p["SQ_INSTS_VALU"] / cyc if cnt_p else None
    l1_rate = cnt_p["TCP_TOTAL_CACHE_ACCESSES_sum"] / cyc if cnt_p else None
    hbm_frac = traffic / t_k / (HBM_PEAK_GBS * 1e9) if traffic else None
    # the texture addresser (vector memory address path) busy share from the
    # same counter pass as the L1 accesses (GRBM_GUI_ACTIVE sums the 8 XCDs)
    ta_frac = (cnt_p["TA_BUSY_avr"] / (cnt_p["GRBM_GUI_ACTIVE_pass_b"] / 8.0)
               if cnt_p and "TA_BUSY_avr" in cnt_p and cnt_p.get("GRBM_GUI_ACTIVE_pass_b") else None)
    if valu_frac is not None:
        bound = "alu" if valu_frac >= (hbm_frac or 0.0) else "hbm"
    else:
        bound = "alu"   # by the last counters taken (VALU issue and L1), not retaken for these sources
    roofline = {"bound": bound, "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                "frac_basis": "algorithmic bytes per launch (per target: 28 + 12 per opening test + 16 per entry "
                              "+ 4 per grid cell crossed, exact counters of this launch) / walk-kernel time / "
                              "8 TB/s; these bytes are served mostly by L1 and L2, measured HBM traffic is "
                              "'traffic'",
                "valu_issue_frac": round(valu_frac, 4) if valu_frac is not None else None,
                "l1_accesses_per_cu_cycle": round(l1_rate, 4) if l1_rate is not None else None,
                "ta_busy_frac": round(ta_frac, 4) if ta_frac is not None else None,
                "hbm_traffic_frac": round(hbm_frac, 4) if hbm_frac is not None else None,
                "counters": "profiles/rates_kernel_fp32c_{}_sq_tcp_counters.txt".format(args.workload)
                if cnt_p else None,
                "kernel": "rates_kernel<FP32C> (tree walk + ray march + Gamma)",
                "algorithmic_bytes_per_launch": alg[prec], "kernel_avg_ms": round(kern[prec]["avg_ms"], 4)}
    ach64 = alg["fp64"] / (kern["fp64"]["avg_ms"] * 1e-3) / 1e9
    if not args.rates_only:
        cbw = copy_bandwidth()
        roofline["copy_GBs"] = round(cbw, 1)          # achievable: a plain device copy
        roofline["frac_of_copy"] = round(ach / cbw, 4)
        log(f"[bench] device copy {cbw:.0f} GB/s")

    serve_stats = batch_stats = None
    if not args.no_serve and not args.rates_only:
        log(f"[bench] batched launch: 256 instances of 2^14 targets")
        batch_stats = batch_bench()
        rates_list = [float(v) for v in args.serve_rates.split(",") if v]
        serve_stats = serve_bench(rates_list, args.serve_window, args.serve_max_requests, args.serve_scenes,
                                  log_fn=log)

    kion_stats = None
    if not args.rates_only:
        log("[bench] k_self and total k_ion terms")
        kion_stats = k_ion_bench(ctx, w, out32)

    lw_stats = None
    if not args.rates_only:
        log("[bench] H2 photodissociation rates")
        lw_stats = lw_bench()

    up_stats = None
    if not args.rates_only:
        log("[bench] upstream-particle chain")
        up_stats = upstream_bench()

    sweep_stats = None
    if not args.rates_only:
        log("[bench] opening-angle sweep on the clumpy medium")
        sweep_stats = theta_sweep_bench()

    tree_err = None
    if not args.rates_only:
        log("[bench] tree approximation against theta = 0 on sampled targets")
        tree_err = tree_error_bench(ctx, w, tree, grid)

    klum_stats = None
    if not args.rates_only:
        log("[bench] kernel-weighted virtual-source luminosities")
        klum_stats = kernel_lum_bench(ctx, w, grid, theta)

    shadow_stats = None
    if not args.rates_only and not args.no_shadow:
        log("[bench] shadowing configuration (2^21 particles)")
        shadow_stats = shadow_bench()

    eq_stats = None
    if not args.no_equilibrium and not args.rates_only:
        log("[bench] photoionisation equilibrium (Test 4 setting)")
        eq_stats = equilibrium_bench()

    cpu = None
    if not args.no_cpu_baseline and not args.rates_only:
        log("[bench] CPU baseline (oracle) on the whole workload")
        cpu = cpu_baseline(w)

    ms_step = result.get("ms_per_step", rates["fp32c"]["ms_per_call"])
    line = {
        "metric": METRIC,
        "value": w.n_tgt / (ms_step * 1e-3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "n_targets": w.n_tgt, "n_sources": w.n_src,
                   "grid": 1 << w.grid_log2, "theta_crit": theta, "precision": "fp32c: fp64 opening test, ray geometry and column sums; fp32 grid values, exp, terms and Kahan-compensated Gamma",
                   "step": "tree build and gas grid (concurrent, start_build_scene) + target order + walk/march/Gamma"
                   if not args.rates_only else "rate call only"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phases_ms": {"tree_build": (tb - ta) * 1e3, "grid_build": (tc - tb) * 1e3,
                      "scene_build_both_streams": (te - td) * 1e3,
                      "rates_fp32c": rates["fp32c"]["ms_per_call"], "rates_fp64": rates["fp64"]["ms_per_call"]},
        "rates_only": {"fp32c_evals_per_s": rates["fp32c"]["evals_per_s"],
                       "fp64_evals_per_s": rates["fp64"]["evals_per_s"],
                       "fp64_walk_kernel_ms": round(kern["fp64"]["avg_ms"], 4),
                       "fp64_roofline_frac": round(ach64 / HBM_PEAK_GBS, 4)},
        "serve": serve_stats,
        "batched": batch_stats,
        "equilibrium": eq_stats,
        "theta_sweep": sweep_stats,
        "tree_error": tree_err,
        "shadow": shadow_stats,
        "kernel_luminosity": klum_stats,
        "k_ion_terms": kion_stats,
        "h2_dissociation": lw_stats,
        "upstream_chain": up_stats,
        "work_per_target": {"opening_tests": float(c[:, 0].mean()), "entries": float(c[:, 1].mean()),
                            "grid_cells": float(c[:, 2].mean())},
        "source_sha": sha,
    }
    print(json.dumps(line), flush=True)
    tree.free()
    grid.free()
    ctx.close()


if __name__ == "__main__":
    main()
