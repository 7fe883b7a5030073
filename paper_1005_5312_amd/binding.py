"""Python binding of libstart (ctypes).  Argument marshalling only: every
step of the computation runs in the HIP library.  Device memory and streams
come from PyTorch; arrays are torch tensors on the context's GPU.

Raises ImportError-like LibraryMissing when libstart.so has not been built and
StartError for every non-zero status of the C-ABI.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstart.so")

OK, EINVAL, ENOMEM, EHIP, EOUTOFBOX, ENONFINITE, EBUDGET, ENOTIMPL, ECAPACITY = 0, -1, -2, -3, -4, -5, -6, -7, -8
FP64, FP32C = 0, 1
LUM_KERNEL_MEAN, LUM_KERNEL_VOLUME = 1, 2
STATUS_NAMES = {OK: "START_OK", EINVAL: "START_EINVAL", ENOMEM: "START_ENOMEM", EHIP: "START_EHIP",
                EOUTOFBOX: "START_EOUTOFBOX", ENONFINITE: "START_ENONFINITE", EBUDGET: "START_EBUDGET",
                ENOTIMPL: "START_ENOTIMPL", ECAPACITY: "START_ECAPACITY"}

# every symbol include/start.h declares
EXPORTS = ("start_ctx_create", "start_ctx_destroy", "start_last_error", "start_synchronize",
           "start_bytes_in_use", "start_build_source_tree", "start_tree_free", "start_build_gas_grid",
           "start_build_scene",
           "start_grid_free", "start_grid_size", "start_compute_rates", "start_compute_rates_batched",
           "start_estimate_bytes", "start_tree_export", "start_interaction_lists", "start_grid_export",
           "start_rate_counters", "start_profile_enable", "start_profile_read", "start_equilibrium_update",
           "start_ionization_equilibrium", "start_recombination_emission", "start_total_ionization",
           "start_compute_dissociation_rates", "start_set_tile_targets", "start_autotune_rates",
           "start_set_graph_replay", "start_compute_rates_upstream", "start_diffuse_equilibrium",
           "start_set_grid_pairs", "start_tree_kernel_luminosity", "start_compute_rates_noalloc",
           "start_rates_plan_create", "start_rates_plan_launch", "start_rates_plan_free")


class LibraryMissing(RuntimeError):
    pass


class StartError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Box(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("size", C.c_double), ("length_unit_cm", C.c_double)]


class _Item(C.Structure):
    _fields_ = [("tree", C.c_void_p), ("grid", C.c_void_p), ("n_t", C.c_int64), ("tgt_xyz", C.c_void_p),
                ("self_src", C.c_void_p), ("theta_crit", C.c_double), ("sigma_cm2", C.c_double),
                ("prec", C.c_int), ("gamma_out", C.c_void_p)]


@dataclasses.dataclass(frozen=True)
class Box:
    lo: tuple
    size: float
    length_unit_cm: float

    def c(self):
        b = _Box()
        for k in range(3):
            b.lo[k] = float(self.lo[k])
        b.size = float(self.size)
        b.length_unit_cm = float(self.length_unit_cm)
        return b


_lib = None


def lib():
    """The loaded libstart.so; raises LibraryMissing if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} not built: run python -m paper_1005_5312_amd.build")
    L = C.CDLL(LIB_PATH)
    P, i64, d = C.c_void_p, C.c_int64, C.c_double
    sig = {
        "start_ctx_create": ([C.c_int, P, C.c_size_t, P], C.c_int),
        "start_ctx_destroy": ([P], None),
        "start_last_error": ([P], C.c_char_p),
        "start_synchronize": ([P], C.c_int),
        "start_bytes_in_use": ([P], C.c_size_t),
        "start_build_source_tree": ([P, P, i64, P, P, P], C.c_int),
        "start_tree_free": ([P, P], C.c_int),
        "start_tree_kernel_luminosity": ([P, P, C.c_int, P, P], C.c_int),
        "start_build_gas_grid": ([P, P, i64, P, P, P, C.c_int, P], C.c_int),
        "start_build_scene": ([P, P, i64, P, P, i64, P, P, P, C.c_int, P, P], C.c_int),
        "start_grid_free": ([P, P], C.c_int),
        "start_grid_size": ([P], C.c_int),
        "start_compute_rates": ([P, P, P, i64, P, P, d, d, C.c_int, P], C.c_int),
        "start_compute_rates_noalloc": ([P, P, P, i64, P, P, d, d, C.c_int, P], C.c_int),
        "start_compute_rates_batched": ([P, C.c_int, P], C.c_int),
        "start_rates_plan_create": ([P, C.c_int, P, P], C.c_int),
        "start_rates_plan_launch": ([P, P], C.c_int),
        "start_rates_plan_free": ([P, P], C.c_int),
        "start_estimate_bytes": ([i64, i64, i64, C.c_int, C.c_int], C.c_size_t),
        "start_tree_export": ([P, P, P, P, P, P, P, P], C.c_int),
        "start_interaction_lists": ([P, P, i64, P, P, d, P, P, i64], C.c_int),
        "start_grid_export": ([P, P, P], C.c_int),
        "start_rate_counters": ([P, P, P, i64, P, P, d, C.c_int, P], C.c_int),
        "start_profile_enable": ([P, C.c_int], C.c_int),
        "start_profile_read": ([P, P, P, P], C.c_int),
        "start_equilibrium_update": ([P, i64, P, P, C.c_int, d, P, P, P], C.c_int),
        "start_ionization_equilibrium": ([P, P, i64, P, P, P, C.c_int, d, d, d, C.c_int, C.c_int, d, P, P, P, P],
                                         C.c_int),
        "start_recombination_emission": ([P, i64, P, P, P, d, d, P, P], C.c_int),
        "start_total_ionization": ([P, i64, P, P, P, C.c_int, P, P], C.c_int),
        "start_compute_dissociation_rates": ([P, P, P, i64, P, P, d, C.c_int, P], C.c_int),
        "start_set_tile_targets": ([P, C.c_int], C.c_int),
        "start_set_graph_replay": ([P, C.c_int], C.c_int),
        "start_set_grid_pairs": ([P, C.c_int], C.c_int),
        "start_diffuse_equilibrium": ([P, P, i64, P, P, P, P, i64, P, P, C.c_int, d, d, d, d, C.c_int, C.c_int, d,
                                       P, P, P, P], C.c_int),
        "start_compute_rates_upstream": ([P, P, P, i64, P, P, P, P, d, d, P, P, P, i64, P], C.c_int),
        "start_autotune_rates": ([P, C.c_int, P, C.c_int, P, P], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return _lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _prec(p):
    if p in (FP64, "fp64", "FP64"):
        return FP64
    if p in (FP32C, "fp32c", "FP32C", "fp32"):
        return FP32C
    raise ValueError(f"unknown precision {p!r}")


def _xyz(t, dev):
    import torch
    t = torch.as_tensor(t)
    if t.dim() != 2 or t.shape[0] != 3:
        raise ValueError("positions must have shape (3, n)")
    return t.to(device=dev, dtype=torch.float64).contiguous()


def _vec(t, dev, dtype=None):
    import torch
    dtype = dtype or torch.float64
    return torch.as_tensor(t).to(device=dev, dtype=dtype).contiguous()


class SourceTree:
    def __init__(self, ctx, handle, box, n_src):
        self.ctx, self._h, self.box, self.n_src = ctx, handle, box, n_src

    def free(self):
        if self._h:
            lib().start_tree_free(self.ctx._h, self._h)
            self._h = None

    def __del__(self):
        try:
            if self._h and self.ctx._h:
                self.free()
        except Exception:
            pass


class GasGrid:
    def __init__(self, ctx, handle, box):
        self.ctx, self._h, self.box = ctx, handle, box
        self.G = lib().start_grid_size(handle)

    def free(self):
        if self._h:
            lib().start_grid_free(self.ctx._h, self._h)
            self._h = None

    def __del__(self):
        try:
            if self._h and self.ctx._h:
                self.free()
        except Exception:
            pass


class RatePlan:
    """A staged batch replayed from a HIP graph (start_rates_plan_*): launch()
    recomputes the outputs the items named.  Keeps the item tensors alive."""

    def __init__(self, ctx, handle, keep):
        self.ctx, self._h, self._keep = ctx, handle, keep

    def launch(self):
        cur = self.ctx._enter(*self._keep)
        self.ctx._check(lib().start_rates_plan_launch(self.ctx._h, self._h), "start_rates_plan_launch")
        self.ctx._leave(cur)

    def free(self):
        if self._h:
            lib().start_rates_plan_free(self.ctx._h, self._h)
            self._h = None

    def __del__(self):
        try:
            if self._h and self.ctx._h:
                self.free()
        except Exception:
            pass


class Context:
    """One libstart context on a GPU.  stream: a torch.cuda.Stream to run on
    (default: a new one); hbm_budget: bytes the library may hold (0 = no cap)."""

    def __init__(self, device: int = 0, stream=None, hbm_budget: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libstart needs a GPU (torch.cuda.is_available() is False)")
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        h = C.c_void_p()
        self._check(lib().start_ctx_create(device, C.c_void_p(self.stream.cuda_stream), int(hbm_budget),
                                           C.byref(h)), "start_ctx_create", ctx=None)
        self._h = h

    def _check(self, rc, what, ctx="self"):
        if rc != OK:
            msg = what
            if ctx == "self" and getattr(self, "_h", None):
                msg = f"{what}: {lib().start_last_error(self._h).decode(errors='replace')}"
            raise StartError(rc, msg)

    def close(self):
        if getattr(self, "_h", None):
            lib().start_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -------------------------------------------------------------- builds --
    def build_source_tree(self, box: Box, src_xyz, src_lum) -> SourceTree:
        xyz = _xyz(src_xyz, self.device)
        lum = _vec(src_lum, self.device)
        n = xyz.shape[1]
        if lum.numel() != n:
            raise ValueError("src_lum length does not match src_xyz")
        h = C.c_void_p()
        b = box.c()
        cur = self._enter(xyz, lum)
        self._check(lib().start_build_source_tree(self._h, C.byref(b), n, _ptr(xyz), _ptr(lum), C.byref(h)),
                    "start_build_source_tree")
        self._leave(cur)
        return SourceTree(self, h, box, n)

    def tree_kernel_luminosity(self, tree: SourceTree, form: int, src_h, src_vol=None) -> SourceTree:
        """Kernel-weighted virtual-source luminosities (LUM_KERNEL_MEAN or
        LUM_KERNEL_VOLUME) in place; src_h and src_vol in source input order."""
        hh = _vec(src_h, self.device)
        vv = None if src_vol is None else _vec(src_vol, self.device)
        if hh.numel() != tree.n_src or (vv is not None and vv.numel() != tree.n_src):
            raise ValueError("src_h / src_vol length does not match the tree's sources")
        cur = self._enter(hh, vv)
        self._check(lib().start_tree_kernel_luminosity(self._h, tree._h, int(form), _ptr(hh), _ptr(vv)),
                    "start_tree_kernel_luminosity")
        self._leave(cur)
        return tree

    def build_gas_grid(self, box: Box, gas_xyz, gas_h, gas_nhi, grid_log2: int = 0) -> GasGrid:
        xyz = _xyz(gas_xyz, self.device)
        hh = _vec(gas_h, self.device)
        nhi = _vec(gas_nhi, self.device)
        n = xyz.shape[1]
        if hh.numel() != n or nhi.numel() != n:
            raise ValueError("gas_h / gas_nhi length does not match gas_xyz")
        h = C.c_void_p()
        b = box.c()
        cur = self._enter(xyz, hh, nhi)
        self._check(lib().start_build_gas_grid(self._h, C.byref(b), n, _ptr(xyz), _ptr(hh), _ptr(nhi),
                                               int(grid_log2), C.byref(h)), "start_build_gas_grid")
        self._leave(cur)
        return GasGrid(self, h, box)

    def build_scene(self, box: Box, src_xyz, src_lum, gas_xyz, gas_h, gas_nhi, grid_log2: int = 0):
        """(SourceTree, GasGrid) of one scene, the two builds run at the same
        time (start_build_scene)."""
        sx = _xyz(src_xyz, self.device)
        sl = _vec(src_lum, self.device)
        gx = _xyz(gas_xyz, self.device)
        gh = _vec(gas_h, self.device)
        gn = _vec(gas_nhi, self.device)
        ns, ng = sx.shape[1], gx.shape[1]
        if sl.numel() != ns:
            raise ValueError("src_lum length does not match src_xyz")
        if gh.numel() != ng or gn.numel() != ng:
            raise ValueError("gas_h / gas_nhi length does not match gas_xyz")
        ht, hg = C.c_void_p(), C.c_void_p()
        b = box.c()
        cur = self._enter(sx, sl, gx, gh, gn)
        self._check(lib().start_build_scene(self._h, C.byref(b), ns, _ptr(sx), _ptr(sl), ng, _ptr(gx), _ptr(gh),
                                            _ptr(gn), int(grid_log2), C.byref(ht), C.byref(hg)),
                    "start_build_scene")
        self._leave(cur)
        return SourceTree(self, ht, box, ns), GasGrid(self, hg, box)

    def _enter(self, *tensors):
        """Orders the context stream after the caller's current stream and
        keeps the inputs alive until the context stream has used them."""
        import torch
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        for t in tensors:
            if t is not None:
                t.record_stream(self.stream)
        return cur

    def _leave(self, cur):
        cur.wait_stream(self.stream)

    # --------------------------------------------------------------- rates --
    def compute_rates(self, tree: SourceTree, grid: GasGrid, tgt_xyz, self_src=None, theta: float = 1.0,
                      sigma: float = 6.3e-18, prec="fp32c", out=None):
        """Gamma per target (s^-1 per H I atom), float64 for fp64 and float32
        for fp32c.  Asynchronous on the context stream; call synchronize()
        before reading device-side input errors."""
        import torch
        p = _prec(prec)
        xyz = _xyz(tgt_xyz, self.device)
        n = xyz.shape[1]
        ss = None if self_src is None else _vec(self_src, self.device, torch.int64)
        if ss is not None and ss.numel() != n:
            raise ValueError("self_src length does not match targets")
        dt = torch.float64 if p == FP64 else torch.float32
        if out is None:
            out = torch.empty(n, dtype=dt, device=self.device)
        elif out.dtype != dt or out.numel() != n or not out.is_contiguous():
            raise ValueError("out has the wrong dtype, size or layout")
        cur = self._enter(xyz, ss, out)
        self._check(lib().start_compute_rates(self._h, tree._h, grid._h, n, _ptr(xyz), _ptr(ss), float(theta),
                                              float(sigma), p, _ptr(out)), "start_compute_rates")
        self._leave(cur)
        return out

    def compute_rates_noalloc(self, tree: SourceTree, grid: GasGrid, tgt_xyz, self_src=None, theta: float = 1.0,
                              sigma: float = 6.3e-18, prec="fp32c", out=None):
        """compute_rates through start_compute_rates_noalloc: the library's
        fixed per-device scratch instead of context memory (at most 2^18
        targets; calls on one GPU must not overlap).  Same results."""
        import torch
        p = _prec(prec)
        xyz = _xyz(tgt_xyz, self.device)
        n = xyz.shape[1]
        ss = None if self_src is None else _vec(self_src, self.device, torch.int64)
        if ss is not None and ss.numel() != n:
            raise ValueError("self_src length does not match targets")
        dt = torch.float64 if p == FP64 else torch.float32
        if out is None:
            out = torch.empty(n, dtype=dt, device=self.device)
        elif out.dtype != dt or out.numel() != n or not out.is_contiguous():
            raise ValueError("out has the wrong dtype, size or layout")
        cur = self._enter(xyz, ss, out)
        self._check(lib().start_compute_rates_noalloc(self._h, tree._h, grid._h, n, _ptr(xyz), _ptr(ss),
                                                      float(theta), float(sigma), p, _ptr(out)),
                    "start_compute_rates_noalloc")
        self._leave(cur)
        return out

    def compute_dissociation_rates(self, tree: SourceTree, grid: GasGrid, tgt_xyz, self_src=None,
                                   theta: float = 1.0, prec="fp32c", out=None):
        """H2 photodissociation rate per target (s^-1): `tree` built from
        Lyman-Werner luminosities, `grid` from n_H2.  float64 for fp64 and
        float32 for fp32c.  Asynchronous."""
        import torch
        p = _prec(prec)
        xyz = _xyz(tgt_xyz, self.device)
        n = xyz.shape[1]
        ss = None if self_src is None else _vec(self_src, self.device, torch.int64)
        if ss is not None and ss.numel() != n:
            raise ValueError("self_src length does not match targets")
        dt = torch.float64 if p == FP64 else torch.float32
        if out is None:
            out = torch.empty(n, dtype=dt, device=self.device)
        elif out.dtype != dt or out.numel() != n or not out.is_contiguous():
            raise ValueError("out has the wrong dtype, size or layout")
        cur = self._enter(xyz, ss, out)
        self._check(lib().start_compute_dissociation_rates(self._h, tree._h, grid._h, n, _ptr(xyz), _ptr(ss),
                                                           float(theta), p, _ptr(out)),
                    "start_compute_dissociation_rates")
        self._leave(cur)
        return out

    def compute_rates_upstream(self, tree: SourceTree, grid: GasGrid, gas_xyz, gas_h, gas_nhi, self_src=None,
                               theta: float = 1.0, sigma: float = 6.3e-18, structure: bool = False):
        """Gamma (float64) of every gas particle with the upstream-particle
        chain optical depths; with structure=True also (offsets [n+1], parents
        [pairs] in list-export order, number of pairs integrated along the
        ray) as numpy arrays.  Synchronous."""
        import torch
        xyz = _xyz(gas_xyz, self.device)
        n = xyz.shape[1]
        h = _vec(gas_h, self.device)
        nhi = _vec(gas_nhi, self.device)
        ss = None if self_src is None else _vec(self_src, self.device, torch.int64)
        out = torch.empty(n, dtype=torch.float64, device=self.device)
        offs = np.zeros(n + 1, np.int64)
        roots = C.c_int64()
        cur = self._enter(xyz, h, nhi, ss, out)
        self._check(lib().start_compute_rates_upstream(self._h, tree._h, grid._h, n, _ptr(xyz), _ptr(h), _ptr(nhi),
                                                       _ptr(ss), float(theta), float(sigma), _ptr(out),
                                                       offs.ctypes.data_as(C.c_void_p) if structure else None,
                                                       None, 0, C.byref(roots)),
                    "start_compute_rates_upstream")
        par = None
        if structure:
            par = np.zeros(max(int(offs[-1]), 1), np.int64)
            self._check(lib().start_compute_rates_upstream(self._h, tree._h, grid._h, n, _ptr(xyz), _ptr(h),
                                                           _ptr(nhi), _ptr(ss), float(theta), float(sigma), _ptr(out),
                                                           None, par.ctypes.data_as(C.c_void_p), par.size,
                                                           C.byref(roots)),
                        "start_compute_rates_upstream")
            par = par[: int(offs[-1])]
        self._leave(cur)
        return (out, offs, par, roots.value) if structure else out

    def compute_rates_raw(self, tree: SourceTree, grid: GasGrid, xyz, ss, theta, sigma, prec, out):
        """Enqueues on the context stream with prepared device tensors and no
        stream bookkeeping (for timing loops that manage streams themselves)."""
        self._check(lib().start_compute_rates(self._h, tree._h, grid._h, xyz.shape[1], _ptr(xyz), _ptr(ss),
                                              float(theta), float(sigma), _prec(prec), _ptr(out)),
                    "start_compute_rates")

    def _items(self, items):
        arr = (_Item * len(items))()
        keep = []
        for k, it in enumerate(items):
            xyz = _xyz(it["tgt_xyz"], self.device)
            keep.append(xyz)
            arr[k].tree = it["tree"]._h
            arr[k].grid = it["grid"]._h
            arr[k].n_t = xyz.shape[1]
            arr[k].tgt_xyz = xyz.data_ptr()
            ss = it.get("self_src")
            arr[k].self_src = None if ss is None else ss.data_ptr()
            arr[k].theta_crit = float(it.get("theta", 1.0))
            arr[k].sigma_cm2 = float(it.get("sigma", 6.3e-18))
            arr[k].prec = _prec(it.get("prec", "fp32c"))
            arr[k].gamma_out = it["out"].data_ptr()
            keep += [ss, it["out"]]
        return arr, keep

    def compute_rates_batched(self, items):
        """items: list of dicts with keys tree, grid, tgt_xyz, self_src, theta,
        sigma, prec, out (tensors prepared as for compute_rates)."""
        arr, keep = self._items(items)
        cur = self._enter(*keep)
        self._check(lib().start_compute_rates_batched(self._h, len(items), arr), "start_compute_rates_batched")
        self._leave(cur)

    def rates_plan(self, items) -> RatePlan:
        """Stages the batch (items as for compute_rates_batched), runs it once
        and captures its rate kernels; RatePlan.launch() replays them."""
        arr, keep = self._items(items)
        cur = self._enter(*keep)
        h = C.c_void_p()
        self._check(lib().start_rates_plan_create(self._h, len(items), arr, C.byref(h)), "start_rates_plan_create")
        self._leave(cur)
        return RatePlan(self, h, [k for k in keep if k is not None])

    def set_graph_replay(self, enable: bool):
        """Replay the equilibrium iterations from a captured HIP graph (default)
        or launch them one by one."""
        self._check(lib().start_set_graph_replay(self._h, 1 if enable else 0), "start_set_graph_replay")

    def set_grid_pairs(self, enable: bool):
        """Refill the equilibrium loops' grids from recorded (cell, particle)
        pairs (default) or search the stencil at every refill."""
        self._check(lib().start_set_grid_pairs(self._h, 1 if enable else 0), "start_set_grid_pairs")

    def set_tile_targets(self, tile_targets: int):
        """Targets per wavefront of the rate kernels (1..64), or 0 for the
        autotuned choice by problem size."""
        self._check(lib().start_set_tile_targets(self._h, int(tile_targets)), "start_set_tile_targets")

    def autotune_rates(self, items, reps: int = 2):
        """Times the batch with every tile size and records the fastest for
        its size class; returns (best tile, mean ms).  Runs the batch (the
        outputs are written)."""
        arr, keep = self._items(items)
        cur = self._enter(*keep)
        best, ms = C.c_int(), C.c_double()
        self._check(lib().start_autotune_rates(self._h, len(items), arr, int(reps), C.byref(best), C.byref(ms)),
                    "start_autotune_rates")
        self._leave(cur)
        return best.value, ms.value

    def synchronize(self):
        self._check(lib().start_synchronize(self._h), "start_synchronize")

    # --------------------------------------------------------- equilibrium --
    def equilibrium_update(self, n_h, gamma, alpha: float, x_hi, n_hi=None, want_change: bool = True):
        """x_hi (float64 device tensor, updated in place) <- equilibrium
        neutral fraction for the rates gamma (float64 or float32); n_hi, if
        given, <- x n_H.  Returns max |change| (waits for the stream) when
        want_change, else None (asynchronous)."""
        import torch
        n = x_hi.numel()
        nh = _vec(n_h, self.device)
        if gamma.dtype == torch.float64:
            p = FP64
        elif gamma.dtype == torch.float32:
            p = FP32C
        else:
            raise ValueError("gamma must be float64 or float32")
        for t in (x_hi, n_hi):
            if t is not None and (t.dtype != torch.float64 or t.numel() != n or not t.is_contiguous()
                                  or t.device != torch.device(self.device)):
                raise ValueError("x_hi and n_hi must be contiguous float64 tensors of n values on the device")
        if nh.numel() != n or gamma.numel() != n or not gamma.is_contiguous():
            raise ValueError("n_h and gamma must have one contiguous value per particle")
        ch = C.c_double()
        cur = self._enter(nh, gamma, x_hi, n_hi)
        self._check(lib().start_equilibrium_update(self._h, n, _ptr(nh), _ptr(gamma), p, float(alpha), _ptr(x_hi),
                                                   _ptr(n_hi), C.byref(ch) if want_change else None),
                    "start_equilibrium_update")
        self._leave(cur)
        return ch.value if want_change else None

    def recombination_emission(self, n_h, x_hi, volume_cm3, sigma: float = 6.3e-18, alpha_1: float = 1.58e-13,
                               want_lum: bool = True, want_k_self: bool = True):
        """(emitter luminosity alpha_1 n_e n_p V, k_self) per particle as
        float64 device tensors (None where not asked for).  Asynchronous."""
        import torch
        nh, x, v = (_vec(t, self.device) for t in (n_h, x_hi, volume_cm3))
        n = nh.numel()
        if x.numel() != n or v.numel() != n:
            raise ValueError("n_h, x_hi and volume_cm3 need one value per particle")
        lum = torch.empty(n, dtype=torch.float64, device=self.device) if want_lum else None
        ks = torch.empty(n, dtype=torch.float64, device=self.device) if want_k_self else None
        cur = self._enter(nh, x, v, lum, ks)
        self._check(lib().start_recombination_emission(self._h, n, _ptr(nh), _ptr(x), _ptr(v), float(sigma),
                                                       float(alpha_1), _ptr(lum), _ptr(ks)),
                    "start_recombination_emission")
        self._leave(cur)
        return lum, ks

    def total_ionization(self, n_h, x_hi, gamma, k_self=None):
        """k_ion = x n_H gamma + k_self (float64 device tensor).  Asynchronous."""
        import torch
        nh, x = _vec(n_h, self.device), _vec(x_hi, self.device)
        n = nh.numel()
        if gamma.dtype == torch.float64:
            p = FP64
        elif gamma.dtype == torch.float32:
            p = FP32C
        else:
            raise ValueError("gamma must be float64 or float32")
        ks = None if k_self is None else _vec(k_self, self.device)
        if x.numel() != n or gamma.numel() != n or (ks is not None and ks.numel() != n) or not gamma.is_contiguous():
            raise ValueError("every array needs one contiguous value per particle")
        out = torch.empty(n, dtype=torch.float64, device=self.device)
        cur = self._enter(nh, x, gamma, ks, out)
        self._check(lib().start_total_ionization(self._h, n, _ptr(nh), _ptr(x), _ptr(gamma), p, _ptr(ks), _ptr(out)),
                    "start_total_ionization")
        self._leave(cur)
        return out

    def diffuse_equilibrium(self, box: Box, gas_xyz, gas_h, n_h, volume_cm3, star_xyz, star_lum, x_init,
                            grid_log2: int, theta: float = 1.0, sigma: float = 6.3e-18, alpha_a: float = 4.18e-13,
                            alpha_1: float = 1.58e-13, prec="fp64", max_iter: int = 100, tol: float = 1e-4):
        """Equilibrium with the transfer of recombination photons (see
        start_diffuse_equilibrium).  Returns (x, gamma, iterations,
        last_change)."""
        import torch
        p = _prec(prec)
        xyz = _xyz(gas_xyz, self.device)
        n = xyz.shape[1]
        h, nh, vol = (_vec(a, self.device) for a in (gas_h, n_h, volume_cm3))
        x = _vec(x_init, self.device).clone()
        sxyz = _xyz(star_xyz, self.device)
        slum = _vec(star_lum, self.device)
        if h.numel() != n or nh.numel() != n or vol.numel() != n or x.numel() != n or slum.numel() != sxyz.shape[1]:
            raise ValueError("per-particle and per-star arrays have the wrong lengths")
        gamma = torch.empty(n, dtype=torch.float64 if p == FP64 else torch.float32, device=self.device)
        it, ch = C.c_int(), C.c_double()
        b = box.c()
        cur = self._enter(xyz, h, nh, vol, x, sxyz, slum, gamma)
        self._check(lib().start_diffuse_equilibrium(self._h, C.byref(b), n, _ptr(xyz), _ptr(h), _ptr(nh), _ptr(vol),
                                                    sxyz.shape[1], _ptr(sxyz), _ptr(slum), int(grid_log2),
                                                    float(theta), float(sigma), float(alpha_a), float(alpha_1), p,
                                                    int(max_iter), float(tol), _ptr(x), _ptr(gamma), C.byref(it),
                                                    C.byref(ch)),
                    "start_diffuse_equilibrium")
        self._leave(cur)
        return x, gamma, it.value, ch.value

    def ionization_equilibrium(self, tree: SourceTree, gas_xyz, gas_h, n_h, x_init, grid_log2: int,
                               theta: float = 1.0, sigma: float = 6.3e-18, alpha: float = 2.6e-13,
                               prec="fp64", max_iter: int = 100, tol: float = 1e-4):
        """Fixed-point photoionisation equilibrium around the sources of
        `tree` (see start_ionization_equilibrium).  Returns (x, gamma,
        iterations, last_change); x float64, gamma float64 or float32."""
        import torch
        p = _prec(prec)
        xyz = _xyz(gas_xyz, self.device)
        n = xyz.shape[1]
        h = _vec(gas_h, self.device)
        nh = _vec(n_h, self.device)
        x = _vec(x_init, self.device).clone()
        if h.numel() != n or nh.numel() != n or x.numel() != n:
            raise ValueError("gas_h, n_h and x_init need one value per particle")
        gamma = torch.empty(n, dtype=torch.float64 if p == FP64 else torch.float32, device=self.device)
        it, ch = C.c_int(), C.c_double()
        cur = self._enter(xyz, h, nh, x, gamma)
        self._check(lib().start_ionization_equilibrium(self._h, tree._h, n, _ptr(xyz), _ptr(h), _ptr(nh),
                                                       int(grid_log2), float(theta), float(sigma), float(alpha), p,
                                                       int(max_iter), float(tol), _ptr(x), _ptr(gamma),
                                                       C.byref(it), C.byref(ch)),
                    "start_ionization_equilibrium")
        self._leave(cur)
        return x, gamma, it.value, ch.value

    def profile(self, enable: bool = True):
        """Time every following walk kernel with HIP events on the context stream."""
        self._check(lib().start_profile_enable(self._h, 1 if enable else 0), "start_profile_enable")

    def profile_read(self):
        """(launches, total_ms, max_ms) of the walk kernels timed since the last read."""
        n, tot, mx = C.c_int64(), C.c_double(), C.c_double()
        self._check(lib().start_profile_read(self._h, C.byref(n), C.byref(tot), C.byref(mx)), "start_profile_read")
        return n.value, tot.value, mx.value

    def bytes_in_use(self) -> int:
        return int(lib().start_bytes_in_use(self._h))

    # --------------------------------------------------------- diagnostics --
    def tree_export(self, tree: SourceTree):
        n = C.c_int64()
        self._check(lib().start_tree_export(self._h, tree._h, C.byref(n), None, None, None, None, None),
                    "start_tree_export")
        m, ns = n.value, tree.n_src
        out = dict(keys=np.zeros(ns, np.uint64), perm=np.zeros(ns, np.uint32), geo=np.zeros((m, 4), np.int32),
                   link=np.zeros((m, 4), np.int32), mom=np.zeros((m, 4)))
        self._check(lib().start_tree_export(self._h, tree._h, C.byref(n), out["keys"].ctypes.data_as(C.c_void_p),
                                            out["perm"].ctypes.data_as(C.c_void_p),
                                            out["geo"].ctypes.data_as(C.c_void_p),
                                            out["link"].ctypes.data_as(C.c_void_p),
                                            out["mom"].ctypes.data_as(C.c_void_p)), "start_tree_export")
        return out

    def interaction_lists(self, tree: SourceTree, tgt_xyz, self_src=None, theta: float = 1.0):
        """(offsets[n_t+1], entries) as numpy arrays."""
        import torch
        xyz = _xyz(tgt_xyz, self.device)
        n = xyz.shape[1]
        ss = None if self_src is None else _vec(self_src, self.device, torch.int64)
        off = np.zeros(n + 1, np.int64)
        self._enter(xyz, ss)
        rc = lib().start_interaction_lists(self._h, tree._h, n, _ptr(xyz), _ptr(ss), float(theta),
                                           off.ctypes.data_as(C.c_void_p), None, 0)
        if rc not in (OK, ECAPACITY):
            self._check(rc, "start_interaction_lists")
        cap = int(off[-1])
        ent = np.zeros(max(cap, 1), np.int64)
        self._check(lib().start_interaction_lists(self._h, tree._h, n, _ptr(xyz), _ptr(ss), float(theta),
                                                  off.ctypes.data_as(C.c_void_p), ent.ctypes.data_as(C.c_void_p),
                                                  cap), "start_interaction_lists")
        return off, ent[:cap]

    def grid_export(self, grid: GasGrid):
        G = grid.G
        out = np.zeros(G ** 3)
        self._check(lib().start_grid_export(self._h, grid._h, out.ctypes.data_as(C.c_void_p)), "start_grid_export")
        return out.reshape(G, G, G)

    def rate_counters(self, tree: SourceTree, grid: GasGrid, tgt_xyz, self_src=None, theta: float = 1.0,
                      prec="fp64"):
        import torch
        xyz = _xyz(tgt_xyz, self.device)
        n = xyz.shape[1]
        ss = None if self_src is None else _vec(self_src, self.device, torch.int64)
        out = np.zeros((n, 4), np.int64)
        self._enter(xyz, ss)
        self._check(lib().start_rate_counters(self._h, tree._h, grid._h, n, _ptr(xyz), _ptr(ss), float(theta),
                                              _prec(prec), out.ctypes.data_as(C.c_void_p)), "start_rate_counters")
        return out


def estimate_bytes(n_t, n_s, n_gas, grid_log2, prec="fp32c") -> int:
    return int(lib().start_estimate_bytes(int(n_t), int(n_s), int(n_gas), int(grid_log2), _prec(prec)))
