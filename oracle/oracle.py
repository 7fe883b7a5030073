"""ctypes loader for the CPU FP64 oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the CPU-baseline
leg of the benchmark to produce the values the HIP library must reproduce.
It never serves the product path.  Every function follows the paper
(Hasegawa & Umemura 2010) as described in start_oracle.h.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB=liboracle_san.so loads the sanitizer build (build.sh sanitize)
_LIB_PATH = os.path.join(_HERE, os.environ.get("ORACLE_LIB", "liboracle.so"))

OK, EINVAL, ENOMEM, EOUTOFBOX, ENONFINITE, ECAPACITY = 0, -1, -2, -4, -5, -6


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


class _Box(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("size", C.c_double), ("unit_cm", C.c_double)]


def build(sanitize=False):
    subprocess.run(["sh", os.path.join(_HERE, "build.sh")] + (["sanitize"] if sanitize else []), check=True)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(sanitize=_LIB_PATH.endswith("_san.so"))
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        i64 = C.c_int64
        L.or_tree_build.argtypes = [P, i64, P, P, P]
        L.or_tree_free.argtypes = [P]
        L.or_tree_ncells.argtypes = [P]
        L.or_tree_ncells.restype = i64
        L.or_tree_export.argtypes = [P] * 9
        L.or_tree_kernel_luminosity.argtypes = [P, P, P, C.c_int]
        L.or_normalise.argtypes = [P, P, P]
        L.or_accept.argtypes = [C.c_int32, P, P, C.c_double]
        L.or_interaction_lists.argtypes = [P, i64, P, P, C.c_double, P, P, i64]
        L.or_kernel_w.argtypes = [C.c_double, C.c_double]
        L.or_kernel_w.restype = C.c_double
        L.or_grid_build.argtypes = [P, i64, P, P, P, C.c_int, P]
        L.or_grid_cells.argtypes = [P, i64, P, P, P, C.c_int, i64, P, P]
        L.or_column.argtypes = [P, C.c_int, P, P, P, P]
        L.or_column.restype = C.c_double
        L.or_rates.argtypes = [P, C.c_int, P, i64, P, P, C.c_double, C.c_double, P, P, C.c_int]
        L.or_fsh.argtypes = [C.c_double]
        L.or_fsh.restype = C.c_double
        L.or_lw_rates.argtypes = [P, C.c_int, P, i64, P, P, C.c_double, P, C.c_int]
        L.or_upstream_rates.argtypes = [P, C.c_int, P, i64, P, P, P, P, C.c_double, C.c_double, P, P, P, i64, P]
        L.or_upstream_rates_ex.argtypes = [P, C.c_int, P, i64, P, P, P, P, C.c_double, C.c_double, P, P, P, i64, P,
                                           C.c_int]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


def make_box(lo, size, unit_cm):
    b = _Box()
    for k in range(3):
        b.lo[k] = float(lo[k])
    b.size = float(size)
    b.unit_cm = float(unit_cm)
    return b


class Tree:
    """Octree over the sources (section 2.2.2) with virtual sources (eqs. 14-15)."""

    def __init__(self, box: _Box, xyz, lum):
        self.box = box
        self.xyz = _f64(xyz).reshape(3, -1)
        self.lum = _f64(lum)
        self.n = self.xyz.shape[1]
        h = C.c_void_p()
        _check(lib().or_tree_build(C.byref(box), self.n, _p(self.xyz), _p(self.lum), C.byref(h)),
               "or_tree_build")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().or_tree_free(h)
            self._h = None

    @property
    def ncells(self):
        return int(lib().or_tree_ncells(self._h))

    def export(self):
        m = self.ncells
        out = dict(level=np.zeros(m, np.int32), coord=np.zeros((m, 3), np.int64),
                   count=np.zeros(m, np.int64), nchild=np.zeros(m, np.int32),
                   lum=np.zeros(m), com=np.zeros((m, 3)), member_off=np.zeros(m, np.int64),
                   member_idx=np.zeros(max(self.n, 1), np.int64))
        _check(lib().or_tree_export(self._h, _p(out["level"]), _p(out["coord"]), _p(out["count"]),
                                    _p(out["nchild"]), _p(out["lum"]), _p(out["com"]),
                                    _p(out["member_off"]), _p(out["member_idx"])), "or_tree_export")
        out["member_idx"] = out["member_idx"][: self.n]
        return out

    def kernel_luminosity(self, h, vol=None, form=1):
        """Kernel-weighted cell luminosities (section 2.2.2, the two forms
        beside eq. (14)) at each cell's centre of luminosity; form 1 is the
        kernel-weighted mean, form 2 the volume-weighted SPH sum."""
        self._kh = _f64(h)
        self._kv = None if vol is None else _f64(vol)
        _check(lib().or_tree_kernel_luminosity(self._h, _p(self._kh), _p(self._kv), int(form)),
               "or_tree_kernel_luminosity")
        return self

    def lists(self, tgt_xyz, self_src=None, theta=1.0, capacity=None):
        """Per-target interaction lists: (offsets[n_t+1], entries[n, 4])."""
        tgt = _f64(tgt_xyz).reshape(3, -1)
        nt = tgt.shape[1]
        ss = None if self_src is None else np.ascontiguousarray(self_src, dtype=np.int64)
        offsets = np.zeros(nt + 1, np.int64)
        cap = capacity if capacity is not None else max(1, nt * 64)
        while True:
            ent = np.zeros((cap, 4), np.int64)
            rc = lib().or_interaction_lists(self._h, nt, _p(tgt), _p(ss), float(theta),
                                            _p(offsets), _p(ent), cap)
            if rc == ECAPACITY and capacity is None:
                cap = int(offsets[-1])
                continue
            _check(rc, "or_interaction_lists")
            return offsets, ent[: offsets[-1]]


def normalise(box, x):
    u = np.zeros(3)
    lib().or_normalise(C.byref(box), _p(_f64(x)), _p(u))
    return u


def accept(level, coord, u, theta):
    c = np.ascontiguousarray(coord, dtype=np.int64)
    return bool(lib().or_accept(int(level), _p(c), _p(_f64(u)), float(theta)))


def kernel_w(r, h):
    return lib().or_kernel_w(float(r), float(h))


def grid(box, xyz, h, nhi, grid_log2):
    """Shepard-normalised SPH n_HI at the G^3 cell centres, [G, G, G] (x, y, z)."""
    xyz = _f64(xyz).reshape(3, -1)
    G = 1 << grid_log2
    out = np.zeros(G ** 3)
    _check(lib().or_grid_build(C.byref(box), xyz.shape[1], _p(xyz), _p(_f64(h)), _p(_f64(nhi)),
                               int(grid_log2), _p(out)), "or_grid_build")
    return out.reshape(G, G, G)


def grid_cells(box, xyz, h, nhi, grid_log2, cells):
    xyz = _f64(xyz).reshape(3, -1)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros(cells.shape[0])
    _check(lib().or_grid_cells(C.byref(box), xyz.shape[1], _p(xyz), _p(_f64(h)), _p(_f64(nhi)),
                               int(grid_log2), cells.shape[0], _p(cells), _p(out)), "or_grid_cells")
    return out


def column(box, grid_log2, grid_values, a, b):
    """Column of n_HI along a->b (cm^-3 x length unit) and the number of cells crossed."""
    g = _f64(grid_values).reshape(-1)
    nc = np.zeros(1, np.int64)
    v = lib().or_column(C.byref(box), int(grid_log2), _p(g), _p(_f64(a)), _p(_f64(b)), _p(nc))
    return v, int(nc[0])


def rates(tree: Tree, grid_log2, grid_values, tgt_xyz, self_src=None, theta=1.0, sigma=6.3e-18,
          counters=False, nthreads=0):
    """Gamma per H I atom (s^-1) per target; optionally per-target counters
    [tests, entries, grid cells, zero-distance skips]."""
    tgt = _f64(tgt_xyz).reshape(3, -1)
    nt = tgt.shape[1]
    g = _f64(grid_values).reshape(-1)
    ss = None if self_src is None else np.ascontiguousarray(self_src, dtype=np.int64)
    out = np.zeros(nt)
    cnt = np.zeros((nt, 4), np.int64) if counters else None
    _check(lib().or_rates(tree._h, int(grid_log2), _p(g), nt, _p(tgt), _p(ss), float(theta),
                          float(sigma), _p(out), _p(cnt), int(nthreads)), "or_rates")
    return (out, cnt) if counters else out


def fsh(x):
    """H2 self-shielding function of Appendix B."""
    return lib().or_fsh(float(x))


def lw_rates(tree: Tree, grid_log2, grid_values, tgt_xyz, self_src=None, theta=1.0, nthreads=0):
    """H2 photodissociation rate (s^-1) per target (Appendix B): the tree holds
    Lyman-Werner luminosities (erg s^-1 Hz^-1), the grid n_H2 (cm^-3)."""
    tgt = _f64(tgt_xyz).reshape(3, -1)
    nt = tgt.shape[1]
    g = _f64(grid_values).reshape(-1)
    ss = None if self_src is None else np.ascontiguousarray(self_src, dtype=np.int64)
    out = np.zeros(nt)
    _check(lib().or_lw_rates(tree._h, int(grid_log2), _p(g), nt, _p(tgt), _p(ss), float(theta), _p(out),
                             int(nthreads)), "or_lw_rates")
    return out


def upstream_rates(tree: Tree, grid_log2, grid_values, xyz, h, nhi, self_src=None, theta=1.0, sigma=6.3e-18,
                   structure=False, all_pairs=False):
    """Gamma per particle with the upstream-particle chain optical depths of
    section 2.2.1 (the particles are the targets).  With structure=True also
    returns (offsets [n+1], parents [pairs] as upstream particle index or -1,
    stats [n, 2] = pairs, pairs integrated along the ray).  all_pairs: test
    every other particle as a neighbour (O(n^2)) instead of the cell list."""
    xyz = _f64(xyz).reshape(3, -1)
    n = xyz.shape[1]
    g = _f64(grid_values).reshape(-1)
    ss = None if self_src is None else np.ascontiguousarray(self_src, dtype=np.int64)
    out = np.zeros(n)
    offs = np.zeros(n + 1, np.int64)
    stats = np.zeros((n, 2), np.int64)
    cap = 0
    par = None
    if structure:
        # the pair count from the lists alone (returns ECAPACITY with the offsets)
        rc = lib().or_interaction_lists(tree._h, n, _p(xyz), _p(ss), float(theta), _p(offs), None, 0)
        if rc not in (OK, ECAPACITY):
            _check(rc, "or_interaction_lists")
        cap = int(offs[-1])
        par = np.zeros(max(cap, 1), np.int64)
    _check(lib().or_upstream_rates_ex(tree._h, int(grid_log2), _p(g), n, _p(xyz), _p(_f64(h)), _p(_f64(nhi)),
                                      _p(ss), float(theta), float(sigma), _p(out), _p(offs), _p(par), cap, _p(stats),
                                      int(bool(all_pairs))),
           "or_upstream_rates")
    return (out, offs, par[:cap], stats) if structure else out
