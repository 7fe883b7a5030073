"""Shared helpers for the GPU parity tests (test infrastructure)."""
from __future__ import annotations

import functools
import math

import numpy as np

from oracle import oracle as O
from paper_1005_5312_amd import workloads as W

KPC = W.KPC_CM
FLOOR = 1e-30          # s^-1: below it compare absolutely
ABS_FLOOR = 2e-34
TOL_FP64 = 1e-5
TOL_FP32C = 2e-4


def morton_keys(xyz, lo, size):
    """Morton key by definition: 21-bit quantised normalised coordinates,
    interleaved with x in the most significant position of each triple."""
    inv = 1.0 / size
    u = np.minimum((xyz - np.asarray(lo, dtype=np.float64)[:, None]) * inv, 1.0)
    q = np.minimum(np.floor(u * 2.0 ** 21), 2 ** 21 - 1).astype(np.uint64)
    key = np.zeros(xyz.shape[1], np.uint64)
    one = np.uint64(1)
    for b in range(21):
        bb = np.uint64(b)
        key |= ((q[0] >> bb) & one) << np.uint64(3 * b + 2)
        key |= ((q[1] >> bb) & one) << np.uint64(3 * b + 1)
        key |= ((q[2] >> bb) & one) << np.uint64(3 * b)
    return key


def gpu_entries_as_cells(ent, geo):
    """GPU list entries -> oracle entry rows (level, c0, c1, c2) / (-1, j, 0, 0)."""
    out = np.zeros((len(ent), 4), np.int64)
    cell = ent >= 0
    g = geo[ent[cell]]
    out[cell, 0] = g[:, 3] & 0xFF
    out[cell, 1:4] = g[:, :3]
    out[~cell, 0] = -1
    out[~cell, 1] = -ent[~cell] - 1
    return out


def rel_errors(got, want, floor=FLOOR):
    """max relative error above the floor and max absolute error below it."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    big = np.abs(want) >= floor
    rel = np.abs(got[big] - want[big]) / np.abs(want[big]) if big.any() else np.zeros(1)
    ab = np.abs(got[~big] - want[~big]) if (~big).any() else np.zeros(1)
    return float(rel.max()), float(ab.max()), int(big.sum())


@functools.lru_cache(maxsize=None)
def workload(name, **kw):
    return W.make(name, **kw)


def box_of(w):
    from paper_1005_5312_amd import Box
    return Box(tuple(float(v) for v in w.box_lo), float(w.box_size), float(w.length_unit_cm))


def obox_of(w):
    return O.make_box(w.box_lo, w.box_size, w.length_unit_cm)


class OracleCase:
    """Oracle tree and grid for one workload (built once)."""

    def __init__(self, w):
        self.w = w
        self.box = obox_of(w)
        self.tree = O.Tree(self.box, w.src_xyz, w.src_lum)
        self.grid = O.grid(self.box, w.gas_xyz, w.gas_h, w.gas_nhi, w.grid_log2)

    def rates(self, theta, idx=None):
        tgt = self.w.tgt_xyz if idx is None else self.w.tgt_xyz[:, idx]
        ss = self.w.self_src
        if ss is not None and idx is not None:
            ss = ss[idx]
        return O.rates(self.tree, self.w.grid_log2, self.grid, tgt, ss, theta, self.w.sigma)


@functools.lru_cache(maxsize=None)
def oracle_case(name):
    return OracleCase(workload(name))


def fsum_rate(terms):
    return math.fsum(terms)
