"""Independent brute-force evaluations for tiny inputs (test infrastructure).

These do not share code or algorithms with the oracle in ``oracle/``:

* cells of the source octree are found by grouping sources on
  floor(u 2^n) at every level n (no recursion);
* the opening test of eqs. (12)-(13) is decided in exact rational arithmetic
  with the closest point of the cube found by clamping;
* the optical depth is the sum over every grid cell of n_cell times the exact
  length of the segment inside that cell, found by slab clipping in rationals
  (instead of sorting plane crossings).
"""
from __future__ import annotations

import math
from fractions import Fraction as F

import numpy as np

MAX_LEVEL = 21


def normalise(lo, size, x):
    """Same input convention as the library: u = min((x - lo) / size, 1)."""
    inv = 1.0 / size
    return [min((x[k] - lo[k]) * inv, 1.0) for k in range(3)]


def cells_by_level(u_all):
    """All cells of the octree of section 2.2.2, grouped level by level.

    Returns dict (level, cx, cy, cz) -> sorted tuple of member indices.  A
    level-(n+1) group exists when its level-n parent has >= 2 members."""
    n = len(u_all)
    cells = {}
    if n == 0:
        return cells
    parents = {(0, 0, 0, 0): tuple(range(n))}
    cells.update(parents)
    for level in range(1, MAX_LEVEL + 1):
        nxt = {}
        for key, mem in parents.items():
            if len(mem) < 2:
                continue
            for j in mem:
                c = tuple(int(math.floor(u_all[j][k] * 2.0 ** level)) for k in range(3))
                c = tuple(min(v, 2 ** level - 1) for v in c)
                nxt.setdefault((level,) + c, []).append(j)
        parents = {k: tuple(sorted(v)) for k, v in nxt.items()}
        cells.update(parents)
        if not parents:
            break
    return cells


def accept_exact(level, coord, u, theta):
    """Eq. (12) in exact arithmetic: l^2 <= theta^2 d^2, d = distance from u to
    the closest point of the closed cube (clamping)."""
    level = int(level)
    l = F(1, 2 ** level)
    d2 = F(0)
    for k in range(3):
        lo = F(int(coord[k]), 2 ** level)
        hi = F(int(coord[k]) + 1, 2 ** level)
        uk = F(float(u[k]))
        p = min(max(uk, lo), hi)
        d2 += (uk - p) ** 2
    th = F(float(theta))
    return l * l <= th * th * d2


def interaction_sets(cells, lum, u, theta, self_idx=-1):
    """Entries of one target, each as a frozenset of source indices: cells that
    pass eq. (12) with no passing ancestor (eq. 13); single sources and the
    members of a failing level-21 group with no passing ancestor."""
    out = []
    keys = sorted(cells, key=lambda k: k[0])

    def ancestors(key):
        level, c = key[0], key[1:]
        for up in range(1, level + 1):
            yield (level - up,) + tuple(v >> up for v in c)

    passing = {}
    for key in keys:
        mem = cells[key]
        if len(mem) >= 2:
            passing[key] = accept_exact(key[0], key[1:], u, theta)
    for key in keys:
        mem = cells[key]
        if any(passing.get(a, False) for a in ancestors(key)):
            continue
        if len(mem) == 1:
            j = mem[0]
            if j != self_idx and lum[j] > 0:
                out.append(frozenset([j]))
        elif passing[key]:
            # the same member set may appear at several levels (single-child
            # chains); only the top-most passing one is reached
            if sum(lum[j] for j in mem) > 0:
                out.append(frozenset(mem))
        elif key[0] == MAX_LEVEL:
            out.extend(frozenset([j]) for j in mem if j != self_idx and lum[j] > 0)
    return out


def segment_cell_length(A, B, cell, G):
    """Exact parameter length of {t in [0,1] : A + t (B - A) in cell} (slab clipping).

    Along an axis the ray does not move on, the ray belongs to the cell
    floor(A) (clamped to the grid): a ray lying in a grid plane takes the
    cells on its upper side."""
    t0, t1 = F(0), F(1)
    for k in range(3):
        lo, hi = F(cell[k]), F(cell[k] + 1)
        d = B[k] - A[k]
        if d == 0:
            if min(max(math.floor(A[k]), 0), G - 1) != cell[k]:
                return F(0)
            continue
        ta, tb = (lo - A[k]) / d, (hi - A[k]) / d
        if ta > tb:
            ta, tb = tb, ta
        t0, t1 = max(t0, ta), min(t1, tb)
        if t1 <= t0:
            return F(0)
    return t1 - t0


def column_exact(lo, size, G, grid, a, b):
    """Column of the piecewise-constant field along a->b: |b-a| sum_cells n_c len_c.

    Cells are those of the closed unit cubes [i, i+1]; a piece on a shared face
    has zero length, so the sum is the exact integral."""
    s = F(G) / F(size)
    A = [(F(a[k]) - F(lo[k])) * s for k in range(3)]
    B = [(F(b[k]) - F(lo[k])) * s for k in range(3)]
    rng = []
    for k in range(3):
        lo_k = max(0, math.floor(min(A[k], B[k])) - 1)
        hi_k = min(G - 1, math.floor(max(A[k], B[k])) + 1)
        rng.append(range(lo_k, hi_k + 1))
    total = F(0)
    for i in rng[0]:
        for j in rng[1]:
            for k in rng[2]:
                ln = segment_cell_length(A, B, (i, j, k), G)
                if ln:
                    total += F(float(grid[i, j, k])) * ln
    return float(total) * math.dist(a, b)


def shepard_grid(lo, size, G, xyz, h, nhi):
    """Shepard-normalised cubic-spline interpolant at cell centres (numpy, all pairs)."""
    delta = size / G
    ax = [lo[k] + (np.arange(G) + 0.5) * delta for k in range(3)]
    X, Y, Z = np.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
    cen = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    r = np.sqrt(((cen[:, None, :] - xyz.T[None, :, :]) ** 2).sum(axis=2))
    q = r / h[None, :]
    f = np.where(q <= 1, 1 - 1.5 * q ** 2 + 0.75 * q ** 3, np.where(q <= 2, 0.25 * (2 - q) ** 3, 0.0))
    w = f / (np.pi * h[None, :] ** 3)
    den = w.sum(axis=1)
    num = (w * nhi[None, :]).sum(axis=1)
    out = np.where(den > 0, num / np.where(den > 0, den, 1), 0.0)
    return out.reshape(G, G, G)


def gamma_brute(lo, size, unit_cm, G, grid, src_xyz, lum, tgt, sigma, self_idx=-1):
    """Rate per H I atom from every source individually (theta = 0)."""
    tot = 0.0
    terms = []
    for j in range(src_xyz.shape[1]):
        if j == self_idx or lum[j] <= 0:
            continue
        a = src_xyz[:, j]
        d = math.dist(a, tgt)
        if d == 0:
            continue
        tau = sigma * column_exact(lo, size, G, grid, a, tgt) * unit_cm
        terms.append(lum[j] * math.exp(-tau) / (d * unit_cm) ** 2)
    tot = math.fsum(terms)
    return sigma / (4 * math.pi) * tot
