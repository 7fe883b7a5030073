"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it pins.  None of them re-types the oracle's own
formulas: they use exact rational geometry, closed forms, printed numbers,
invariances and an independent brute force (tests/bruteforce.py).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from tests import bruteforce as BF

HERE = os.path.dirname(os.path.abspath(__file__))
KPC = 3.0856775814913673e21
SIGMA = 6.3e-18
ALPHA_B = 2.6e-13


def unit_box(size=1.0, unit=KPC, lo=(0.0, 0.0, 0.0)):
    return O.make_box(lo, size, unit)


def rand_pts(rng, n, size=1.0, lo=0.0):
    return np.ascontiguousarray(lo + rng.random((3, n)) * size)


def member_sets(tree_export):
    e = tree_export
    out = {}
    for i in range(len(e["level"])):
        key = (int(e["level"][i]),) + tuple(int(v) for v in e["coord"][i])
        mem = e["member_idx"][e["member_off"][i]: e["member_off"][i] + e["count"][i]]
        out[key] = tuple(sorted(int(v) for v in mem))
    return out


# ------------------------------------------------------------------ tree ---

@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (17, 2), (200, 3), (1000, 4)])
def test_tree_cells_equal_level_groups(n, seed):
    """Section 2.2.2: cubes split into 8 until one source is left.  Every cell
    of the oracle is exactly a group of sources sharing floor(u 2^n) at its
    level, and every such group exists."""
    rng = np.random.default_rng(seed)
    box = unit_box(6.6)
    xyz = rand_pts(rng, n, 6.6)
    lum = rng.uniform(0.5, 2.0, n)
    t = O.Tree(box, xyz, lum)
    got = member_sets(t.export())
    u = [BF.normalise([0, 0, 0], 6.6, xyz[:, j]) for j in range(n)]
    want = BF.cells_by_level(u)
    assert got == want


def test_tree_partition_and_moments():
    """Children partition the parent; leaves hold one source except level-21
    buckets; L = sum L_j (eq. 14) and r = sum L_j r_j / L (eq. 15) against
    correctly rounded sums (math.fsum)."""
    rng = np.random.default_rng(7)
    n = 3000
    xyz = rand_pts(rng, n, 6.6)
    lum = 10.0 ** rng.uniform(36, 50, n)
    t = O.Tree(unit_box(6.6), xyz, lum)
    e = t.export()
    sets = member_sets(e)
    for key, mem in sets.items():
        level = key[0]
        kids = [k for k in sets if k[0] == level + 1 and all((k[1 + a] >> 1) == key[1 + a] for a in range(3))]
        if len(mem) >= 2 and level < 21:
            assert sorted(j for k in kids for j in sets[k]) == list(mem)
        else:
            assert not kids
            assert len(mem) == 1 or level == 21
    for i in range(len(e["level"])):
        mem = e["member_idx"][e["member_off"][i]: e["member_off"][i] + e["count"][i]]
        L = math.fsum(lum[mem])
        assert e["lum"][i] == pytest.approx(L, rel=4e-16 * len(mem) + 1e-16)
        for k in range(3):
            c = math.fsum(lum[mem] * xyz[k, mem]) / L
            assert abs(e["com"][i, k] - c) <= (4e-16 * len(mem) + 2e-16) * 6.6


def test_tree_coincident_sources_bucket():
    """Coincident sources cannot be separated: subdivision stops at level 21
    and the bucket keeps all of them."""
    xyz = np.array([[1.0, 1.0, 1.0, 3.0], [2.0, 2.0, 2.0, 3.0], [3.0, 3.0, 3.0, 3.0]])
    t = O.Tree(unit_box(6.6), xyz, np.ones(4))
    sets = member_sets(t.export())
    assert max(k[0] for k in sets) == 21
    assert sets[max(sets, key=lambda k: (k[0], len(sets[k])))] == (0, 1, 2)


def test_tree_input_errors():
    box = unit_box(1.0)
    with pytest.raises(O.OracleError) as e:
        O.Tree(box, np.array([[0.5], [1.5], [0.5]]), np.ones(1))
    assert e.value.code == O.EOUTOFBOX
    with pytest.raises(O.OracleError) as e:
        O.Tree(box, np.array([[0.5], [np.nan], [0.5]]), np.ones(1))
    assert e.value.code == O.ENONFINITE
    with pytest.raises(O.OracleError) as e:
        O.Tree(box, np.array([[0.5], [0.5], [0.5]]), -np.ones(1))
    assert e.value.code == O.EINVAL
    assert O.Tree(box, np.zeros((3, 0)), np.zeros(0)).ncells == 0


# ------------------------------------------------------- opening criterion ---

def test_accept_matches_exact_geometry():
    """Eq. (12) with d the distance to the closest point of the cube: the FP64
    decision equals the exact rational one away from exact ties."""
    rng = np.random.default_rng(11)
    mism = 0
    for _ in range(4000):
        level = int(rng.integers(0, 8))
        coord = rng.integers(0, 2 ** level, 3)
        u = rng.random(3)
        theta = float(rng.choice([0.3, 0.5, 0.8, 1.0, 1.4]))
        mism += O.accept(level, coord, u, theta) != BF.accept_exact(level, coord, u, theta)
    assert mism == 0


def test_accept_on_equality_and_inside():
    """Eq. (12) uses <=: a cube of side 1/2 at distance exactly 1/2 passes at
    theta = 1; a point inside (d = 0) never passes."""
    assert O.accept(1, [0, 0, 0], [1.0, 0.25, 0.25], 1.0)
    assert not O.accept(1, [0, 0, 0], [1.0, 0.25, 0.25], 0.999)
    assert not O.accept(1, [0, 0, 0], [0.25, 0.25, 0.25], 100.0)
    assert not O.accept(3, [1, 1, 1], [0.125, 0.2, 0.25], 1e6)   # on the face


def test_accept_monotone_parent_child():
    """Eqs. (12)-(13) applied at every level: a child of a passing cell passes,
    so a top-down walk equals the level-by-level rule."""
    rng = np.random.default_rng(12)
    for _ in range(3000):
        level = int(rng.integers(0, 12))
        coord = rng.integers(0, 2 ** level, 3)
        u = rng.random(3)
        theta = float(rng.uniform(0.1, 1.5))
        if O.accept(level, coord, u, theta):
            for o in range(8):
                ch = [2 * coord[0] + (o >> 2 & 1), 2 * coord[1] + (o >> 1 & 1), 2 * coord[2] + (o & 1)]
                assert O.accept(level + 1, ch, u, theta)


# -------------------------------------------------------------------- walk ---

@pytest.mark.parametrize("n,theta,seed", [(2, 1.0, 1), (16, 0.5, 2), (16, 1.0, 3), (60, 0.8, 4),
                                          (150, 1.0, 5), (150, 1.4, 6), (150, 0.0, 7)])
def test_lists_equal_definition(n, theta, seed):
    """Interaction list = cells passing eq. (12) whose ancestors fail (eq. 13),
    plus single sources and failing level-21 buckets below no passing cell;
    the member sets partition all sources but the target's own."""
    rng = np.random.default_rng(seed)
    size = 6.6
    xyz = rand_pts(rng, n, size)
    lum = rng.uniform(0.0, 1.0, n)
    lum[rng.random(n) < 0.1] = 0.0
    tgt = np.concatenate([rand_pts(rng, 20, size), xyz[:, :5]], axis=1)
    self_src = np.array([-1] * 20 + list(range(min(5, n))) + [-1] * max(0, 5 - n), np.int64)
    tgt = tgt[:, : len(self_src)]
    t = O.Tree(unit_box(size), xyz, lum)
    cells = member_sets(t.export())
    off, ent = t.lists(tgt, self_src, theta)
    u_src = [BF.normalise([0, 0, 0], size, xyz[:, j]) for j in range(n)]
    groups = BF.cells_by_level(u_src)
    for i in range(tgt.shape[1]):
        got = []
        for e in ent[off[i]: off[i + 1]]:
            if e[0] < 0:
                got.append(frozenset([int(e[1])]))
            else:
                got.append(frozenset(cells[tuple(int(v) for v in e)]))
        u = BF.normalise([0, 0, 0], size, tgt[:, i])
        want = BF.interaction_sets(groups, lum, u, theta, int(self_src[i]))
        assert sorted(map(sorted, got)) == sorted(map(sorted, want))
        covered = [j for s in got for j in s]
        # each source is used at most once, never the target's own, and every
        # lit source is used
        assert len(covered) == len(set(covered))
        assert int(self_src[i]) not in covered
        lit = {j for j in range(n) if lum[j] > 0 and j != self_src[i]}
        assert lit <= set(covered)


def test_theta_zero_lists_every_source():
    """theta = 0: no cell passes eq. (12), every source is used individually,
    which is the method without the tree (section 2.2.2, last paragraph)."""
    rng = np.random.default_rng(21)
    xyz = rand_pts(rng, 300, 6.6)
    t = O.Tree(unit_box(6.6), xyz, np.ones(300))
    off, ent = t.lists(xyz[:, :10], np.arange(10), 0.0)
    for i in range(10):
        e = ent[off[i]: off[i + 1]]
        assert (e[:, 0] == -1).all()
        assert sorted(e[:, 1]) == [j for j in range(300) if j != i]


# -------------------------------------------------------------------- grid ---

def test_kernel_normalised():
    """Section 2.1 kernel: the 3-D integral of W over its support is 1."""
    from scipy.integrate import quad
    for h in (0.3, 1.0, 7.5):
        v, _ = quad(lambda r: 4 * math.pi * r * r * O.kernel_w(r, h), 0, 2 * h, points=[h], epsabs=0,
                    epsrel=1e-13)
        assert v == pytest.approx(1.0, rel=1e-11)
    assert O.kernel_w(2.0, 1.0) == 0.0 and O.kernel_w(2.5, 1.0) == 0.0
    assert O.kernel_w(0.0, 1.0) == pytest.approx(1.0 / math.pi, rel=1e-15)


def test_grid_single_particle_and_uniform():
    """Shepard interpolation reproduces a constant: one particle gives its own
    density wherever its kernel reaches, 0 elsewhere; uniform particles give
    the uniform value everywhere they cover."""
    box = unit_box(1.0)
    xyz = np.array([[0.3], [0.55], [0.61]])
    g = O.grid(box, xyz, np.array([0.11]), np.array([7.25e-3]), 4)
    G = 16
    cen = (np.arange(G) + 0.5) / G
    X, Y, Z = np.meshgrid(cen, cen, cen, indexing="ij")
    inside = np.sqrt((X - 0.3) ** 2 + (Y - 0.55) ** 2 + (Z - 0.61) ** 2) < 0.22
    assert np.allclose(g[inside], 7.25e-3, rtol=2e-16, atol=0)
    assert (g[~inside] == 0).all()
    rng = np.random.default_rng(3)
    xyz = rand_pts(rng, 500)
    g = O.grid(box, xyz, rng.uniform(0.05, 0.2, 500), np.full(500, 3e-4), 4)
    cov = g > 0
    assert cov.mean() > 0.99
    assert np.allclose(g[cov], 3e-4, rtol=1e-14, atol=0)


def test_grid_matches_all_pairs_bruteforce():
    """Binned evaluation equals the all-pairs sum bit for bit (zero terms add
    nothing) and equals an independent numpy evaluation to rounding."""
    rng = np.random.default_rng(5)
    box = unit_box(2.0, lo=(-1.0, -1.0, -1.0))
    xyz = rand_pts(rng, 700, 2.0, -1.0)
    h = rng.uniform(0.02, 0.3, 700)
    nhi = 10 ** rng.uniform(-6, -2, 700)
    g = O.grid(box, xyz, h, nhi, 4)
    cells = np.arange(16 ** 3)
    assert np.array_equal(O.grid_cells(box, xyz, h, nhi, 4, cells), g.reshape(-1))
    ref = BF.shepard_grid([-1, -1, -1], 2.0, 16, xyz, h, nhi)
    assert np.allclose(g, ref, rtol=1e-12, atol=0)


# ------------------------------------------------------------------ column ---

def test_column_axis_and_diagonal_single_cell():
    """A ray along an axis through one lit cell collects n * side; along the
    cell's body diagonal n * side * sqrt(3)."""
    box = unit_box(8.0)
    g = np.zeros((8, 8, 8))
    g[3, 4, 5] = 2.5e-3
    v, nc = O.column(box, 3, g, [0.2, 4.5, 5.5], [7.9, 4.5, 5.5])
    assert v == pytest.approx(2.5e-3, rel=1e-15)
    v, _ = O.column(box, 3, g, [3.0, 4.0, 5.0], [4.0, 5.0, 6.0])
    assert v == pytest.approx(2.5e-3 * math.sqrt(3), rel=1e-15)
    v, _ = O.column(box, 3, g, [0.5, 0.5, 0.5], [7.5, 0.5, 7.5])
    assert v == 0.0


def test_column_additive_symmetric_and_exact():
    """tau(a->c) = tau(a->b) + tau(b->c) for b on the segment, tau(a->b) =
    tau(b->a), and both equal the exact rational cell-by-cell clipping sum."""
    rng = np.random.default_rng(9)
    box = unit_box(6.6)
    G = 8
    g = 10 ** rng.uniform(-5, -2, (G, G, G))
    for _ in range(40):
        a = rng.random(3) * 6.6
        c = rng.random(3) * 6.6
        b = a + 0.375 * (c - a)
        ac, _ = O.column(box, 3, g, a, c)
        ab, _ = O.column(box, 3, g, a, b)
        bc, _ = O.column(box, 3, g, b, c)
        ca, _ = O.column(box, 3, g, c, a)
        assert ac == pytest.approx(ab + bc, rel=1e-13)
        assert ac == pytest.approx(ca, rel=1e-13)
        assert ac == pytest.approx(BF.column_exact([0, 0, 0], 6.6, G, g, a, c), rel=1e-13)


def test_column_endpoints_on_planes_and_faces():
    """Rays starting on grid planes or on the box faces (the star at the box
    centre sits on three planes) integrate the same field exactly."""
    box = unit_box(4.0)
    rng = np.random.default_rng(2)
    g = rng.uniform(0, 1e-3, (4, 4, 4))
    for a, b in [([2.0, 2.0, 2.0], [0.1, 3.9, 0.7]), ([0.0, 0.0, 0.0], [4.0, 4.0, 4.0]),
                 ([4.0, 1.0, 2.0], [0.0, 3.0, 2.0]), ([1.0, 1.0, 1.0], [3.0, 1.0, 1.0])]:
        v, _ = O.column(box, 2, g, a, b)
        assert v == pytest.approx(BF.column_exact([0, 0, 0], 4.0, 4, g, a, b), rel=1e-13)


def test_paper_printed_optical_depths():
    """Numbers printed in the paper (tests/golden/paper_numbers.json): the
    Stromgren radius of Test 1, about 20 and 0.2 optical depths per particle
    spacing in Tests 1 and 2, and the 51.4 pc mean free path of Test 6 --
    the latter three as columns through a uniform grid."""
    gold = json.load(open(os.path.join(HERE, "golden", "paper_numbers.json")))
    s = gold["stromgren_radius_test1"]
    rs = (3 * s["ndot_per_s"] / (4 * math.pi * s["n_h_cm3"] ** 2 * ALPHA_B)) ** (1 / 3) / KPC
    assert round(rs, 1) == s["value_kpc"]
    box = unit_box(132.0)
    for key in ("tau_per_spacing_test1", "tau_per_spacing_test2"):
        p = gold[key]
        g = np.full((4, 4, 4), p["n_h_cm3"])
        sp = p["box_kpc"] / p["particles_per_axis"]
        col, _ = O.column(box, 2, g, [10.0, 20.0, 30.0], [10.0 + sp, 20.0, 30.0])
        tau = SIGMA * col * KPC
        assert abs(tau - p["value"]) < 0.05 * p["value"]
    m = gold["mean_free_path_test6"]
    g = np.full((2, 2, 2), m["n_h_cm3"])
    col, _ = O.column(unit_box(1.0, unit=KPC), 1, g, [0.1, 0.2, 0.3], [0.1 + m["value_pc"] / 1000, 0.2, 0.3])
    assert SIGMA * col * KPC == pytest.approx(1.0, abs=1e-3)


# ------------------------------------------------------------------- rates ---

def _uniform_grid(G, n):
    return np.full((G, G, G), n)


def test_rate_single_source_uniform_gas():
    """One source in uniform gas: tau = n sigma d, Gamma = L sigma e^-tau / (4 pi d^2)
    for every theta (the tree method equals the plain one for N_s = 1)."""
    rng = np.random.default_rng(4)
    box = unit_box(6.6)
    n = 1e-3
    src = np.array([[1.1], [2.2], [3.3]])
    L = np.array([5e48])
    tgt = rand_pts(rng, 200, 6.6)
    t = O.Tree(box, src, L)
    d = np.sqrt(((tgt - src) ** 2).sum(axis=0)) * KPC
    want = L[0] * SIGMA * np.exp(-n * SIGMA * d) / (4 * math.pi * d ** 2)
    for theta in (0.0, 0.5, 1.0, 5.0):
        got = O.rates(t, 4, _uniform_grid(16, n), tgt, None, theta, SIGMA)
        assert np.allclose(got, want, rtol=1e-12, atol=0)


def test_rate_optically_thin_sum():
    """n_HI = 0: Gamma_i = sigma/(4 pi) sum_j L_j / d_ij^2; exact at theta = 0
    (the tree-free method), and the tree error shrinks with theta."""
    rng = np.random.default_rng(6)
    box = unit_box(6.6)
    src = rand_pts(rng, 400, 6.6)
    L = 10 ** rng.uniform(47, 50, 400)
    tgt = rand_pts(rng, 50, 6.6)
    t = O.Tree(box, src, L)
    want = np.array([SIGMA / (4 * math.pi) * math.fsum(
        L / (np.sqrt(((src - tgt[:, [i]]) ** 2).sum(axis=0)) * KPC) ** 2) for i in range(50)])
    g0 = O.rates(t, 3, np.zeros((8, 8, 8)), tgt, None, 0.0, SIGMA)
    assert np.allclose(g0, want, rtol=1e-13, atol=0)
    errs = [np.abs(O.rates(t, 3, np.zeros((8, 8, 8)), tgt, None, th, SIGMA) / want - 1).max()
            for th in (0.25, 0.5, 1.0)]
    assert errs[0] < errs[1] < errs[2] < 0.3


def test_rate_two_emitters_exclude_self():
    """Two emitters (section 4.1, eqs. 25-26): each particle gets only the
    other's photons, attenuated by the column between them."""
    box = unit_box(6.6)
    xyz = np.array([[1.0, 2.5], [3.0, 3.5], [3.0, 2.0]])
    L = np.array([2e42, 7e41])
    G = 8
    g = np.random.default_rng(1).uniform(0, 2e-3, (G, G, G))
    t = O.Tree(box, xyz, L)
    got = O.rates(t, 3, g, xyz, np.array([0, 1]), 1.0, SIGMA)
    d = math.dist(xyz[:, 0], xyz[:, 1]) * KPC
    col = BF.column_exact([0, 0, 0], 6.6, G, g, xyz[:, 1], xyz[:, 0])
    want0 = SIGMA * L[1] * math.exp(-SIGMA * col * KPC) / (4 * math.pi * d * d)
    col = BF.column_exact([0, 0, 0], 6.6, G, g, xyz[:, 0], xyz[:, 1])
    want1 = SIGMA * L[0] * math.exp(-SIGMA * col * KPC) / (4 * math.pi * d * d)
    assert got[0] == pytest.approx(want0, rel=1e-13)
    assert got[1] == pytest.approx(want1, rel=1e-13)


@pytest.mark.parametrize("seed", [1, 2])
def test_rate_theta_zero_equals_bruteforce(seed):
    """theta = 0 reduces to the method without the tree (section 2.2.2):
    compare with the independent brute force (exact rational columns)."""
    rng = np.random.default_rng(seed)
    size, G = 6.6, 8
    box = unit_box(size)
    src = rand_pts(rng, 12, size)
    L = 10 ** rng.uniform(47, 49, 12)
    gas = rand_pts(rng, 300, size)
    h = rng.uniform(0.3, 0.8, 300)
    nhi = 10 ** rng.uniform(-4, -3, 300)
    g = O.grid(box, gas, h, nhi, 3)
    tgt = np.concatenate([rand_pts(rng, 8, size), src[:, :3]], axis=1)
    self_src = np.array([-1] * 8 + [0, 1, 2])
    t = O.Tree(box, src, L)
    got = O.rates(t, 3, g, tgt, self_src, 0.0, SIGMA)
    for i in range(tgt.shape[1]):
        want = BF.gamma_brute([0, 0, 0], size, KPC, G, g, src, L, tgt[:, i], SIGMA, int(self_src[i]))
        assert got[i] == pytest.approx(want, rel=1e-12)


def test_invariances():
    """Permuting sources or targets, translating the box, and rescaling the
    length unit by a power of two leave the rates unchanged (to rounding of
    the moment sums); lists are unchanged up to source relabelling."""
    rng = np.random.default_rng(8)
    size = 6.6
    box = unit_box(size)
    src = rand_pts(rng, 200, size)
    L = 10 ** rng.uniform(40, 48, 200)
    gas = rand_pts(rng, 400, size)
    h = np.full(400, 0.6)
    nhi = 10 ** rng.uniform(-4, -3, 400)
    g = O.grid(box, gas, h, nhi, 3)
    tgt = rand_pts(rng, 40, size)
    base = O.rates(O.Tree(box, src, L), 3, g, tgt, None, 0.8, SIGMA)
    off0, ent0 = O.Tree(box, src, L).lists(tgt, None, 0.8)
    perm = rng.permutation(200)
    tp = O.Tree(box, src[:, perm], L[perm])
    assert np.allclose(O.rates(tp, 3, g, tgt, None, 0.8, SIGMA), base, rtol=1e-13, atol=0)
    offp, entp = tp.lists(tgt, None, 0.8)
    assert np.array_equal(off0, offp)
    src_rows = entp[:, 0] < 0
    entp[src_rows, 1] = perm[entp[src_rows, 1]]
    assert np.array_equal(ent0, entp)
    tperm = rng.permutation(40)
    got = O.rates(O.Tree(box, src, L), 3, g, tgt[:, tperm], None, 0.8, SIGMA)
    assert np.array_equal(got, base[tperm])
    # translation by an exactly representable offset
    sh = np.array([[-64.0], [128.0], [32.0]])
    boxs = O.make_box(sh[:, 0], size, KPC)
    gs = O.grid(boxs, gas + sh, h, nhi, 3)
    got = O.rates(O.Tree(boxs, src + sh, L), 3, gs, tgt + sh, None, 0.8, SIGMA)
    assert np.allclose(got, base, rtol=1e-10, atol=0)
    # unit change kpc -> kpc/1024
    boxu = O.make_box([0, 0, 0], size * 1024, KPC / 1024)
    gu = O.grid(boxu, gas * 1024, h * 1024, nhi, 3)
    assert np.array_equal(gu, g)
    got = O.rates(O.Tree(boxu, src * 1024, L), 3, gu, tgt * 1024, None, 0.8, SIGMA)
    assert np.allclose(got, base, rtol=1e-14, atol=0)
