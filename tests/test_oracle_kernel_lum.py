"""Pins of the oracle's kernel-weighted cell luminosities (section 2.2.2: the
two SPH-kernel forms offered beside the sum of eq. (14)).

Form 1 is the kernel-weighted mean of the members' luminosities, form 2 the
SPH sum with the members' volumes m_j / rho_j; both are evaluated at the
cell's centre of luminosity (eq. 15) with each member's own smoothing length.
The pins use closed forms of the cubic spline at chosen q, the partition of
unity of the SPH sum on a lattice, the bounds of a weighted mean, cells whose
members' kernels do not reach the centre, and a brute force over cubes found
by geometry.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O

KPC = 3.0856775814913673e21


def unit_box():
    return O.make_box((0.0, 0.0, 0.0), 1.0, KPC)


def cells(tree):
    e = tree.export()
    out = []
    for i in range(len(e["level"])):
        mem = e["member_idx"][e["member_off"][i]: e["member_off"][i] + e["count"][i]]
        out.append((int(e["level"][i]), tuple(int(v) for v in e["coord"][i]), np.array(mem), e["lum"][i],
                    e["com"][i]))
    return out


def spline(q):
    """Cubic spline shape of section 2.1 as a piecewise polynomial in (2 - q)
    and (1 - q): 0.25 (2 - q)^3 - (1 - q)^3 inside q <= 1."""
    q = np.asarray(q, dtype=np.float64)
    return 0.25 * np.maximum(2.0 - q, 0.0) ** 3 - np.maximum(1.0 - q, 0.0) ** 3


def test_two_sources_closed_form():
    # L = 2 at x = 1/4 and L = 1 at x = 5/8 share only the root cube; their
    # centre of luminosity is x = 3/8, 1/8 and 1/4 from them.  With h = 1/4
    # and 1/6 the spline is read at q = 1/2 (f = 23/32) and q = 3/2 (f = 1/32),
    # so W = f / (pi h^3) = 46 / pi and 27 / (4 pi).
    xyz = np.array([[0.25, 0.625], [0.5, 0.5], [0.5, 0.5]])
    lum = np.array([2.0, 1.0])
    h = np.array([0.25, 1.0 / 6.0])
    vol = np.array([0.1, 0.2])
    for form, want in [(1, (2 * 46 + 6.75) / (46 + 6.75)), (2, (0.1 * 2 * 46 + 0.2 * 6.75) / math.pi)]:
        t = O.Tree(unit_box(), xyz, lum).kernel_luminosity(h, vol, form)
        multi = [c for c in cells(t) if len(c[2]) >= 2]
        assert len(multi) == 1 and multi[0][0] == 0
        assert np.allclose(multi[0][4], [0.375, 0.5, 0.5], rtol=0, atol=1e-16)
        assert abs(multi[0][3] - want) <= 1e-14 * want


def test_equal_luminosities_mean_form_keeps_them():
    # a weighted mean of equal values is that value, whatever the weights
    rng = np.random.default_rng(11)
    n = 300
    xyz = rng.random((3, n))
    lum = np.full(n, 3e48)
    h = rng.uniform(0.6, 1.0, n)   # every kernel reaches every point of the box
    t = O.Tree(unit_box(), xyz, lum).kernel_luminosity(h, None, 1)
    for level, coord, mem, L, com in cells(t):
        assert abs(L - 3e48) <= 1e-14 * 3e48, (level, coord)


def test_mean_form_lies_between_reaching_members():
    rng = np.random.default_rng(12)
    n = 500
    xyz = rng.random((3, n))
    lum = 10.0 ** rng.uniform(45.0, 50.0, n)
    h = 10.0 ** rng.uniform(-3.0, -1.0, n)
    t = O.Tree(unit_box(), xyz, lum).kernel_luminosity(h, None, 1)
    zero = reach = 0
    for level, coord, mem, L, com in cells(t):
        if len(mem) < 2:
            assert L == lum[mem[0]]   # a single source is used as itself
            continue
        d = np.sqrt(((xyz[:, mem] - com[:, None]) ** 2).sum(axis=0))
        reaching = d < 2.0 * h[mem]
        if not reaching.any():
            assert L == 0.0
            zero += 1
        else:
            lo, hi = lum[mem][reaching].min(), lum[mem][reaching].max()
            assert lo * (1 - 1e-14) <= L <= hi * (1 + 1e-14)
            reach += 1
    assert zero > 0 and reach > 0


def test_volume_form_is_a_partition_of_unity_on_a_lattice():
    # On a lattice of spacing a with V = a^3 and h = 2a the SPH sum
    # sum_j V W(|r - r_j|, h) is 1 to better than 1e-4, so form 2 returns the
    # common luminosity for every cube whose members fill the kernel's support
    # around its centre (half-side >= 2h: the root and the 8 level-1 cubes).
    k = 16
    a = 1.0 / k
    g = (np.arange(k) + 0.5) * a
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    n = xyz.shape[1]
    L0 = 7e47
    h = np.full(n, 2.0 * a)
    t = O.Tree(unit_box(), xyz, np.full(n, L0)).kernel_luminosity(h, np.full(n, a ** 3), 2)
    inner = 0
    for level, coord, mem, L, com in cells(t):
        if len(mem) < 2:
            continue
        centre = (np.array(coord) + 0.5) * 2.0 ** -level
        assert np.allclose(com, centre, rtol=0, atol=1e-13)
        if 0.5 * 2.0 ** -level >= 2.0 * h[0]:
            assert abs(L / L0 - 1.0) <= 1e-3, (level, coord, L / L0)
            inner += 1
        else:
            assert L < 0.99 * L0   # members no longer fill the support
    assert inner == 9


def test_narrow_kernels_leave_multi_source_cells_dark():
    rng = np.random.default_rng(13)
    n = 200
    xyz = rng.random((3, n))
    lum = rng.uniform(1e47, 1e48, n)
    h = np.full(n, 1e-7)
    for form in (1, 2):
        t = O.Tree(unit_box(), xyz, lum).kernel_luminosity(h, np.full(n, 1e-3), form)
        for level, coord, mem, L, com in cells(t):
            assert L == (0.0 if len(mem) >= 2 else lum[mem[0]])


def test_brute_force_over_cubes():
    # members of every cube found by geometry, centre of luminosity and both
    # forms summed directly
    rng = np.random.default_rng(14)
    n = 40
    xyz = rng.random((3, n))
    lum = rng.uniform(1.0, 5.0, n)
    h = rng.uniform(0.05, 0.3, n)
    vol = rng.uniform(1e-4, 1e-3, n)
    for form in (1, 2):
        t = O.Tree(unit_box(), xyz, lum).kernel_luminosity(h, vol, form)
        for level, coord, mem, L, com in cells(t):
            side = 2.0 ** -level
            inside = np.all((xyz >= np.array(coord)[:, None] * side) & (xyz < (np.array(coord)[:, None] + 1) * side),
                            axis=0)
            j = np.nonzero(inside)[0]
            assert np.array_equal(np.sort(mem), j)
            if len(j) < 2:
                continue
            r = (xyz[:, j] * lum[j]).sum(axis=1) / lum[j].sum()
            q = np.sqrt(((xyz[:, j] - r[:, None]) ** 2).sum(axis=0)) / h[j]
            w = spline(q) / (math.pi * h[j] ** 3)
            want = (lum[j] * w).sum() / w.sum() if form == 1 else (vol[j] * lum[j] * w).sum()
            if form == 1 and w.sum() == 0.0:
                want = 0.0
            assert abs(L - want) <= 1e-12 * abs(want) + 1e-300, (level, coord)


def test_repeat_and_switch_forms():
    rng = np.random.default_rng(15)
    n = 120
    xyz = rng.random((3, n))
    lum = rng.uniform(1.0, 2.0, n)
    h = rng.uniform(0.05, 0.5, n)
    vol = rng.uniform(1e-3, 1e-2, n)
    t = O.Tree(unit_box(), xyz, lum)
    once = [c[3] for c in cells(t.kernel_luminosity(h, vol, 1))]
    after_two = [c[3] for c in cells(t.kernel_luminosity(h, vol, 2).kernel_luminosity(h, vol, 1))]
    assert once == after_two


def test_theta_zero_rates_do_not_see_cells():
    # at theta = 0 every source is used as itself, so the cells' luminosities
    # cannot change Gamma
    rng = np.random.default_rng(16)
    n = 64
    xyz = rng.random((3, n))
    lum = rng.uniform(1e47, 1e48, n)
    tgt = rng.random((3, 50))
    grid = np.full(8 ** 3, 1e-3)
    plain = O.Tree(unit_box(), xyz, lum)
    kern = O.Tree(unit_box(), xyz, lum).kernel_luminosity(rng.uniform(0.05, 0.2, n), None, 1)
    a = O.rates(plain, 3, grid, tgt, None, 0.0, 6.3e-18)
    b = O.rates(kern, 3, grid, tgt, None, 0.0, 6.3e-18)
    assert np.array_equal(a, b)
    c = O.rates(kern, 3, grid, tgt, None, 1.0, 6.3e-18)
    assert not np.array_equal(a, c)


def test_bad_arguments():
    xyz = np.array([[0.2, 0.7], [0.5, 0.5], [0.5, 0.5]])
    lum = np.array([1.0, 1.0])
    t = O.Tree(unit_box(), xyz, lum)
    with pytest.raises(O.OracleError) as e:
        t.kernel_luminosity(np.array([0.1, 0.0]), None, 1)
    assert e.value.code == O.EINVAL
    with pytest.raises(O.OracleError) as e:
        t.kernel_luminosity(np.array([0.1, np.nan]), None, 1)
    assert e.value.code == O.ENONFINITE
    with pytest.raises(O.OracleError) as e:
        t.kernel_luminosity(np.array([0.1, 0.1]), None, 2)
    assert e.value.code == O.EINVAL
    with pytest.raises(O.OracleError) as e:
        t.kernel_luminosity(np.array([0.1, 0.1]), np.array([1.0, -1.0]), 2)
    assert e.value.code == O.EINVAL
    with pytest.raises(O.OracleError) as e:
        t.kernel_luminosity(np.array([0.1, 0.1]), None, 3)
    assert e.value.code == O.EINVAL
