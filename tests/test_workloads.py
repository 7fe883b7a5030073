"""The seeded input generators (test infrastructure shared by the oracle and
the HIP path): reproducible draws, the constants and distributions of the
benchmark configurations, and smoothing lengths against a brute-force
neighbour search.  A slip here would pass parity and still measure the wrong
problem."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_1005_5312_amd import workloads as W

KPC = W.KPC_CM


@pytest.mark.parametrize("maker,kw", [(W.make_small, dict(n_gas=1000, n_src=8)),
                                      (W.make_clumpy, dict(n_gas=1000, n_src=16)),
                                      (W.make_diffuse, dict(n_gas=1000)),
                                      (W.make_shadow, dict(n_gas=1000)),
                                      (W.make_lw, dict(n_gas=1000, n_src=16))])
def test_seeds_reproduce(maker, kw):
    a, b, c = maker(seed=7, **kw), maker(seed=7, **kw), maker(seed=8, **kw)
    for f in ("gas_xyz", "gas_h", "gas_nhi", "src_xyz", "src_lum", "tgt_xyz"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert not np.array_equal(a.gas_xyz, c.gas_xyz)
    assert a.gas_xyz.dtype == np.float64 and a.gas_xyz.flags.c_contiguous and a.gas_xyz.shape == (3, 1000)


def test_smoothing_lengths_are_the_32nd_neighbour_by_brute_force():
    rng = np.random.default_rng(3)
    for xyz in (rng.random((3, 400)) * 6.6, np.concatenate([rng.normal(1, 0.05, (3, 200)),
                                                            rng.random((3, 200)) * 6.6], axis=1)):
        h = W.smoothing_lengths(np.ascontiguousarray(xyz))
        d = np.sqrt(((xyz[:, :, None] - xyz[:, None, :]) ** 2).sum(axis=0))
        np.fill_diagonal(d, np.inf)
        want = np.sort(d, axis=1)[:, 31] / 2.0          # 32nd nearest other particle
        assert np.allclose(h, want, rtol=1e-14, atol=0)


def test_small_configuration():
    w = W.make_small()
    assert w.n_gas == 4096 and w.n_src == 16 and w.grid_log2 == 4
    assert w.box_size == 6.6 and np.all(w.box_lo == 0) and w.length_unit_cm == KPC
    assert np.all(w.src_lum == 5e48) and np.all(w.gas_nhi == 1e-3)
    assert w.self_src is None and w.tgt_xyz is w.gas_xyz
    assert w.gas_xyz.min() >= 0 and w.gas_xyz.max() < 6.6


def test_clumpy_configuration():
    """Lognormal n_H with sigma_ln = 1 and mean 1e-3, x_HI uniform in
    [0.5, 1], 1024 sources log-uniform in 1e47-1e50, G = 64."""
    w = W.make_clumpy()
    assert w.n_gas == 1 << 18 and w.n_src == 1024 and w.grid_log2 == 6
    g = np.log(w.gas_nh / 1e-3) + 0.5
    assert abs(g.mean()) < 0.01 and abs(g.std() - 1.0) < 0.01
    assert stats.kstest(g, "norm").pvalue > 1e-3
    assert abs(w.gas_nh.mean() / 1e-3 - 1.0) < 0.02
    x = w.gas_nhi / w.gas_nh
    assert x.min() >= 0.5 and x.max() <= 1.0
    assert stats.kstest((x - 0.5) / 0.5, "uniform").pvalue > 1e-3
    lg = np.log10(w.src_lum)
    assert lg.min() >= 47.0 and lg.max() <= 50.0
    assert stats.kstest((lg - 47.0) / 3.0, "uniform").pvalue > 1e-3


def test_diffuse_configuration():
    """2^20 emitters plus the star: alpha_B n_e n_p V with V = box / N gives
    ~2.09e42 photons/s inside the HII sphere (r < 0.3 box) and ~2.1e36
    outside (x_HII = 1e-3), ~2.5e47 in all; the 1e50 star at the centre is
    source 2^20; every target's own source is itself; G = 128."""
    w = W.make_diffuse()
    n = 1 << 20
    assert w.n_gas == n and w.n_src == n + 1 and w.grid_log2 == 7
    assert np.array_equal(w.self_src, np.arange(n))
    assert np.array_equal(w.src_xyz[:, :n], w.gas_xyz)
    assert np.all(w.src_xyz[:, n] == 3.3) and w.src_lum[n] == 1e50
    r = np.sqrt(((w.gas_xyz - 3.3) ** 2).sum(axis=0))
    inside = r < 0.3 * 6.6
    lin, lout = w.src_lum[:n][inside], w.src_lum[:n][~inside]
    assert np.all(lin == lin[0]) and np.all(lout == lout[0])
    assert abs(lin[0] / 2.09e42 - 1) < 0.005 and abs(lout[0] / 2.09e36 - 1) < 0.005
    assert abs(lin[0] / lout[0] - 1e6) < 1e-3                  # (x_HII inside / outside)^2
    assert abs(w.src_lum[:n].sum() / 2.5e47 - 1) < 0.02
    assert abs(inside.mean() - 4 / 3 * math.pi * 0.3 ** 3) < 0.002
    assert np.all(w.gas_nhi[inside] == 0.0)
    assert np.allclose(w.gas_nhi[~inside], 0.999e-3, rtol=1e-15)


def test_shadow_clumps():
    """16 clumps of 200x density and radius 0.05 box, centres in the +x
    hemisphere 0.1-0.3 box from the star, neutral (x_HII = 1e-3); elsewhere
    as the diffuse configuration."""
    w = W.make_shadow(n_gas=1 << 17)
    L = 6.6
    c = w.meta["clump_centres"]
    star = w.meta["star"]
    assert c.shape == (3, 16) and np.all(star == 3.3)
    d = np.sqrt(((c - star[:, None]) ** 2).sum(axis=0))
    assert np.all(d >= 0.1 * L - 1e-12) and np.all(d <= 0.3 * L + 1e-12)
    assert np.all(c[0] >= star[0])
    dc = np.sqrt(((w.gas_xyz[:, :, None] - c[:, None, :]) ** 2).sum(axis=0)).min(axis=1)
    in_clump = dc < 0.05 * L
    assert in_clump.sum() > 0
    assert np.all(w.gas_nh[in_clump] == 0.2) and np.all(w.gas_nh[~in_clump] == 1e-3)
    assert np.allclose(w.gas_nhi[in_clump], 0.2 * 0.999, rtol=1e-15)
    r = np.sqrt(((w.gas_xyz - 3.3) ** 2).sum(axis=0))
    hii = (r < 0.3 * L) & ~in_clump
    assert np.all(w.gas_nhi[hii] == 0.0)
    assert np.allclose(w.gas_nhi[~hii & ~in_clump], 0.999e-3, rtol=1e-15)
    # emitters follow the local state: dense neutral clump gas emits
    # alpha_B (1e-3 x 0.2)^2 V
    vol = (L * KPC) ** 3 / w.n_gas
    assert np.allclose(w.src_lum[:w.n_gas][in_clump], W.ALPHA_B * (1e-3 * 0.2) ** 2 * vol, rtol=1e-14)


def test_grid_sizes_follow_the_particle_count():
    assert [W.auto_grid_log2(n) for n in (4096, 1 << 18, 1 << 20, 1 << 21)] == [4, 6, 7, 7]
    assert W.auto_grid_log2(1 << 14) == 5 and W.auto_grid_log2(1) == 1


def test_sample_indices():
    a = W.sample_indices(1000, 100, 3)
    assert np.array_equal(a, W.sample_indices(1000, 100, 3))
    assert len(np.unique(a)) == 100 and np.all(np.diff(a) > 0) and a.min() >= 0 and a.max() < 1000
    assert len(W.sample_indices(10, 100, 3)) == 10
