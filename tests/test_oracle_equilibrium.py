"""Pins of the equilibrium oracle (oracle/equilibrium.py) against what the
mathematics and the paper fix: the closed-form root, its limits, the order
property of the iteration, and the Stromgren radius of Test 4 (section 4.2.1,
eq. 17: 5.4 kpc for 5e48 photons/s in n_H = 1e-3 cm^-3)."""
import math

import numpy as np
import pytest

from oracle import equilibrium as E
from oracle import oracle as O
from paper_1005_5312_amd import workloads as W


def test_root_at_gamma_equal_a_is_the_golden_section():
    # (1 - x)^2 = x  =>  x = (3 - sqrt 5) / 2
    for a in (1e-20, 2.6e-16, 3.0):
        x = E.neutral_fraction(a, a / 2.6e-13, 2.6e-13)
        assert abs(x - (3.0 - math.sqrt(5.0)) / 2.0) <= 4e-16


def test_limits():
    alpha = 2.6e-13
    # no radiation: fully neutral; no gas and no radiation: neutral by convention
    assert E.neutral_fraction(0.0, 1e-3, alpha) == 1.0
    assert E.neutral_fraction(0.0, 0.0, alpha) == 1.0
    # radiation but no recombination: fully ionised
    assert E.neutral_fraction(1e-12, 0.0, alpha) == 0.0
    # strong field: x = eps (1 - x)^2 with eps = a / Gamma has the series
    # x = sum_k (-1)^k C_k eps^(k+1), C_k the Catalan numbers 1, 2, 5, 14, ...
    catalan = [1, 1, 2, 5, 14, 42, 132, 429, 1430]
    for eps in (1e-3, 1e-6, 1e-9, 1e-15):
        a = alpha * 1e-3
        x = E.neutral_fraction(a / eps, 1e-3, alpha)
        series = sum((-1) ** k * catalan[k + 1] * eps ** (k + 1) for k in range(8))
        assert abs(x - series) <= 1e-14 * series


def test_root_against_the_textbook_formula_in_60_digits():
    """The smaller root of a x^2 - (2a + Gamma) x + a = 0 by the plain
    quadratic formula, evaluated with 60 significant digits (where its
    cancellation is harmless), over rates spanning 14 decades."""
    import decimal
    decimal.getcontext().prec = 60
    D = decimal.Decimal
    rng = np.random.default_rng(7)
    g = 10.0 ** rng.uniform(-22, -8, 400)
    nh = 10.0 ** rng.uniform(-6, 2, 400)
    alpha = 2.6e-13
    x = E.neutral_fraction(g, nh, alpha)
    assert np.all((x > 0) & (x <= 1))
    for gi, ni, xi in zip(g, nh, x):
        a = D(alpha) * D(float(ni))
        b = 2 * a + D(float(gi))
        want = (b - (b * b - 4 * a * a).sqrt()) / (2 * a)
        assert abs(D(float(xi)) - want) <= D("4e-16") * want


def test_order_in_the_rate():
    rng = np.random.default_rng(8)
    g = 10.0 ** rng.uniform(-22, -8, 20000)
    nh = 10.0 ** rng.uniform(-6, 2, 20000)
    alpha = 2.6e-13
    x = E.neutral_fraction(g, nh, alpha)
    # larger rate, less neutral gas
    x2 = E.neutral_fraction(g * 1.001, nh, alpha)
    assert np.all(x2 <= x)


@pytest.mark.slow
def test_stromgren_radius_of_test4():
    """One 5e48 photons/s source at the centre of a 13.2 kpc box of uniform
    n_H = 1e-3: from a neutral start the iterates fall monotonically; the
    converged ionised volume is a sphere of radius within 5% of the 5.4 kpc
    printed for this test, and the photoionisations in the box account for
    the source's photons within 10%."""
    e = W.make_stromgren(n_gas=1 << 18, grid_log2=6)
    w = e.work
    box = O.make_box(w.box_lo, w.box_size, w.length_unit_cm)
    tree = O.Tree(box, w.src_xyz, w.src_lum)
    x, gam, it, ch, hist = E.ionization_equilibrium(box, tree, w.gas_xyz, w.gas_h, e.n_h, e.x_init, w.grid_log2,
                                                    1.0, w.sigma, e.alpha_b, max_iter=200, tol=1e-4,
                                                    history=True)
    assert ch <= 1e-4 and it < 200
    for k in range(len(hist) - 1):
        assert np.all(hist[k + 1] <= hist[k] + 1e-15)
    r_eq = E.ionised_volume_radius(x, e.volume_cm3) / W.KPC_CM
    assert abs(r_eq / 5.4 - 1.0) <= 0.05, r_eq
    # the generator's constants reproduce the printed radius itself
    assert abs(e.stromgren_radius_cm(1e-3) / W.KPC_CM - 5.4) <= 0.05
    ph = E.photoionisations(x, gam, e.n_h, e.volume_cm3)
    assert abs(ph / w.src_lum.sum() - 1.0) <= 0.10, ph / w.src_lum.sum()
    # ionised inside, neutral outside
    r = np.sqrt(((w.gas_xyz - 0.5 * w.box_size) ** 2).sum(axis=0))
    assert np.mean(x[r < 3.0]) < 0.02 and np.mean(x[r > 6.2]) > 0.99


def test_iterates_fall_monotonically_small():
    """The order property on a coarse case with several sources: each
    iterate is <= the previous one everywhere."""
    w = W.make_small(seed=3, n_gas=2048, n_src=8)
    box = O.make_box(w.box_lo, w.box_size, w.length_unit_cm)
    tree = O.Tree(box, w.src_xyz, w.src_lum)
    nh = np.full(w.n_gas, 1e-3)
    x0 = np.ones(w.n_gas)
    _, _, it, _, hist = E.ionization_equilibrium(box, tree, w.gas_xyz, w.gas_h, nh, x0, w.grid_log2, 0.5,
                                                 w.sigma, W.ALPHA_B, max_iter=12, tol=0.0, history=True)
    assert it == 12
    assert np.all(hist[0] <= x0)
    for k in range(len(hist) - 1):
        assert np.all(hist[k + 1] <= hist[k] + 1e-15)


# --- recombination photons: eq. (19), eqs. (27)-(30), eq. (25) -------------

def test_k_self_closed_form_equals_the_transfer_integral():
    """Eq. (27) with the constant one-frequency source function of eq. (29),
    S / (h nu) = alpha_1 n_e n_p / (4 pi n_HI sigma), integrated numerically
    over tau' in [0, tau], equals the closed form of eq. (30)."""
    from scipy.integrate import quad
    alpha_1, sigma = 1.58e-13, 6.3e-18
    for n_h, x, vol in ((1e-3, 0.5, 1e60), (1.0, 0.01, 3e55), (1e-2, 0.9, 7.2e60), (1e-3, 1e-3, 1e58)):
        ne = (1 - x) * n_h
        nhi = x * n_h
        tau = E.self_optical_depth(n_h, x, vol, sigma)
        s_over_hnu = alpha_1 * ne * ne / (4 * math.pi * nhi * sigma)
        val, _ = quad(lambda tp: s_over_hnu * sigma * math.exp(-tau + tp), 0.0, tau, epsabs=0, epsrel=1e-13)
        want = 4 * math.pi * nhi * val
        got = float(E.k_self(n_h, x, vol, sigma, alpha_1))
        assert abs(got - want) <= 1e-11 * want, (got, want)


def test_k_self_limits_and_self_depth():
    alpha_1, sigma = 1.58e-13, 6.3e-18
    # V of a sphere of radius R: tau = sigma n_HI R exactly
    R = 2.5e20
    vol = 4.0 / 3.0 * math.pi * R ** 3
    assert abs(float(E.self_optical_depth(1e-3, 0.4, vol, sigma)) / (sigma * 4e-4 * R) - 1) <= 1e-15
    # very opaque: every recombination photon is absorbed in place, k_self =
    # alpha_1 n_e n_p (the limit stated after eq. 30)
    k = float(E.k_self(10.0, 0.5, vol, sigma, alpha_1))
    assert k == alpha_1 * 25.0
    # optically thin: k_self = alpha_1 n_e n_p tau to first order
    k = float(E.k_self(1e-9, 0.5, vol, sigma, alpha_1))
    tau = sigma * 0.5e-9 * R
    assert abs(k / (alpha_1 * (0.5e-9) ** 2 * tau) - 1) <= 1e-6
    # no neutral gas: nothing to absorb; fully neutral: nothing to emit
    assert float(E.k_self(1e-3, 0.0, vol, sigma, alpha_1)) == 0.0
    assert float(E.k_self(1e-3, 1.0, vol, sigma, alpha_1)) == 0.0


def test_emission_and_total_rate():
    alpha_1 = 1.58e-13
    n = 1000
    rng = np.random.default_rng(3)
    x = rng.random(n)
    nh = 10.0 ** rng.uniform(-4, 0, n)
    vol = 10.0 ** rng.uniform(55, 62, n)
    em = E.recombination_emission(nh, x, vol, alpha_1)
    assert np.allclose(em, alpha_1 * ((1 - x) * nh) ** 2 * vol, rtol=1e-15, atol=0)
    g = 10.0 ** rng.uniform(-20, -10, n)
    ks = E.k_self(nh, x, vol, 6.3e-18, alpha_1)
    kt = E.k_ion_total(g, nh, x, ks)
    assert np.allclose(kt, x * nh * g + ks, rtol=1e-15, atol=0)


def test_opaque_medium_total_rate_is_alpha_1_ne_np():
    """The statement after eq. (30): in a medium opaque everywhere, k_self +
    k_other = alpha_1 n_e n_p, i.e. the net recombination coefficient is
    alpha_B.  Uniform gas of 4096 particles in a 1 kpc box at n_H = 1, x = 0.5
    (tau from edge to centre of a particle ~380): k_other from every other
    particle's emission through the tree is negligible, except between the
    few random pairs much closer than the mean spacing."""
    w = W.make_small(seed=4, n_gas=4096, n_src=1)
    L = 1.0
    gas = w.gas_xyz / w.box_size * L
    from paper_1005_5312_amd.workloads import smoothing_lengths
    h = smoothing_lengths(gas)
    box = O.make_box(np.zeros(3), L, W.KPC_CM)
    nh = np.full(w.n_gas, 1.0)
    x = np.full(w.n_gas, 0.5)
    vol = np.full(w.n_gas, (L * W.KPC_CM) ** 3 / w.n_gas)
    alpha_1, sigma = 1.58e-13, 6.3e-18
    lum = E.recombination_emission(nh, x, vol, alpha_1)
    tree = O.Tree(box, gas, lum)
    g = O.grid(box, gas, h, x * nh, 4)
    gam = O.rates(tree, 4, g, gas, np.arange(w.n_gas), 1.0, sigma)
    kt = E.k_ion_total(gam, nh, x, E.k_self(nh, x, vol, sigma, alpha_1))
    r = kt / (alpha_1 * 0.25) - 1.0
    assert np.all(r >= -1e-15) and np.all(r <= 0.01)
    assert np.mean(np.abs(r) <= 1e-12) >= 0.99


# --- equilibrium with the transfer of recombination photons ---------------

def test_effective_recombination_limits():
    """alpha_eff = alpha_A - alpha_1 (1 - e^-tau): alpha_B where the particle
    is opaque to its own photons, alpha_A where it is transparent."""
    aA, a1 = 4.18e-13, 1.58e-13
    vol = 1e60
    assert E.effective_recombination(10.0, 0.5, vol, 6.3e-18, aA, a1) == aA - a1
    assert E.effective_recombination(1e-3, 0.0, vol, 6.3e-18, aA, a1) == aA
    t = float(E.self_optical_depth(1e-3, 0.5, vol, 6.3e-18))
    want = aA - a1 * (1 - math.exp(-t))
    assert abs(float(E.effective_recombination(1e-3, 0.5, vol, 6.3e-18, aA, a1)) - want) <= 1e-15 * want


def test_diffuse_loop_without_ground_state_photons_is_the_plain_loop():
    """alpha_1 = 0: no particle emits and alpha_eff = alpha_A, so the loop is
    the on-the-spot loop with alpha = alpha_A (the particles sit in the tree
    with zero luminosity and are left out of the lists): identical x."""
    e = W.make_stromgren(n_gas=1 << 12, grid_log2=4)
    w = e.work
    box = O.make_box(w.box_lo, w.box_size, w.length_unit_cm)
    xd, gd, itd, chd = E.diffuse_equilibrium(box, w.gas_xyz, w.gas_h, e.n_h, e.volume_cm3, w.src_xyz, w.src_lum,
                                             e.x_init, 4, 1.0, w.sigma, 4.18e-13, 0.0, max_iter=8, tol=0.0)
    tree = O.Tree(box, w.src_xyz, w.src_lum)
    xo, go, ito, cho = E.ionization_equilibrium(box, tree, w.gas_xyz, w.gas_h, e.n_h, e.x_init, 4, 1.0, w.sigma,
                                                4.18e-13, max_iter=8, tol=0.0)
    assert itd == ito == 8
    assert np.array_equal(xd, xo) and np.array_equal(gd, go)


def test_diffuse_loop_in_an_opaque_medium_is_the_case_b_loop():
    """The statement after eq. (30): where every particle is opaque to its own
    recombination photons the transfer of those photons reduces to case B.
    2048 particles in a 1 kpc box at n_H = 1 (optical depth from a
    particle's edge to its centre ~960 x), 32 stars of 5e44 photons/s each
    placed 0.5 pc from a particle, which they ionise in part (x down to ~0.07,
    still > 60 optical depths), theta = 0.  The converged diffuse loop
    (alpha_A, alpha_1 > 0; every particle an emitter) equals the on-the-spot
    loop with alpha_B = alpha_A - alpha_1 (the other particles' photons are
    absorbed before they reach a neighbour); with alpha_A instead it does
    not, so the comparison has power."""
    w = W.make_small(seed=4, n_gas=2048, n_src=1)
    size = 1.0
    gas = np.ascontiguousarray(w.gas_xyz / w.box_size * size)
    h = W.smoothing_lengths(gas)
    box = O.make_box(np.zeros(3), size, W.KPC_CM)
    n = w.n_gas
    nh = np.full(n, 1.0)
    vol = np.full(n, (size * W.KPC_CM) ** 3 / n)
    rng = np.random.default_rng(8)
    pick = rng.choice(n, 32, replace=False)
    v = rng.normal(size=(3, 32))
    v /= np.linalg.norm(v, axis=0)
    stars = np.ascontiguousarray(np.clip(gas[:, pick] + v * 0.5e-3, 0.0, size))
    slum = np.full(32, 5e44)
    aA, a1, sigma = 4.18e-13, 1.58e-13, 6.3e-18
    x0 = np.ones(n)
    xd, _, itd, chd = E.diffuse_equilibrium(box, gas, h, nh, vol, stars, slum, x0, 4, 0.0, sigma, aA, a1,
                                            max_iter=60, tol=1e-11)
    tree = O.Tree(box, stars, slum)
    xb, _, itb, chb = E.ionization_equilibrium(box, tree, gas, h, nh, x0, 4, 0.0, sigma, aA - a1,
                                               max_iter=60, tol=1e-11)
    xa, _, _, _ = E.ionization_equilibrium(box, tree, gas, h, nh, x0, 4, 0.0, sigma, aA, max_iter=60, tol=1e-11)
    assert chd <= 1e-11 and chb <= 1e-11
    tau = E.self_optical_depth(nh, xd, vol, sigma)
    assert tau.min() >= 40.0                        # opaque everywhere, also at the ionised particles
    assert int((xd < 0.9).sum()) >= 20              # not the trivial all-neutral state
    assert np.max(np.abs(xd - xb)) <= 1e-12
    assert np.max(np.abs(xd - xa)) >= 1e-2
