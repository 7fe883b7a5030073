"""Pins of the equilibrium checker (oracle/equilibrium.py) against what the
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
