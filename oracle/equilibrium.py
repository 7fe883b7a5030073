"""Photoionisation equilibrium on top of the rate oracle.

TEST INFRASTRUCTURE ONLY: the plain CPU FP64 definition that the HIP
library's equilibrium update and equilibrium loop are compared against.  It
shares no code with the HIP library; it calls only the oracle in oracle.py.

Physics (pure hydrogen, static gas, fixed temperature):

* A particle with total hydrogen density n_H, neutral fraction x and
  photoionisation rate per H I atom Gamma is in equilibrium when the
  ionisations per unit volume, n_HI Gamma = x n_H Gamma (Appendix A, eq. A1
  with eq. A2 for one frequency), balance the recombinations
  alpha n_e n_p = alpha (1 - x)^2 n_H^2, with n_e = n_p = (1 - x) n_H.  Under
  the on-the-spot approximation (section 2.1) alpha is the case-B
  coefficient alpha_B.
* The rates depend on x through the optical depths (n_HI = x n_H along every
  ray), so the field is found by fixed-point iteration: n_HI -> gas grid ->
  Gamma -> x -> n_HI ...  Starting from a neutral medium the iterates
  decrease monotonically (more neutral gas means more absorption, smaller
  Gamma and a larger equilibrium x), so the loop converges from above to the
  equilibrium whose ionised volume the Stromgren radius of eq. (17)
  describes.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def neutral_fraction(gamma, n_h, alpha):
    """Equilibrium neutral fraction x in [0, 1] of  x Gamma = alpha n_H (1 - x)^2.

    With a = alpha n_H the balance is the quadratic a x^2 - (2a + Gamma) x + a = 0.
    Its two roots multiply to 1, so the one in [0, 1] is the reciprocal of the
    larger root:  x = 2a / (2a + Gamma + sqrt(Gamma (Gamma + 4a))).
    No ionisation and no recombination (a = Gamma = 0) leaves the gas neutral
    (x = 1)."""
    g = np.asarray(gamma, dtype=np.float64)
    a = alpha * np.asarray(n_h, dtype=np.float64)
    den = 2.0 * a + g + np.sqrt(g * (g + 4.0 * a))
    with np.errstate(invalid="ignore", divide="ignore"):
        x = np.where(den > 0.0, 2.0 * a / den, 1.0)
    return x


def ionization_equilibrium(box, tree, gas_xyz, gas_h, n_h, x_init, grid_log2, theta, sigma, alpha,
                           max_iter=100, tol=1e-4, history=False):
    """Fixed-point iteration of the equilibrium field around the sources of
    `tree`, with the gas particles as targets.

    Each iteration grids n_HI = x n_H (section 2.1 kernel), evaluates Gamma for
    every particle through the tree (eqs. 12-15, A2) and replaces x by
    neutral_fraction(Gamma).  Stops after the first iteration whose largest
    change |x_new - x| is <= tol, or after max_iter iterations.

    Returns (x, gamma, iterations, last_change[, list of x after each
    iteration]); gamma is the rate field the final x was computed from."""
    x = np.array(x_init, dtype=np.float64, copy=True)
    n_h = np.asarray(n_h, dtype=np.float64)
    hist = []
    change = np.inf
    it = 0
    gamma = None
    while it < max_iter:
        it += 1
        g = O.grid(box, gas_xyz, gas_h, x * n_h, grid_log2)
        gamma = O.rates(tree, grid_log2, g, gas_xyz, None, theta, sigma)
        x_new = neutral_fraction(gamma, n_h, alpha)
        change = float(np.max(np.abs(x_new - x))) if x.size else 0.0
        x = x_new
        if history:
            hist.append(x.copy())
        if change <= tol:
            break
    out = (x, gamma, it, change)
    return out + (hist,) if history else out


def ionised_volume_radius(x, volume_cm3):
    """Radius (cm) of the sphere whose volume equals the ionised volume
    sum_i (1 - x_i) V_i."""
    v = float(np.sum((1.0 - np.asarray(x)) * np.asarray(volume_cm3)))
    return (3.0 * v / (4.0 * np.pi)) ** (1.0 / 3.0)


def photoionisations(x, gamma, n_h, volume_cm3):
    """Photoionisations per second in the whole box, sum_i x_i n_H,i Gamma_i V_i."""
    return float(np.sum(np.asarray(x) * np.asarray(n_h) * np.asarray(gamma) * np.asarray(volume_cm3)))


# ---------------------------------------------------------------------------
# Transfer of recombination photons (section 4.1)
# ---------------------------------------------------------------------------

def recombination_emission(n_h, x, volume_cm3, alpha_1):
    """Recombination photons per second emitted by each particle, eq. (19):
    alpha_1 n_e n_p V with n_e = n_p = (1 - x) n_H and alpha_1 = alpha_A -
    alpha_B the coefficient of recombinations to the ground state."""
    ne = (1.0 - np.asarray(x, dtype=np.float64)) * np.asarray(n_h, dtype=np.float64)
    return alpha_1 * ne * ne * np.asarray(volume_cm3, dtype=np.float64)


def self_optical_depth(n_h, x, volume_cm3, sigma):
    """Optical depth from the edge to the centre of a particle, eq. (28):
    sigma n_HI (3 V / (4 pi))^(1/3)."""
    nhi = np.asarray(x, dtype=np.float64) * np.asarray(n_h, dtype=np.float64)
    return sigma * nhi * np.cbrt(3.0 * np.asarray(volume_cm3, dtype=np.float64) / (4.0 * np.pi))


def k_self(n_h, x, volume_cm3, sigma, alpha_1):
    """Ionisations per unit volume and time by a particle's own recombination
    photons, eq. (30) for one frequency (from eqs. 27-29 with a flat source
    function): alpha_1 n_e n_p (1 - exp(-tau)), with
    1 - exp(-tau) evaluated as -expm1(-tau) (no cancellation at small tau)."""
    ne = (1.0 - np.asarray(x, dtype=np.float64)) * np.asarray(n_h, dtype=np.float64)
    tau = self_optical_depth(n_h, x, volume_cm3, sigma)
    return alpha_1 * ne * ne * (-np.expm1(-tau))


def k_ion_total(gamma_other, n_h, x, k_self_values):
    """Eq. (25): k_ion = k_self + k_other, with k_other = n_HI Gamma (eq. 26,
    Gamma the rate per H I atom from every other emitter, eq. A2)."""
    return np.asarray(x, dtype=np.float64) * np.asarray(n_h, dtype=np.float64) * \
        np.asarray(gamma_other, dtype=np.float64) + np.asarray(k_self_values, dtype=np.float64)


def effective_recombination(n_h, x, volume_cm3, sigma, alpha_a, alpha_1):
    """With the transfer of recombination photons every recombination (alpha_A)
    counts, and a particle's own ground-state photons reionise it at the rate
    k_self of eq. (30).  Taking k_self's optical depth from the previous
    iterate, k_ion = alpha_A n_e n_p becomes x n_H Gamma = alpha_eff n_H^2 (1-x)^2
    with alpha_eff = alpha_A - alpha_1 (1 - exp(-tau_self)), which tends to
    alpha_B = alpha_A - alpha_1 where the gas is opaque (the statement after
    eq. 30)."""
    tau = self_optical_depth(n_h, x, volume_cm3, sigma)
    return alpha_a - alpha_1 * (-np.expm1(-tau))


def diffuse_equilibrium(box, gas_xyz, gas_h, n_h, volume_cm3, star_xyz, star_lum, x_init, grid_log2, theta, sigma,
                        alpha_a, alpha_1, max_iter=100, tol=1e-4):
    """Equilibrium with the transfer of recombination photons (section 4.1):
    every particle emits alpha_1 n_e n_p V (eq. 19) from its position, the
    stars their own photons; each iteration builds the source tree of the
    particles and stars, grids n_HI = x n_H, evaluates Gamma of every
    particle from every other emitter (self excluded, eqs. 25-26) and solves
    x Gamma = alpha_eff n_H (1 - x)^2 (effective_recombination).  Stops as
    ionization_equilibrium does.  Returns (x, gamma, iterations, last_change)."""
    x = np.array(x_init, dtype=np.float64, copy=True)
    n = x.size
    n_h = np.asarray(n_h, dtype=np.float64)
    src = np.ascontiguousarray(np.concatenate([np.asarray(gas_xyz, dtype=np.float64),
                                               np.asarray(star_xyz, dtype=np.float64).reshape(3, -1)], axis=1))
    self_src = np.arange(n, dtype=np.int64)
    change, it, gamma = np.inf, 0, None
    while it < max_iter:
        it += 1
        lum = np.concatenate([recombination_emission(n_h, x, volume_cm3, alpha_1), np.asarray(star_lum, float)])
        tree = O.Tree(box, src, lum)
        g = O.grid(box, gas_xyz, gas_h, x * n_h, grid_log2)
        gamma = O.rates(tree, grid_log2, g, gas_xyz, self_src, theta, sigma)
        x_new = neutral_fraction(gamma, n_h, effective_recombination(n_h, x, volume_cm3, sigma, alpha_a, alpha_1))
        change = float(np.max(np.abs(x_new - x))) if n else 0.0
        x = x_new
        if change <= tol:
            break
    return x, gamma, it, change
