"""Pins of the oracle's H2 photodissociation rate (Appendix B): the
self-shielding function, one source in uniform H2 gas (closed form for any
theta), the unshielded limit (pure inverse-square sum), and theta = 0 against
an independent brute force with exact columns."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests import bruteforce as BF

KPC = 3.0856775814913673e21


def box(size):
    return O.make_box([0.0, 0.0, 0.0], size, KPC)


def test_fsh_values():
    assert O.fsh(0.0) == 1.0 and O.fsh(1.0) == 1.0
    assert O.fsh(16.0) == 0.125                 # 16^(-3/4) = 2^-3
    assert O.fsh(1e4) == pytest.approx(1e-3, rel=1e-15)
    # continuous at the shielding threshold
    assert O.fsh(1.0 + 1e-12) == pytest.approx(1.0, abs=1e-11)


def test_lw_single_source_uniform_h2():
    """One source in uniform n_H2: N = n d, k = 1.13e8 L / (4 pi d^2)
    f_sh(n d / 1e14), for any theta (one source: no tree error)."""
    rng = np.random.default_rng(14)
    size = 6.6
    n = 1e-8
    src = np.array([[1.1], [2.2], [3.3]])
    L = np.array([3e24])
    tgt = rng.random((3, 300)) * size
    t = O.Tree(box(size), src, L)
    d = np.sqrt(((tgt - src) ** 2).sum(axis=0)) * KPC
    N = n * d
    fsh = np.where(N <= 1e14, 1.0, (N / 1e14) ** -0.75)
    want = 1.13e8 * L[0] / (4 * math.pi * d ** 2) * fsh
    assert (N > 1e14).any() and (N <= 1e14).any()      # both branches of f_sh
    for theta in (0.0, 0.7, 3.0):
        got = O.lw_rates(t, 4, np.full((16, 16, 16), n), tgt, None, theta)
        assert np.allclose(got, want, rtol=1e-12, atol=0)


def test_lw_unshielded_is_inverse_square_sum():
    rng = np.random.default_rng(15)
    size = 6.6
    src = rng.random((3, 200)) * size
    L = 10 ** rng.uniform(23, 25, 200)
    tgt = rng.random((3, 30)) * size
    t = O.Tree(box(size), src, L)
    got = O.lw_rates(t, 3, np.full((8, 8, 8), 1e-12), tgt, None, 0.0)   # N far below 1e14
    for i in range(30):
        d = np.sqrt(((src - tgt[:, [i]]) ** 2).sum(axis=0)) * KPC
        want = 1.13e8 / (4 * math.pi) * math.fsum(L / d ** 2)
        assert got[i] == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("seed", [3, 4])
def test_lw_theta_zero_equals_bruteforce(seed):
    rng = np.random.default_rng(seed)
    size, G = 6.6, 8
    src = rng.random((3, 10)) * size
    L = 10 ** rng.uniform(23, 25, 10)
    gas = rng.random((3, 300)) * size
    h = rng.uniform(0.3, 0.8, 300)
    nh2 = 10 ** rng.uniform(-7, -5, 300)
    g = O.grid(box(size), gas, h, nh2, 3)
    tgt = np.concatenate([rng.random((3, 6)) * size, src[:, :2]], axis=1)
    self_src = np.array([-1] * 6 + [0, 1])
    t = O.Tree(box(size), src, L)
    got = O.lw_rates(t, 3, g, tgt, self_src, 0.0)
    for i in range(tgt.shape[1]):
        terms = []
        for j in range(src.shape[1]):
            if j == self_src[i]:
                continue
            d = math.dist(src[:, j], tgt[:, i]) * KPC
            N = BF.column_exact([0, 0, 0], size, G, g, src[:, j], tgt[:, i]) * KPC
            f = 1.0 if N <= 1e14 else (N / 1e14) ** -0.75
            terms.append(L[j] / (4 * math.pi * d * d) * f)
        want = 1.13e8 * math.fsum(terms)
        assert got[i] == pytest.approx(want, rel=1e-12)
