"""Seeded synthetic inputs shaped like the test problems of START
(Hasegawa & Umemura 2010, MNRAS 407, 2632).

This module only draws input data: particle and source positions, smoothing
lengths, neutral-hydrogen densities and source photon rates.  It holds none of
the rate computation, so the HIP path and the CPU oracle can both consume it.

All arrays are float64, positions in structure-of-arrays layout ``[3, N]``,
lengths in kpc with ``length_unit_cm`` converting to cm.

Workloads (sizes of the paper's tests, drawn synthetically; no simulation data
from the paper is available):

* ``small``     4096 particles, 16 sources of 5e48 photons/s in a uniform
  neutral medium (n_H = 1e-3 cm^-3), the setting of Test 1 (section 3.1.1).
* ``clumpy``    2^18 particles with i.i.d. lognormal density and neutral
  fraction in [0.5, 1]; 1024 sources with log-uniform rates 1e47-1e50.
* ``diffuse``   2^20 particles, every particle a recombination emitter
  (section 4.1, eq. 19 with the case-B coefficient) inside a spherical HII
  region of radius 0.3 box, plus a central 1e50 photons/s star.
* ``shadow``    2^21 particles as ``diffuse`` plus 16 dense neutral clumps of
  200x overdensity and radius 0.05 box in one hemisphere around the star
  (the shadowing setting of Test 6, section 4.2.3).

* ``lw``        H2 photodissociation by the Lyman-Werner band (Appendix B):
  lognormal gas as ``clumpy`` with H2 fractions 10^U[-7, -3] of n_H and
  sources of 10^U[23, 25] erg s^-1 Hz^-1 in the band (``src_lum`` holds the
  Lyman-Werner luminosities, ``gas_nh2`` the H2 densities).

Equilibrium problems (``make_stromgren``) add the total hydrogen density of
each particle and an initial neutral fraction: one 5e48 photons/s source at
the centre of a 13.2 kpc box of uniform gas with n_H = 1e-3 cm^-3, the
setting of Test 4 (section 4.2.1), whose Stromgren radius is 5.4 kpc (eq. 17).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

KPC_CM = 3.0856775814913673e21     # 1 kpc in cm
SIGMA_HI = 6.3e-18                 # H I cross-section at the Lyman limit, cm^2
ALPHA_B = 2.6e-13                  # case-B recombination coefficient, cm^3 s^-1
BOX_KPC = 6.6                      # box side for all workloads (Test 4 scale)
N_NEIGHBOURS = 32                  # smoothing length: 2h = distance to 32nd neighbour


@dataclasses.dataclass
class Workload:
    name: str
    box_lo: np.ndarray          # (3,) float64
    box_size: float             # cube side, in length units
    length_unit_cm: float
    gas_xyz: np.ndarray         # (3, N_gas) float64
    gas_h: np.ndarray           # (N_gas,) float64 smoothing lengths
    gas_nhi: np.ndarray         # (N_gas,) float64 neutral hydrogen density, cm^-3
    src_xyz: np.ndarray         # (3, N_s)
    src_lum: np.ndarray         # (N_s,) ionizing photons per second
    tgt_xyz: np.ndarray         # (3, N_t) targets (the gas particles)
    self_src: np.ndarray | None  # (N_t,) int64 source index of the target itself, -1 = none
    thetas: tuple
    grid_log2: int
    sigma: float = SIGMA_HI
    gas_nh2: np.ndarray | None = None   # (N_gas,) H2 density, cm^-3 (Lyman-Werner workloads)
    gas_nh: np.ndarray | None = None    # (N_gas,) total hydrogen density, cm^-3, where drawn
    meta: dict = dataclasses.field(default_factory=dict)   # drawn geometry (centres, radii)

    @property
    def n_gas(self):
        return self.gas_xyz.shape[1]

    @property
    def n_src(self):
        return self.src_xyz.shape[1]

    @property
    def n_tgt(self):
        return self.tgt_xyz.shape[1]


def smoothing_lengths(xyz: np.ndarray, k: int = N_NEIGHBOURS) -> np.ndarray:
    """h such that 2h is the distance to the k-th nearest other particle."""
    from scipy.spatial import cKDTree
    pts = np.ascontiguousarray(xyz.T)
    n = pts.shape[0]
    kk = min(k, n - 1)
    if kk < 1:
        return np.full(n, 0.5, dtype=np.float64)
    d, _ = cKDTree(pts).query(pts, k=kk + 1, workers=-1)
    return np.ascontiguousarray(d[:, kk] * 0.5)


def _uniform_positions(rng, n, size):
    return np.ascontiguousarray(rng.random((3, n)) * size)


def auto_grid_log2(n_particles: int) -> int:
    """G = 2^ceil(log2(N^(1/3))): about one gas particle per grid cell."""
    if n_particles <= 1:
        return 1
    return max(1, int(math.ceil(math.log2(round(n_particles ** (1.0 / 3.0), 9)))))


def make_small(seed: int = 1, n_gas: int = 4096, n_src: int = 16) -> Workload:
    rng = np.random.default_rng(seed)
    L = BOX_KPC
    gas = _uniform_positions(rng, n_gas, L)
    src = _uniform_positions(rng, n_src, L)
    lum = np.full(n_src, 5e48)
    nhi = np.full(n_gas, 1e-3)
    return Workload("small", np.zeros(3), L, KPC_CM, gas, smoothing_lengths(gas), nhi,
                    src, lum, gas, None, (0.0, 0.5, 1.0), auto_grid_log2(n_gas), gas_nh=nhi.copy())


def make_clumpy(seed: int = 2, n_gas: int = 1 << 18, n_src: int = 1024) -> Workload:
    rng = np.random.default_rng(seed)
    L = BOX_KPC
    gas = _uniform_positions(rng, n_gas, L)
    src = _uniform_positions(rng, n_src, L)
    lum = 10.0 ** rng.uniform(47.0, 50.0, n_src)
    g = rng.standard_normal(n_gas)
    nh = 1e-3 * np.exp(g - 0.5)             # lognormal, sigma_ln = 1, mean 1e-3
    xhi = rng.uniform(0.5, 1.0, n_gas)
    return Workload("clumpy", np.zeros(3), L, KPC_CM, gas, smoothing_lengths(gas), nh * xhi,
                    src, lum, gas, None, (0.3, 0.5, 0.8, 1.0), auto_grid_log2(n_gas), gas_nh=nh)


def _emitters(gas, nh, xhii, L, n_gas):
    """Recombination photon rate per particle, alpha_B n_e n_p V with
    n_e = n_p = x_HII n_H (pure hydrogen) and V = box volume / N."""
    vol_cm3 = (L * KPC_CM) ** 3 / n_gas
    return ALPHA_B * (xhii * nh) ** 2 * vol_cm3


def make_diffuse(seed: int = 3, n_gas: int = 1 << 20, star_lum: float = 1e50,
                 hii_radius: float = 0.3) -> Workload:
    rng = np.random.default_rng(seed)
    L = BOX_KPC
    gas = _uniform_positions(rng, n_gas, L)
    c = np.full((3, 1), 0.5 * L)
    r = np.sqrt(((gas - c) ** 2).sum(axis=0))
    nh = np.full(n_gas, 1e-3)
    xhii = np.where(r < hii_radius * L, 1.0, 1e-3)
    nhi = (1.0 - xhii) * nh
    lum = _emitters(gas, nh, xhii, L, n_gas)
    src = np.ascontiguousarray(np.concatenate([gas, c], axis=1))
    src_lum = np.concatenate([lum, [star_lum]])
    self_src = np.arange(n_gas, dtype=np.int64)
    return Workload("diffuse", np.zeros(3), L, KPC_CM, gas, smoothing_lengths(gas), nhi,
                    src, src_lum, gas, self_src, (1.0,), auto_grid_log2(n_gas), gas_nh=nh,
                    meta={"star": c[:, 0].copy(), "hii_radius": hii_radius * L})


def make_shadow(seed: int = 4, n_gas: int = 1 << 21, n_clumps: int = 16,
                star_lum: float = 1e50) -> Workload:
    rng = np.random.default_rng(seed)
    L = BOX_KPC
    gas = _uniform_positions(rng, n_gas, L)
    c = np.full((3, 1), 0.5 * L)
    # clump centres: +x hemisphere, 0.1L-0.3L from the star
    v = rng.standard_normal((3, n_clumps))
    v /= np.sqrt((v ** 2).sum(axis=0))
    v[0] = np.abs(v[0])
    rad = rng.uniform(0.1, 0.3, n_clumps) * L
    centres = c + v * rad
    r_star = np.sqrt(((gas - c) ** 2).sum(axis=0))
    xhii = np.where(r_star < 0.3 * L, 1.0, 1e-3)
    nh = np.full(n_gas, 1e-3)
    in_clump = np.zeros(n_gas, dtype=bool)
    for k in range(n_clumps):
        d = np.sqrt(((gas - centres[:, k:k + 1]) ** 2).sum(axis=0))
        in_clump |= d < 0.05 * L
    nh[in_clump] *= 200.0
    xhii[in_clump] = 1e-3
    nhi = (1.0 - xhii) * nh
    lum = _emitters(gas, nh, xhii, L, n_gas)
    src = np.ascontiguousarray(np.concatenate([gas, c], axis=1))
    src_lum = np.concatenate([lum, [star_lum]])
    self_src = np.arange(n_gas, dtype=np.int64)
    return Workload("shadow", np.zeros(3), L, KPC_CM, gas, smoothing_lengths(gas), nhi,
                    src, src_lum, gas, self_src, (1.0,), auto_grid_log2(n_gas), gas_nh=nh,
                    meta={"star": c[:, 0].copy(), "hii_radius": 0.3 * L, "clump_centres": centres,
                          "clump_radius": 0.05 * L})


@dataclasses.dataclass
class Equilibrium:
    """A medium to bring into photoionisation equilibrium around fixed sources.

    ``work`` holds the positions, smoothing lengths, sources and grid size
    (its ``gas_nhi`` is the initial n_HI = x_init * n_h); ``n_h`` is the total
    hydrogen density of each particle (cm^-3), ``x_init`` the initial neutral
    fraction and ``volume_cm3`` the volume each particle stands for."""
    work: Workload
    n_h: np.ndarray
    x_init: np.ndarray
    volume_cm3: np.ndarray
    alpha_b: float = ALPHA_B

    def stromgren_radius_cm(self, n_h: float) -> float:
        """R_s = (3 N / (4 pi n_H^2 alpha_B))^(1/3) of eq. (17) for the total
        photon rate of all sources."""
        q = float(self.work.src_lum.sum())
        return (3.0 * q / (4.0 * math.pi * n_h * n_h * self.alpha_b)) ** (1.0 / 3.0)


def make_stromgren(seed: int = 5, n_gas: int = 1 << 15, box_kpc: float = 13.2, lum: float = 5e48,
                   n_h: float = 1e-3, x_ion0: float = 1.2e-3, grid_log2: int | None = None) -> Equilibrium:
    """Test 4 (section 4.2.1): one source at the box centre in uniform static gas."""
    rng = np.random.default_rng(seed)
    L = box_kpc
    gas = _uniform_positions(rng, n_gas, L)
    c = np.full((3, 1), 0.5 * L)
    nh = np.full(n_gas, n_h)
    x0 = np.full(n_gas, 1.0 - x_ion0)
    vol = np.full(n_gas, (L * KPC_CM) ** 3 / n_gas)
    g = auto_grid_log2(n_gas) if grid_log2 is None else grid_log2
    w = Workload("stromgren", np.zeros(3), L, KPC_CM, gas, smoothing_lengths(gas), x0 * nh,
                 np.ascontiguousarray(c), np.array([lum]), gas, None, (1.0,), g)
    return Equilibrium(w, nh, x0, vol)


def make_lw(seed: int = 6, n_gas: int = 1 << 16, n_src: int = 256) -> Workload:
    rng = np.random.default_rng(seed)
    L = BOX_KPC
    gas = _uniform_positions(rng, n_gas, L)
    src = _uniform_positions(rng, n_src, L)
    lum = 10.0 ** rng.uniform(23.0, 25.0, n_src)
    nh = 1e-3 * np.exp(rng.standard_normal(n_gas) - 0.5)
    nh2 = nh * 10.0 ** rng.uniform(-7.0, -3.0, n_gas)
    return Workload("lw", np.zeros(3), L, KPC_CM, gas, smoothing_lengths(gas), np.zeros(n_gas),
                    src, lum, gas, None, (0.0, 0.5, 1.0), auto_grid_log2(n_gas), gas_nh2=nh2)


MAKERS = {"small": make_small, "clumpy": make_clumpy, "diffuse": make_diffuse,
          "shadow": make_shadow, "lw": make_lw}


def source_kernel_inputs(w: Workload):
    """Smoothing lengths and volumes m/rho of the sources, for the kernel-
    weighted cell luminosities: h from the sources' own 32nd neighbour (as
    for the gas), and the volume of a uniform medium holding N_NEIGHBOURS
    particles in the sphere of radius 2h, (4 pi / 3) (2h)^3 / N_NEIGHBOURS."""
    h = smoothing_lengths(w.src_xyz)
    vol = (4.0 * math.pi / 3.0) * (2.0 * h) ** 3 / N_NEIGHBOURS
    return np.ascontiguousarray(h), np.ascontiguousarray(vol)


def make(name: str, **kw) -> Workload:
    return MAKERS[name](**kw)


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """A seeded, sorted subset of k distinct indices out of n."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
