"""GPU equilibrium update and equilibrium loop (through the C-ABI) against
the CPU oracle in oracle/equilibrium.py."""
import numpy as np
import pytest

from oracle import equilibrium as E
from oracle import oracle as O
from tests import gpu_common as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ALPHA = H.W.ALPHA_B


@pytest.fixture(scope="module")
def ctx():
    from paper_1005_5312_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


def update_inputs(n, seed, f32):
    rng = np.random.default_rng(seed)
    g = 10.0 ** rng.uniform(-24, -6, n)
    g[rng.random(n) < 0.05] = 0.0
    if f32:
        g = g.astype(np.float32)
    nh = 10.0 ** rng.uniform(-7, 3, n)
    nh[rng.random(n) < 0.02] = 0.0
    x0 = rng.random(n)
    return g, nh, x0


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("n", [1, 255, 100_003])
def test_update_matches_oracle(ctx, prec, n):
    g, nh, x0 = update_inputs(n, seed=11 + n, f32=(prec == "fp32c"))
    dev = ctx.device
    x = torch.from_numpy(x0.copy()).to(dev)
    nhi = torch.empty(n, dtype=torch.float64, device=dev)
    ch = ctx.equilibrium_update(torch.from_numpy(nh).to(dev), torch.from_numpy(g).to(dev), ALPHA, x, nhi)
    got = x.cpu().numpy()
    want = E.neutral_fraction(g.astype(np.float64), nh, ALPHA)
    # same closed form in FP64 on both sides: a few ulp at most
    assert np.all(np.abs(got - want) <= 4.5e-16 * np.abs(want)), np.max(np.abs(got - want) / np.maximum(want, 1e-300))
    assert np.array_equal(nhi.cpu().numpy(), got * nh)
    assert ch == np.max(np.abs(got - x0))


def test_update_without_change_is_asynchronous(ctx):
    g, nh, x0 = update_inputs(4096, seed=5, f32=False)
    dev = ctx.device
    x = torch.from_numpy(x0.copy()).to(dev)
    assert ctx.equilibrium_update(torch.from_numpy(nh).to(dev), torch.from_numpy(g).to(dev), ALPHA, x,
                                  want_change=False) is None
    ctx.synchronize()
    assert np.allclose(x.cpu().numpy(), E.neutral_fraction(g, nh, ALPHA), rtol=4.5e-16, atol=0)


def test_update_input_errors(ctx):
    from paper_1005_5312_amd import binding
    dev = ctx.device
    n = 1000
    g, nh, x0 = update_inputs(n, seed=6, f32=False)
    for bad_g, bad_nh in ((g, -nh), (np.where(np.arange(n) == 7, np.nan, g), nh), (-g, nh)):
        x = torch.from_numpy(x0.copy()).to(dev)
        with pytest.raises(binding.StartError) as ei:
            ctx.equilibrium_update(torch.from_numpy(bad_nh).to(dev), torch.from_numpy(bad_g).to(dev), ALPHA, x)
        assert ei.value.code == binding.EINVAL
    ctx.synchronize()   # the error was reported once and cleared
    with pytest.raises(binding.StartError):
        ctx.equilibrium_update(torch.from_numpy(nh).to(dev), torch.from_numpy(g).to(dev), 0.0,
                               torch.from_numpy(x0.copy()).to(dev))
    # n = 0 is a no-op
    e = torch.empty(0, dtype=torch.float64, device=dev)
    assert ctx.equilibrium_update(e, e, ALPHA, e) == 0.0


def loop_case(name):
    if name == "stromgren":
        e = H.W.make_stromgren(seed=5, n_gas=1 << 15, grid_log2=5)
        return e.work, e.n_h, e.x_init, 1.0
    w = H.W.make_small(seed=9, n_gas=4096, n_src=16)
    return w, np.full(w.n_gas, 1e-3), np.ones(w.n_gas), 0.5


def gpu_loop(ctx, w, nh, x0, theta, prec, max_iter, tol):
    from paper_1005_5312_amd import binding
    dev = ctx.device
    tree = ctx.build_source_tree(H.box_of(w), torch.from_numpy(w.src_xyz).to(dev),
                                 torch.from_numpy(w.src_lum).to(dev))
    x, gam, it, ch = ctx.ionization_equilibrium(tree, w.gas_xyz, w.gas_h, nh, x0, w.grid_log2, theta=theta,
                                                sigma=w.sigma, alpha=ALPHA, prec=prec, max_iter=max_iter, tol=tol)
    assert isinstance(tree, binding.SourceTree)
    return x.cpu().numpy(), gam.cpu().numpy().astype(np.float64), it, ch


# Parity of whole loops: both sides start from the same neutral field and run
# the same number of iterations, and are held to the tolerance of one rate
# call.  For x the bound follows from the closed form: |d ln x / d ln Gamma|
# = (1 - x) / (1 + x) <= 1, so a relative rate error e moves x by at most
# x e <= e.  (Feeding x back into the optical depths could in principle
# amplify errors from one iteration to the next; the printed errors show it
# does not at these sizes.)
LOOP_TOL = {"fp64": dict(gamma=H.TOL_FP64, x=H.TOL_FP64), "fp32c": dict(gamma=H.TOL_FP32C, x=H.TOL_FP32C)}


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("name", ["stromgren", "small"])
def test_loop_matches_oracle(ctx, name, prec):
    w, nh, x0, theta = loop_case(name)
    iters = 25 if name == "stromgren" else 10
    x, gam, it, ch = gpu_loop(ctx, w, nh, x0, theta, prec, iters, 0.0)
    box = H.obox_of(w)
    tree = O.Tree(box, w.src_xyz, w.src_lum)
    xo, go, ito, cho = E.ionization_equilibrium(box, tree, w.gas_xyz, w.gas_h, nh, x0, w.grid_log2, theta,
                                                w.sigma, ALPHA, max_iter=iters, tol=0.0)
    assert it == ito == iters
    rel, ab, nbig = H.rel_errors(gam, go)
    dx = float(np.max(np.abs(x - xo)))
    print(f"  {name} {prec}: gamma rel {rel:.2e} (abs below floor {ab:.1e}), max |dx| {dx:.2e}, "
          f"last change gpu {ch:.3e} oracle {cho:.3e}")
    assert rel <= LOOP_TOL[prec]["gamma"] and ab <= H.ABS_FLOOR
    assert dx <= LOOP_TOL[prec]["x"]


def test_loop_converges_like_oracle(ctx):
    w, nh, x0, theta = loop_case("stromgren")
    x, gam, it, ch = gpu_loop(ctx, w, nh, x0, theta, "fp64", 300, 1e-3)
    box = H.obox_of(w)
    tree = O.Tree(box, w.src_xyz, w.src_lum)
    xo, go, ito, cho = E.ionization_equilibrium(box, tree, w.gas_xyz, w.gas_h, nh, x0, w.grid_log2, theta,
                                                w.sigma, ALPHA, max_iter=300, tol=1e-3)
    print(f"  converged after {it} (oracle {ito}) iterations")
    assert it == ito and ch <= 1e-3
    assert float(np.max(np.abs(x - xo))) <= 1e-6


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_stromgren_sphere_full_size(ctx, prec):
    """Test 4 at 2^21 particles on a 128^3 grid: properties that hold at any
    size (the oracle cannot run this many iterations here): a converged
    field, the 5.4 kpc radius of eq. (17) within 5%, photon balance within
    10%, ionised inside and neutral outside."""
    import time
    e = H.W.make_stromgren(seed=5, n_gas=1 << 21, grid_log2=7)
    w = e.work
    t0 = time.perf_counter()
    x, gam, it, ch = gpu_loop(ctx, w, e.n_h, e.x_init, 1.0, prec, 200, 1e-4)
    dt = time.perf_counter() - t0
    r_eq = E.ionised_volume_radius(x, e.volume_cm3) / H.KPC
    ph = E.photoionisations(x, gam, e.n_h, e.volume_cm3) / w.src_lum.sum()
    print(f"  {prec}: {it} iterations in {dt:.2f} s, R_eq {r_eq:.3f} kpc, photons {ph:.4f}")
    assert ch <= 1e-4 and it < 200
    assert abs(r_eq / 5.4 - 1.0) <= 0.05
    assert abs(ph - 1.0) <= 0.10
    r = np.sqrt(((w.gas_xyz - 0.5 * w.box_size) ** 2).sum(axis=0))
    assert np.mean(x[r < 3.0]) < 0.02 and np.mean(x[r > 6.2]) > 0.99


# --- recombination photons (section 4.1) ----------------------------------

ALPHA_1 = 1.58e-13


def recomb_inputs(n, seed):
    rng = np.random.default_rng(seed)
    nh = 10.0 ** rng.uniform(-5, 2, n)
    x = rng.random(n)
    if n >= 3:
        x[:3] = (0.0, 1.0, 1e-12)
    vol = 10.0 ** rng.uniform(50, 63, n)
    return nh, x, vol


@pytest.mark.parametrize("n", [1, 300, 65_537])
def test_recombination_emission_matches_oracle(ctx, n):
    nh, x, vol = recomb_inputs(n, seed=n)
    dev = ctx.device
    lum, ks = ctx.recombination_emission(torch.from_numpy(nh).to(dev), torch.from_numpy(x).to(dev),
                                         torch.from_numpy(vol).to(dev), 6.3e-18, ALPHA_1)
    ctx.synchronize()
    # the same products in the same order: bit for bit
    assert np.array_equal(lum.cpu().numpy(), E.recombination_emission(nh, x, vol, ALPHA_1))
    # cube root and expm1 are library functions on both sides: a few ulp
    want = E.k_self(nh, x, vol, 6.3e-18, ALPHA_1)
    got = ks.cpu().numpy()
    big = want > 0
    assert np.all(got[~big] == 0.0)
    assert np.max(np.abs(got[big] - want[big]) / want[big]) <= 1e-14
    # one output only
    lum2, none = ctx.recombination_emission(nh, x, vol, 6.3e-18, ALPHA_1, want_k_self=False)
    assert none is None and torch.equal(lum2, lum)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_total_ionization_matches_oracle(ctx, prec):
    n = 10_001
    nh, x, vol = recomb_inputs(n, seed=77)
    rng = np.random.default_rng(78)
    g = 10.0 ** rng.uniform(-20, -8, n)
    if prec == "fp32c":
        g = g.astype(np.float32)
    ks = E.k_self(nh, x, vol, 6.3e-18, ALPHA_1)
    dev = ctx.device
    got = ctx.total_ionization(torch.from_numpy(nh).to(dev), torch.from_numpy(x).to(dev),
                               torch.from_numpy(g).to(dev), torch.from_numpy(ks).to(dev)).cpu().numpy()
    assert np.array_equal(got, E.k_ion_total(g.astype(np.float64), nh, x, ks))
    got0 = ctx.total_ionization(nh, x, torch.from_numpy(g).to(dev)).cpu().numpy()
    assert np.array_equal(got0, x * nh * g.astype(np.float64))


def test_recombination_input_errors(ctx):
    from paper_1005_5312_amd import binding
    nh, x, vol = recomb_inputs(100, seed=3)
    for bad in ((-nh, x, vol), (nh, x + 1.0, vol), (nh, x, -vol)):
        ctx.recombination_emission(*bad, 6.3e-18, ALPHA_1)
        with pytest.raises(binding.StartError) as ei:
            ctx.synchronize()
        assert ei.value.code == binding.EINVAL
    with pytest.raises(binding.StartError):
        ctx.recombination_emission(nh, x, vol, -1.0, ALPHA_1)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_diffuse_k_ion_pipeline_matches_oracle(ctx, prec):
    """Every particle an emitter (eq. 19), Gamma from all other emitters
    through the tree (self excluded), plus k_self: k_ion of eq. (25) on a
    partly ionised medium, against the oracle."""
    w = H.W.make_small(seed=12, n_gas=4096, n_src=1)
    rng = np.random.default_rng(13)
    nh = np.full(w.n_gas, 1e-3) * np.exp(rng.standard_normal(w.n_gas) * 0.5)
    x = rng.uniform(0.01, 1.0, w.n_gas)
    vol = np.full(w.n_gas, (w.box_size * H.KPC) ** 3 / w.n_gas)
    dev = ctx.device
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    lum, ks = ctx.recombination_emission(d(nh), d(x), d(vol), w.sigma, ALPHA_1)
    box = H.box_of(w)
    tree = ctx.build_source_tree(box, d(w.gas_xyz), lum)
    grid = ctx.build_gas_grid(box, d(w.gas_xyz), d(w.gas_h), d(x * nh), w.grid_log2)
    ss = d(np.arange(w.n_gas, dtype=np.int64))
    gam = ctx.compute_rates(tree, grid, d(w.gas_xyz), ss, 1.0, w.sigma, prec)
    kion = ctx.total_ionization(d(nh), d(x), gam, ks).cpu().numpy()
    ob = H.obox_of(w)
    lum_o = E.recombination_emission(nh, x, vol, ALPHA_1)
    go = O.rates(O.Tree(ob, w.gas_xyz, lum_o), w.grid_log2, O.grid(ob, w.gas_xyz, w.gas_h, x * nh, w.grid_log2),
                 w.gas_xyz, np.arange(w.n_gas), 1.0, w.sigma)
    want = E.k_ion_total(go, nh, x, E.k_self(nh, x, vol, w.sigma, ALPHA_1))
    rel = float(np.max(np.abs(kion - want) / want))
    print(f"  k_ion {prec}: max rel {rel:.2e}")
    assert rel <= (H.TOL_FP64 if prec == "fp64" else H.TOL_FP32C)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_graph_replay_equals_eager_loop(ctx, prec):
    """The iterations after the first are replayed from one captured HIP graph;
    after 1, 2, 3, 7 and 25 iterations (one synchronisation and a host read
    between replays) x and Gamma equal those of the loop launched kernel by
    kernel, bit for bit."""
    w, nh, x0, theta = loop_case("small")
    for iters in (1, 2, 3, 7, 25):
        outs = {}
        for graphs in (False, True):
            ctx.set_graph_replay(graphs)
            outs[graphs] = gpu_loop(ctx, w, nh, x0, theta, prec, iters, 0.0)
        ctx.set_graph_replay(True)
        (xa, ga, ia, ca), (xb, gb, ib, cb) = outs[False], outs[True]
        # (the loop also stops early once no x changes at all)
        assert ia == ib and ia <= iters and ca == cb
        assert np.array_equal(xa, xb) and np.array_equal(ga, gb), iters


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_recorded_pairs_equal_stencil_search(ctx, prec):
    """Grids refilled from the recorded (cell, particle) pairs equal those of
    the stencil search bit for bit: x, Gamma and the iteration count of the
    loops agree exactly with the recording on and off, on the small medium,
    the Stromgren sphere and with recombination photons."""
    for name in ("small", "stromgren"):
        w, nh, x0, theta = loop_case(name)
        outs = {}
        for pairs in (False, True):
            ctx.set_grid_pairs(pairs)
            outs[pairs] = gpu_loop(ctx, w, nh, x0, theta, prec, 6, 0.0)
        ctx.set_grid_pairs(True)
        (xa, ga, ia, ca), (xb, gb, ib, cb) = outs[False], outs[True]
        assert ia == ib and ca == cb, name
        assert np.array_equal(xa, xb) and np.array_equal(ga, gb), name
    e = H.W.make_stromgren(n_gas=1 << 14, grid_log2=5)
    outs = {}
    for pairs in (False, True):
        ctx.set_grid_pairs(pairs)
        outs[pairs] = gpu_diffuse(ctx, e, prec, 5, 0.0)
    ctx.set_grid_pairs(True)
    (xa, ga, ia, ca), (xb, gb, ib, cb) = outs[False], outs[True]
    assert ia == ib and ca == cb
    assert np.array_equal(xa, xb) and np.array_equal(ga, gb)


# --- equilibrium with the transfer of recombination photons ---------------

ALPHA_A = 4.18e-13


def gpu_diffuse(ctx, e, prec, max_iter, tol, alpha_1=ALPHA_1, theta=1.0):
    w = e.work
    x, g, it, ch = ctx.diffuse_equilibrium(H.box_of(w), w.gas_xyz, w.gas_h, e.n_h, e.volume_cm3, w.src_xyz,
                                           w.src_lum, e.x_init, w.grid_log2, theta, w.sigma, ALPHA_A, alpha_1, prec,
                                           max_iter, tol)
    return x.cpu().numpy(), g.cpu().numpy().astype(np.float64), it, ch


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_diffuse_loop_matches_oracle(ctx, prec):
    e = H.W.make_stromgren(seed=6, n_gas=1 << 13, grid_log2=4)
    w = e.work
    x, g, it, ch = gpu_diffuse(ctx, e, prec, 6, 0.0)
    ob = H.obox_of(w)
    xo, go, ito, cho = E.diffuse_equilibrium(ob, w.gas_xyz, w.gas_h, e.n_h, e.volume_cm3, w.src_xyz, w.src_lum,
                                             e.x_init, w.grid_log2, 1.0, w.sigma, ALPHA_A, ALPHA_1, max_iter=6,
                                             tol=0.0)
    assert it == ito == 6
    rel, ab, _ = H.rel_errors(g, go)
    dx = float(np.max(np.abs(x - xo)))
    print(f"  diffuse loop {prec}: gamma rel {rel:.2e}, max |dx| {dx:.2e}")
    tol = H.TOL_FP64 if prec == "fp64" else H.TOL_FP32C
    assert rel <= tol and ab <= H.ABS_FLOOR and dx <= tol


def test_diffuse_loop_without_ground_state_photons_equals_plain_loop(ctx):
    e = H.W.make_stromgren(seed=6, n_gas=1 << 13, grid_log2=4)
    w = e.work
    x, g, it, ch = gpu_diffuse(ctx, e, "fp64", 8, 0.0, alpha_1=0.0)
    tree = ctx.build_source_tree(H.box_of(w), torch.from_numpy(w.src_xyz).to(ctx.device),
                                 torch.from_numpy(w.src_lum).to(ctx.device))
    xo, go, ito, cho = ctx.ionization_equilibrium(tree, w.gas_xyz, w.gas_h, e.n_h, e.x_init, w.grid_log2, 1.0,
                                                  w.sigma, ALPHA_A, "fp64", 8, 0.0)
    # (the star's virtual-source centre may round differently inside a
    # tree of zero-luminosity particles: equal to rounding, not bit for bit)
    assert it == ito
    assert np.allclose(x, xo.cpu().numpy(), rtol=1e-12, atol=0)
    assert np.allclose(g, go.cpu().numpy(), rtol=1e-12, atol=0)


def test_diffuse_photons_extend_the_hii_region(ctx):
    """Test 4 (section 4.2.1): with the transfer of recombination photons the
    ionised region is more extended than on the spot, and near the source
    the gas is more neutral (all recombinations count there, alpha_A >
    alpha_B, while the photons escape); 2^15 particles, G = 32."""
    e = H.W.make_stromgren(seed=5, n_gas=1 << 15, grid_log2=5)
    w = e.work
    xd, gd, itd, chd = gpu_diffuse(ctx, e, "fp32c", 400, 1e-3)
    tree = ctx.build_source_tree(H.box_of(w), torch.from_numpy(w.src_xyz).to(ctx.device),
                                 torch.from_numpy(w.src_lum).to(ctx.device))
    xo, go, ito, cho = ctx.ionization_equilibrium(tree, w.gas_xyz, w.gas_h, e.n_h, e.x_init, w.grid_log2, 1.0,
                                                  w.sigma, H.W.ALPHA_B, "fp32c", 400, 1e-3)
    xo = xo.cpu().numpy()
    rd = E.ionised_volume_radius(xd, e.volume_cm3) / H.KPC
    ro = E.ionised_volume_radius(xo, e.volume_cm3) / H.KPC
    r = np.sqrt(((w.gas_xyz - 0.5 * w.box_size) ** 2).sum(axis=0))
    inner = r < 3.0
    print(f"  R_eq on the spot {ro:.3f} kpc ({ito} it), with diffuse photons {rd:.3f} kpc ({itd} it); "
          f"inner x {xo[inner].mean():.2e} vs {xd[inner].mean():.2e}")
    assert chd <= 1e-3 and cho <= 1e-3
    assert rd > ro * 1.02
    assert xd[inner].mean() > xo[inner].mean()
