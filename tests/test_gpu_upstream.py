"""GPU upstream-particle chain (section 2.2.1, through the C-ABI) against the
oracle's or_upstream_rates: the same upstream particle for every (particle,
list entry) pair, bit for bit, and the same rates to the FP64 tolerance."""
import numpy as np
import pytest

from oracle import oracle as O
from tests import gpu_common as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_1005_5312_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


def cases():
    w1 = H.W.make_small(seed=7, n_gas=2048, n_src=8)
    w2 = H.W.make_clumpy(seed=10, n_gas=4096, n_src=64)
    w3 = H.W.make_diffuse(seed=9, n_gas=3000)
    w4 = H.W.make_small(seed=11, n_gas=4096, n_src=32)
    x = w4.gas_xyz
    w4.gas_nhi = 1e-4 * (1 + 0.5 * np.sin(2 * np.pi * x[0] / w4.box_size) * np.cos(2 * np.pi * x[1] / w4.box_size))
    return {"uniform": (w1, 1.0), "lognormal": (w2, 1.0), "emitters": (w3, 1.0), "smooth": (w4, 0.5),
            "uniform_theta0": (w1, 0.0)}


def many_source_case():
    # few particles, many sources: the membership table's rows exceed what a
    # wave keeps in LDS (more than 2048 words of n_nodes + n_src bits)
    return {"many_sources": (H.W.make_small(seed=14, n_gas=2048, n_src=70000), 1.0)}


def membership_path(ctx, tree, n_gas, n_pairs):
    """How the call tests a source's membership in a neighbour's list, by the
    rule the library states: a bit table when it takes at most max(8 bytes per
    pair, 64 MiB) (and 4 GiB), built in LDS for rows up to 2048 words;
    otherwise searches of the sorted lists."""
    nodes = ctx.tree_export(tree)["geo"].shape[0]
    w = (nodes + tree.n_src + 31) // 32
    table = n_gas * w * 4
    if table <= max(8 * n_pairs, 64 << 20) and table <= 4 << 30:
        return "rows" if w <= 2048 else "atomics"
    return "search"


EXPECTED_PATH = {"uniform": "rows", "lognormal": "rows", "emitters": "rows", "smooth": "rows",
                 "uniform_theta0": "rows", "lognormal_2^15": "rows", "emitters_2^15": "search",
                 "many_sources": "atomics"}


def large_cases():
    # 2^15 particles: several grid cells of particles per kernel support, the
    # neighbour lists' full range of lengths and deep chains (the oracle's
    # cell-list search makes these sizes affordable)
    return {"lognormal_2^15": (H.W.make_clumpy(seed=12, n_gas=1 << 15, n_src=1024), 1.0),
            "emitters_2^15": (H.W.make_diffuse(seed=13, n_gas=1 << 15), 1.0)}


@pytest.mark.parametrize("name", ["uniform", "lognormal", "emitters", "smooth", "uniform_theta0",
                                  "lognormal_2^15", "emitters_2^15", "many_sources"])
def test_upstream_chain_matches_oracle(ctx, name):
    w, theta = {**cases(), **large_cases(), **many_source_case()}[name]
    print(f"[case] upstream {name}: {w.n_gas} particles, {w.n_src} sources, theta {theta}", flush=True)
    dev = ctx.device
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    box = H.box_of(w)
    tree = ctx.build_source_tree(box, d(w.src_xyz), d(w.src_lum))
    grid = ctx.build_gas_grid(box, d(w.gas_xyz), d(w.gas_h), d(w.gas_nhi), w.grid_log2)
    gam, offs, par, roots = ctx.compute_rates_upstream(tree, grid, w.gas_xyz, w.gas_h, w.gas_nhi, w.self_src, theta,
                                                       w.sigma, structure=True)
    ob = H.obox_of(w)
    otree = O.Tree(ob, w.src_xyz, w.src_lum)
    ogrid = O.grid(ob, w.gas_xyz, w.gas_h, w.gas_nhi, w.grid_log2)
    want, ooffs, opar, ost = O.upstream_rates(otree, w.grid_log2, ogrid, w.gas_xyz, w.gas_h, w.gas_nhi, w.self_src,
                                              theta, w.sigma, structure=True)
    path = membership_path(ctx, tree, w.n_gas, int(offs[-1]))
    print(f"  membership by {path}")
    assert path == EXPECTED_PATH[name]
    assert np.array_equal(offs, ooffs)
    assert np.array_equal(par, opar)              # the same upstream particle for every pair
    assert roots == int(ost[:, 1].sum())
    rel, ab, nbig = H.rel_errors(gam.cpu().numpy(), want)
    print(f"  {name}: {offs[-1]} pairs, {roots} integrated along the ray, max rel {rel:.2e}")
    assert rel <= H.TOL_FP64 and ab <= H.ABS_FLOOR
    if name.startswith("uniform"):
        # uniform gas: the chain telescopes to the ray integral
        ray = ctx.compute_rates(tree, grid, w.gas_xyz, w.self_src, theta, w.sigma, "fp64").cpu().numpy()
        assert np.max(np.abs(gam.cpu().numpy() / ray - 1)) <= 1e-11


def test_upstream_empty_and_errors(ctx):
    from paper_1005_5312_amd import binding
    w = H.W.make_small(seed=7, n_gas=512, n_src=4)
    dev = ctx.device
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    box = H.box_of(w)
    tree = ctx.build_source_tree(box, d(w.src_xyz), d(w.src_lum))
    grid = ctx.build_gas_grid(box, d(w.gas_xyz), d(w.gas_h), d(w.gas_nhi), w.grid_log2)
    e = np.zeros((3, 0))
    out = ctx.compute_rates_upstream(tree, grid, e, np.zeros(0), np.zeros(0))
    assert out.numel() == 0
    with pytest.raises(binding.StartError):
        ctx.compute_rates_upstream(tree, grid, w.gas_xyz, -w.gas_h, w.gas_nhi)
    with pytest.raises(binding.StartError):
        ctx.compute_rates_upstream(tree, grid, w.gas_xyz, w.gas_h, w.gas_nhi, theta=-1.0)
