"""GPU H2 photodissociation rates (Appendix B, through the C-ABI) against the
oracle's or_lw_rates: same lists and rays as the photoionisation rates, the
H2 column shielding by f_sh instead of exp(-tau)."""
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


def built(ctx, w):
    dev = ctx.device
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    box = H.box_of(w)
    tree = ctx.build_source_tree(box, d(w.src_xyz), d(w.src_lum))
    grid = ctx.build_gas_grid(box, d(w.gas_xyz), d(w.gas_h), d(w.gas_nh2), w.grid_log2)
    return tree, grid


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("theta", [0.0, 0.5, 1.0])
def test_lw_small_all_targets(ctx, theta, prec):
    w = H.W.make_lw(seed=31, n_gas=4096, n_src=64)
    tree, grid = built(ctx, w)
    got = ctx.compute_dissociation_rates(tree, grid, w.tgt_xyz, None, theta, prec).cpu().numpy()
    ob = H.obox_of(w)
    want = O.lw_rates(O.Tree(ob, w.src_xyz, w.src_lum), w.grid_log2,
                      O.grid(ob, w.gas_xyz, w.gas_h, w.gas_nh2, w.grid_log2), w.tgt_xyz, None, theta)
    rel, ab, nbig = H.rel_errors(got.astype(np.float64), want)
    print(f"  lw theta {theta} {prec}: max rel {rel:.2e}")
    assert nbig == w.n_tgt
    assert rel <= (H.TOL_FP64 if prec == "fp64" else H.TOL_FP32C)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_lw_clumpy_size_sampled(ctx, prec):
    """2^18 particles and 1024 sources on a 64^3 grid, with self exclusion of
    a few targets placed on sources, 2048 sampled targets."""
    w = H.W.make_lw(seed=32, n_gas=1 << 18, n_src=1024)
    tree, grid = built(ctx, w)
    idx = H.W.sample_indices(w.n_tgt, 2048, 5)
    tgt = np.ascontiguousarray(np.concatenate([w.tgt_xyz[:, idx], w.src_xyz[:, :16]], axis=1))
    ss = np.concatenate([np.full(len(idx), -1), np.arange(16)]).astype(np.int64)
    got = ctx.compute_dissociation_rates(tree, grid, tgt, ss, 1.0, prec).cpu().numpy()
    ob = H.obox_of(w)
    want = O.lw_rates(O.Tree(ob, w.src_xyz, w.src_lum), w.grid_log2,
                      O.grid(ob, w.gas_xyz, w.gas_h, w.gas_nh2, w.grid_log2), tgt, ss, 1.0)
    rel, ab, nbig = H.rel_errors(got.astype(np.float64), want)
    print(f"  lw 2^18 {prec}: max rel {rel:.2e}")
    assert rel <= (H.TOL_FP64 if prec == "fp64" else H.TOL_FP32C)


def test_lw_does_not_change_photoionisation(ctx):
    """The same tree and grid through both channels: the photoionisation
    call is unaffected by a dissociation call before it."""
    w = H.W.make_lw(seed=33, n_gas=4096, n_src=32)
    tree, grid = built(ctx, w)
    a = ctx.compute_rates(tree, grid, w.tgt_xyz, None, 1.0, w.sigma, "fp64").cpu().numpy()
    ctx.compute_dissociation_rates(tree, grid, w.tgt_xyz, None, 1.0, "fp64")
    b = ctx.compute_rates(tree, grid, w.tgt_xyz, None, 1.0, w.sigma, "fp64").cpu().numpy()
    assert np.array_equal(a, b)
