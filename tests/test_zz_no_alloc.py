"""start_compute_rates_noalloc (fixed device scratch, no allocation) against
start_compute_rates through the C-ABI: the same kernels, so the same results
bit for bit, on two calls in a row (the second smaller), in both precisions;
sizes beyond the fixed scratch are refused."""
import numpy as np
import pytest

from paper_1005_5312_amd import binding as B
from paper_1005_5312_amd import workloads as W
from tests import gpu_common as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def ctx():
    import paper_1005_5312_amd as S
    c = S.Context(0)
    yield c
    c.close()


def test_noalloc_matches_compute_rates(ctx):
    w = W.make_diffuse(seed=31, n_gas=20000)
    print(f"[case] noalloc: diffuse {w.n_tgt} targets, {w.n_src} sources", flush=True)
    box = H.box_of(w)
    tree = ctx.build_source_tree(box, _dev(w.src_xyz), _dev(w.src_lum))
    grid = ctx.build_gas_grid(box, _dev(w.gas_xyz), _dev(w.gas_h), _dev(w.gas_nhi), w.grid_log2)
    # two calls in a row, the second on fewer (and other) targets
    first = np.arange(w.n_tgt)
    second = H.W.sample_indices(w.n_tgt, 3001, seed=4)
    for prec in ("fp32c", "fp64"):
        for idx in (first, second):
            tgt = _dev(w.tgt_xyz[:, idx])
            ss = _dev(w.self_src[idx])
            want = ctx.compute_rates(tree, grid, tgt, ss, 1.0, w.sigma, prec)
            got = ctx.compute_rates_noalloc(tree, grid, tgt, ss, 1.0, w.sigma, prec)
            ctx.synchronize()
            a, b = got.cpu().numpy(), want.cpu().numpy()
            print(f"  {prec} {len(idx)} targets: identical {np.array_equal(a, b)}", flush=True)
            assert np.all(np.isfinite(a))
            assert np.array_equal(a, b)


def test_noalloc_refuses_beyond_its_scratch(ctx):
    w = W.make_small(seed=2, n_gas=512, n_src=4)
    print("[case] noalloc: 2^18 + 1 targets refused", flush=True)
    box = H.box_of(w)
    tree = ctx.build_source_tree(box, _dev(w.src_xyz), _dev(w.src_lum))
    grid = ctx.build_gas_grid(box, _dev(w.gas_xyz), _dev(w.gas_h), _dev(w.gas_nhi), w.grid_log2)
    rng = np.random.default_rng(0)
    tgt = _dev(w.box_lo[:, None] + rng.uniform(0, w.box_size, (3, (1 << 18) + 1)))
    with pytest.raises(B.StartError) as e:
        ctx.compute_rates_noalloc(tree, grid, tgt, None, 1.0, w.sigma, "fp32c")
    assert e.value.code == B.ECAPACITY
    # the context is still usable, and the largest size passes
    ok = ctx.compute_rates_noalloc(tree, grid, tgt[:, : 1 << 18].contiguous(), None, 1.0, w.sigma, "fp32c")
    ref = ctx.compute_rates(tree, grid, tgt[:, : 1 << 18].contiguous(), None, 1.0, w.sigma, "fp32c")
    ctx.synchronize()
    assert np.array_equal(ok.cpu().numpy(), ref.cpu().numpy())
