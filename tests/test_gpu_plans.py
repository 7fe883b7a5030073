"""Rate plans (start_rates_plan_*): a staged batch whose rate kernels are
replayed from a HIP graph gives the outputs of start_compute_rates_batched
bit for bit, at creation and on every replay, with other work and
synchronisations between the replays."""
import numpy as np
import pytest

from tests import gpu_common as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def ctx():
    from paper_1005_5312_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


def _items(ctx, prec_pair):
    out = []
    for (w, prec) in zip((H.W.make_diffuse(seed=51, n_gas=5000), H.W.make_clumpy(seed=52, n_gas=3000, n_src=64)),
                         prec_pair):
        box = H.box_of(w)
        tree = ctx.build_source_tree(box, _dev(w.src_xyz), _dev(w.src_lum))
        grid = ctx.build_gas_grid(box, _dev(w.gas_xyz), _dev(w.gas_h), _dev(w.gas_nhi), w.grid_log2)
        dt = torch.float64 if prec == "fp64" else torch.float32
        ss = None if w.self_src is None else _dev(w.self_src)
        out.append(dict(tree=tree, grid=grid, tgt_xyz=_dev(w.tgt_xyz), self_src=ss, theta=1.0, sigma=w.sigma,
                        prec=prec, out=torch.empty(w.n_tgt, dtype=dt, device="cuda")))
    return out


@pytest.mark.parametrize("precs", [("fp32c", "fp64"), ("fp32c", "fp32c")])
def test_plan_replays_equal_batched_call(ctx, precs):
    print(f"[case] rate plan {precs}", flush=True)
    items = _items(ctx, precs)
    ctx.compute_rates_batched(items)
    ctx.synchronize()
    want = [it["out"].cpu().numpy().copy() for it in items]
    for it in items:
        it["out"].fill_(-1.0)
    plan = ctx.rates_plan(items)
    ctx.synchronize()
    for a, it in zip(want, items):
        assert np.array_equal(a, it["out"].cpu().numpy())          # written at creation
    for rep in range(4):
        for it in items:
            it["out"].fill_(-1.0)
        # other work on the same context and stream between replays
        extra = ctx.compute_rates(items[0]["tree"], items[0]["grid"], items[0]["tgt_xyz"][:, :100].contiguous(),
                                  None, 0.5, items[0]["sigma"], "fp64")
        plan.launch()
        ctx.synchronize()
        torch.cuda.synchronize()
        assert torch.isfinite(extra).all()
        for a, it in zip(want, items):
            assert np.array_equal(a, it["out"].cpu().numpy()), rep
    plan.free()


def test_empty_plan_and_errors(ctx):
    from paper_1005_5312_amd import binding
    items = _items(ctx, ("fp32c", "fp64"))
    empty = [dict(items[0], tgt_xyz=torch.empty((3, 0), dtype=torch.float64, device="cuda"),
                  self_src=None, out=torch.empty(0, dtype=torch.float32, device="cuda"))]
    plan = ctx.rates_plan(empty)
    plan.launch()
    ctx.synchronize()
    plan.free()
    bad = [dict(items[0], theta=-1.0)]
    with pytest.raises(binding.StartError):
        ctx.rates_plan(bad)
