"""The two-stream scene build (start_build_scene) against the separate tree
and grid builds: the same tree and grid bit for bit, the same rates, no
memory left behind on failures, and the failing build's status."""
import numpy as np
import pytest

from paper_1005_5312_amd import binding as B
from tests import gpu_common as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("name", ["small", "clumpy"])
def test_scene_equals_separate_builds(ctx, name):
    w = H.workload(name)
    print(f"[case] scene {name}", flush=True)
    box = H.box_of(w)
    args = (dev(w.src_xyz), dev(w.src_lum), dev(w.gas_xyz), dev(w.gas_h), dev(w.gas_nhi))
    t1 = ctx.build_source_tree(box, args[0], args[1])
    g1 = ctx.build_gas_grid(box, args[2], args[3], args[4], w.grid_log2)
    t2, g2 = ctx.build_scene(box, *args, w.grid_log2)
    e1, e2 = ctx.tree_export(t1), ctx.tree_export(t2)
    assert sorted(e1) == sorted(e2)
    for k in e1:
        assert np.array_equal(e1[k], e2[k]), k
    assert np.array_equal(ctx.grid_export(g1), ctx.grid_export(g2))
    tgt = dev(w.tgt_xyz)
    ss = None if w.self_src is None else dev(w.self_src)
    for prec in ("fp32c", "fp64"):
        a = ctx.compute_rates(t1, g1, tgt, ss, 1.0, w.sigma, prec).cpu().numpy()
        b = ctx.compute_rates(t2, g2, tgt, ss, 1.0, w.sigma, prec).cpu().numpy()
        assert np.array_equal(a, b), prec
    for o in (t1, g1, t2, g2):
        o.free()


def test_scene_repeated_builds_release_memory(ctx):
    """Ten builds in a row (blocks handed back and forth between the two
    build threads through the context's pool): same grid every time, and the
    memory held returns to where it was."""
    w = H.workload("clumpy")
    box = H.box_of(w)
    args = (dev(w.src_xyz), dev(w.src_lum), dev(w.gas_xyz), dev(w.gas_h), dev(w.gas_nhi))
    base = ctx.bytes_in_use()
    ref = None
    for _ in range(10):
        t, g = ctx.build_scene(box, *args, w.grid_log2)
        v = ctx.grid_export(g)
        if ref is None:
            ref = v
        assert np.array_equal(v, ref)
        t.free()
        g.free()
        assert ctx.bytes_in_use() == base


@pytest.mark.parametrize("bad,code", [("gas_out_of_box", B.EOUTOFBOX), ("src_nonfinite", B.ENONFINITE),
                                      ("both", B.ENONFINITE), ("gas_h_negative", B.EINVAL)])
def test_scene_failures(ctx, bad, code):
    w = H.workload("small")
    box = H.box_of(w)
    sx, sl = w.src_xyz.copy(), w.src_lum.copy()
    gx, gh = w.gas_xyz.copy(), w.gas_h.copy()
    if bad in ("gas_out_of_box", "both"):
        gx[0, 5] = w.box_lo[0] + 2 * w.box_size
    if bad in ("src_nonfinite", "both"):
        sx[1, 3] = np.nan
    if bad == "gas_h_negative":
        gh[7] = -1.0
    base = ctx.bytes_in_use()
    with pytest.raises(B.StartError) as ei:
        ctx.build_scene(box, dev(sx), dev(sl), dev(gx), dev(gh), dev(w.gas_nhi), w.grid_log2)
    assert ei.value.code == code
    assert ctx.bytes_in_use() == base
    # the context stays usable
    t, g = ctx.build_scene(box, dev(w.src_xyz), dev(w.src_lum), dev(w.gas_xyz), dev(w.gas_h), dev(w.gas_nhi),
                           w.grid_log2)
    t.free()
    g.free()


def test_scene_budget():
    w = H.workload("small")
    box = H.box_of(w)
    with B.Context(0, hbm_budget=1 << 16) as c:
        with pytest.raises(B.StartError) as ei:
            c.build_scene(box, dev(w.src_xyz), dev(w.src_lum), dev(w.gas_xyz), dev(w.gas_h), dev(w.gas_nhi),
                          w.grid_log2)
        assert ei.value.code == B.EBUDGET
        assert c.bytes_in_use() == 0


@pytest.mark.parametrize("case", ["no_sources", "no_gas", "both_empty", "auto_grid"])
def test_scene_edge_cases(ctx, case):
    """Empty source or gas sets and the automatic grid size go through the
    scene build exactly as through the separate builds."""
    w = H.workload("small")
    box = H.box_of(w)
    sx, sl = w.src_xyz, w.src_lum
    gx, gh, gn = w.gas_xyz, w.gas_h, w.gas_nhi
    gl = w.grid_log2
    if case in ("no_sources", "both_empty"):
        sx, sl = np.zeros((3, 0)), np.zeros(0)
    if case in ("no_gas", "both_empty"):
        gx, gh, gn = np.zeros((3, 0)), np.zeros(0), np.zeros(0)
    if case == "auto_grid":
        gl = 0
    print(f"[case] scene edge {case}", flush=True)
    t1 = ctx.build_source_tree(box, dev(sx), dev(sl))
    g1 = ctx.build_gas_grid(box, dev(gx), dev(gh), dev(gn), gl)
    t2, g2 = ctx.build_scene(box, dev(sx), dev(sl), dev(gx), dev(gh), dev(gn), gl)
    assert g1.G == g2.G
    assert np.array_equal(ctx.grid_export(g1), ctx.grid_export(g2))
    tgt = dev(w.tgt_xyz[:, :300])
    a = ctx.compute_rates(t1, g1, tgt, None, 1.0, w.sigma, "fp64").cpu().numpy()
    b = ctx.compute_rates(t2, g2, tgt, None, 1.0, w.sigma, "fp64").cpu().numpy()
    assert np.array_equal(a, b)
    if sx.shape[1] == 0:
        assert not b.any()
    for o in (t1, g1, t2, g2):
        o.free()


def test_pooled_blocks_give_way_under_a_budget():
    """Under an HBM budget that holds one scene and its rate call but not two,
    scenes of alternating sizes build and run one after another: blocks kept
    for reuse are handed back to the device when a request of another size
    needs the room."""
    from paper_1005_5312_amd import workloads as W
    wa = W.make_small(seed=3, n_gas=4096, n_src=64)
    wb = W.make_small(seed=4, n_gas=8192, n_src=256)
    need = max(B.estimate_bytes(w.n_tgt, w.n_src, w.n_gas, w.grid_log2) for w in (wa, wb))
    with B.Context(0, hbm_budget=int(need * 1.3)) as c:
        ref = {}
        for k in range(6):
            w = (wa, wb)[k % 2]
            box = H.box_of(w)
            t, g = c.build_scene(box, dev(w.src_xyz), dev(w.src_lum), dev(w.gas_xyz), dev(w.gas_h),
                                 dev(w.gas_nhi), w.grid_log2)
            out = c.compute_rates(t, g, dev(w.tgt_xyz), None, 1.0, w.sigma, "fp32c").cpu().numpy()
            if k < 2:
                ref[k % 2] = out
            assert np.array_equal(out, ref[k % 2])
            t.free()
            g.free()
