"""Full-size parity: the diffuse (2^20 emitters + star) and shadow (2^21
emitters + star, 16 dense clumps) workloads, rate call exactly as bench.py
launches it, checked on seeded samples of targets that the oracle computes
one by one (with its own tree and grid)."""
import numpy as np
import pytest

from oracle import oracle as O
from tests import gpu_common as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    import paper_1005_5312_amd as S
    c = S.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("name,sample", [("diffuse", 768), ("shadow", 512)])
def test_fullsize_sampled(ctx, name, sample):
    w = H.workload(name)
    print(f"[case] full size {name}: {w.n_tgt} targets, {w.n_src} sources", flush=True)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    box = H.box_of(w)
    tree = ctx.build_source_tree(box, d(w.src_xyz), d(w.src_lum))
    grid = ctx.build_gas_grid(box, d(w.gas_xyz), d(w.gas_h), d(w.gas_nhi), w.grid_log2)
    tgt, ss = d(w.tgt_xyz), d(w.self_src)
    g32 = ctx.compute_rates(tree, grid, tgt, ss, 1.0, w.sigma, "fp32c").cpu().numpy()
    g64 = ctx.compute_rates(tree, grid, tgt, ss, 1.0, w.sigma, "fp64").cpu().numpy()
    ctx.synchronize()
    assert np.all(np.isfinite(g32)) and np.all(np.isfinite(g64))
    assert np.all(g32 >= 0) and np.all(g64 >= 0)
    obox = H.obox_of(w)
    ot = O.Tree(obox, w.src_xyz, w.src_lum)
    og = O.grid(obox, w.gas_xyz, w.gas_h, w.gas_nhi, w.grid_log2)
    # the sample: seeded uniform draws plus the targets inside dense clumps or
    # deepest in the neutral shell, where FP32 errors would show first
    idx = H.W.sample_indices(w.n_tgt, sample, seed=101)
    dense = np.argsort(-w.gas_nhi)[: sample // 8]
    idx = np.unique(np.concatenate([idx, dense]))
    want = O.rates(ot, w.grid_log2, og, w.tgt_xyz[:, idx], w.self_src[idx], 1.0, w.sigma)
    r64 = H.rel_errors(g64[idx], want)
    r32 = H.rel_errors(g32[idx].astype(np.float64), want)
    print(f"  fp64 max rel {r64[0]:.3e} (abs below floor {r64[1]:.1e}); "
          f"fp32c max rel {r32[0]:.3e} (abs below floor {r32[1]:.1e}) over {r32[2]} targets", flush=True)
    assert r64[0] <= H.TOL_FP64 and r64[1] <= H.ABS_FLOOR
    assert r32[0] <= H.TOL_FP32C and r32[1] <= H.ABS_FLOOR
    # the grid itself on sampled cells (brute force over all particles)
    cells = H.W.sample_indices((1 << w.grid_log2) ** 3, 256, seed=5)
    gw = O.grid_cells(obox, w.gas_xyz, w.gas_h, w.gas_nhi, w.grid_log2, cells)
    gg = ctx.grid_export(grid).reshape(-1)[cells]
    nz = gw != 0
    assert np.array_equal(gg == 0, gw == 0)
    assert np.max(np.abs(gg[nz] / gw[nz] - 1)) <= 1e-12


def test_fullsize_kernel_luminosity(ctx):
    """The kernel-weighted luminosities (volume form) of every node of the
    2^20 + 1-source benchmark tree against the oracle's cells, and the FP32C
    rates on that tree on sampled targets, in the launch configuration the
    benchmark times."""
    w = H.workload("diffuse")
    print(f"[case] full size kernel luminosity: {w.n_src} sources", flush=True)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    h, vol = H.W.source_kernel_inputs(w)
    box = H.box_of(w)
    tree = ctx.build_source_tree(box, d(w.src_xyz), d(w.src_lum))
    ctx.tree_kernel_luminosity(tree, 2, d(h), d(vol))
    grid = ctx.build_gas_grid(box, d(w.gas_xyz), d(w.gas_h), d(w.gas_nhi), w.grid_log2)
    g32 = ctx.compute_rates(tree, grid, d(w.tgt_xyz), d(w.self_src), 1.0, w.sigma, "fp32c").cpu().numpy()
    e = ctx.tree_export(tree)
    obox = H.obox_of(w)
    ot = O.Tree(obox, w.src_xyz, w.src_lum).kernel_luminosity(h, vol, 2)
    oe = ot.export()
    want = {(int(oe["level"][i]),) + tuple(int(v) for v in oe["coord"][i]): oe["lum"][i]
            for i in range(len(oe["level"]))}
    geo, mom = e["geo"], e["mom"]
    multi = (geo[:, 3] >> 8) != 2
    got = mom[multi, 3]
    ref = np.array([want[(int(g[3] & 0xFF), int(g[0]), int(g[1]), int(g[2]))] for g in geo[multi]])
    assert np.array_equal(got == 0, ref == 0)
    nz = ref != 0
    worst = float(np.max(np.abs(got[nz] / ref[nz] - 1)))
    print(f"  {int(multi.sum())} cells, max rel {worst:.2e}", flush=True)
    assert worst <= 1e-10
    og = O.grid(obox, w.gas_xyz, w.gas_h, w.gas_nhi, w.grid_log2)
    idx = H.W.sample_indices(w.n_tgt, 256, seed=103)
    wr = O.rates(ot, w.grid_log2, og, w.tgt_xyz[:, idx], w.self_src[idx], 1.0, w.sigma)
    r32 = H.rel_errors(g32[idx].astype(np.float64), wr)
    print(f"  fp32c max rel {r32[0]:.3e} over {r32[2]} targets", flush=True)
    assert r32[0] <= H.TOL_FP32C and r32[1] <= H.ABS_FLOOR


@pytest.mark.parametrize("name", ["diffuse", "shadow"])
def test_fullsize_tree_and_lists_bit_exact(ctx, name):
    """The 2^20 + 1 and 2^21 + 1 source trees the benchmark builds: Morton
    keys and source order against the definition and against the oracle's
    own member order, the set of cells of two or more sources in both
    directions with their source ranges and moments, and the interaction
    lists of 1024 seeded targets (self excluded) bit for bit."""
    w = H.workload(name)
    print(f"[case] full-size tree {name}: {w.n_src} sources", flush=True)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    box = H.box_of(w)
    tree = ctx.build_source_tree(box, d(w.src_xyz), d(w.src_lum))
    e = ctx.tree_export(tree)
    perm = e["perm"].astype(np.int64)
    keys = H.morton_keys(w.src_xyz, w.box_lo, w.box_size)
    order = np.lexsort((np.arange(w.n_src), keys))
    assert np.array_equal(perm, order)
    assert np.array_equal(e["keys"], keys[order])

    ot = O.Tree(H.obox_of(w), w.src_xyz, w.src_lum)
    oe = ot.export()
    # the oracle splits cubes in octant (= Morton) order and keeps members in
    # index order, so its member order is the sorted order
    assert np.array_equal(oe["member_idx"], perm)
    geo, link, mom = e["geo"], e["link"], e["mom"]
    kind = geo[:, 3] >> 8
    level = geo[:, 3] & 0xFF
    multi = kind != 2
    g_rows = np.stack([level[multi], geo[multi, 0], geo[multi, 1], geo[multi, 2]], axis=1).astype(np.int64)
    canon = (oe["count"] >= 2) & ((oe["nchild"] >= 2) | (oe["level"] == 21))
    o_rows = np.concatenate([oe["level"][canon, None].astype(np.int64), oe["coord"][canon]], axis=1)
    gs = np.lexsort(g_rows.T[::-1])
    os_ = np.lexsort(o_rows.T[::-1])
    assert g_rows.shape == o_rows.shape
    assert np.array_equal(g_rows[gs], o_rows[os_])           # the same cells, both directions
    g_first, g_count = link[multi, 1][gs], link[multi, 2][gs]
    assert np.array_equal(g_first, oe["member_off"][canon][os_])
    assert np.array_equal(g_count, oe["count"][canon][os_])
    n_mem = g_count.astype(np.float64)
    gl, ol = mom[multi, 3][gs], oe["lum"][canon][os_]
    assert np.all(np.abs(gl - ol) <= 4e-16 * n_mem * ol)
    gc, oc = mom[multi, :3][gs], oe["com"][canon][os_]
    assert np.all(np.abs(gc - oc) <= (4e-16 * n_mem[:, None] + 2e-16) * w.box_size)
    assert int((kind == 2).sum()) == int((oe["count"] == 1).sum())
    leaf = kind == 2
    assert np.array_equal(perm[link[leaf, 1]], link[leaf, 3])   # a single source is itself
    print(f"  {int(multi.sum())} cells of >= 2 sources, {int(leaf.sum())} single sources: identical", flush=True)

    idx = H.W.sample_indices(w.n_tgt, 1024, seed=211)
    tgt = np.ascontiguousarray(w.tgt_xyz[:, idx])
    ss = w.self_src[idx]
    off, ent = ctx.interaction_lists(tree, d(tgt), d(ss), 1.0)
    ooff, oent = ot.lists(tgt, ss, 1.0)
    assert np.array_equal(off, ooff)
    assert np.array_equal(H.gpu_entries_as_cells(ent, geo), oent)
    print(f"  lists of {len(idx)} targets: {int(off[-1])} entries identical", flush=True)


def test_fullsize_upstream_chain(ctx):
    """The upstream-particle chain at the size the benchmark runs it (the
    clumpy medium: 2^18 particles, 1024 sources, theta = 1, ~3.8e7 pairs):
    list offsets, the upstream particle of every pair and the number of pairs
    integrated along the ray bit for bit, rates to the FP64 tolerance."""
    w = H.workload("clumpy")
    print(f"[case] full-size upstream chain: {w.n_gas} particles, {w.n_src} sources", flush=True)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    box = H.box_of(w)
    tree = ctx.build_source_tree(box, d(w.src_xyz), d(w.src_lum))
    grid = ctx.build_gas_grid(box, d(w.gas_xyz), d(w.gas_h), d(w.gas_nhi), w.grid_log2)
    gam, offs, par, roots = ctx.compute_rates_upstream(tree, grid, d(w.gas_xyz), d(w.gas_h), d(w.gas_nhi), None,
                                                       1.0, w.sigma, structure=True)
    gam = gam.cpu().numpy()
    print(f"  GPU: {int(offs[-1])} pairs, {roots} along the ray; oracle running", flush=True)
    ob = H.obox_of(w)
    otree = O.Tree(ob, w.src_xyz, w.src_lum)
    ogrid = O.grid(ob, w.gas_xyz, w.gas_h, w.gas_nhi, w.grid_log2)
    want, ooffs, opar, ost = O.upstream_rates(otree, w.grid_log2, ogrid, w.gas_xyz, w.gas_h, w.gas_nhi, None, 1.0,
                                              w.sigma, structure=True)
    assert np.array_equal(offs, ooffs)
    assert np.array_equal(par, opar)
    assert roots == int(ost[:, 1].sum())
    rel, ab, nbig = H.rel_errors(gam, want)
    print(f"  parents identical; max rel {rel:.2e} over {nbig} particles", flush=True)
    assert rel <= H.TOL_FP64 and ab <= H.ABS_FLOOR
