"""GPU parity: the HIP library against the CPU FP64 oracle, through the C-ABI.

Bit-exact: Morton keys, source order, octree cells, interaction lists.
FP64 path: grid rel 1e-12, Gamma rel 1e-5.  FP32C path: Gamma rel 2e-4 above
Gamma* = 1e-30 s^-1 and |Gamma - Gamma*| <= 2e-34 below it.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests import gpu_common as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    import paper_1005_5312_amd as S
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = S.Context(0)
    yield c
    c.close()


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def build(ctx, w):
    tree = ctx.build_source_tree(H.box_of(w), dev(w.src_xyz), dev(w.src_lum))
    grid = ctx.build_gas_grid(H.box_of(w), dev(w.gas_xyz), dev(w.gas_h), dev(w.gas_nhi), w.grid_log2)
    return tree, grid


# ---------------------------------------------------------------- tree ---

@pytest.mark.parametrize("name", ["small", "clumpy"])
def test_keys_and_order_bit_exact(ctx, name):
    w = H.workload(name)
    print(f"[case] keys {name} n_s={w.n_src}", flush=True)
    tree = ctx.build_source_tree(H.box_of(w), dev(w.src_xyz), dev(w.src_lum))
    e = ctx.tree_export(tree)
    keys = H.morton_keys(w.src_xyz, w.box_lo, w.box_size)
    order = np.lexsort((np.arange(w.n_src), keys))
    assert np.array_equal(e["perm"].astype(np.int64), order)
    assert np.array_equal(e["keys"], keys[order])


def _oracle_cells(ot):
    e = ot.export()
    cells = {}
    for i in range(len(e["level"])):
        key = (int(e["level"][i]),) + tuple(int(v) for v in e["coord"][i])
        mem = e["member_idx"][e["member_off"][i]: e["member_off"][i] + e["count"][i]]
        cells[key] = (np.sort(mem), int(e["nchild"][i]), e["lum"][i], e["com"][i])
    return cells


@pytest.mark.parametrize("name", ["small", "clumpy"])
def test_tree_cells_and_moments(ctx, name):
    w = H.workload(name)
    print(f"[case] tree {name}", flush=True)
    tree = ctx.build_source_tree(H.box_of(w), dev(w.src_xyz), dev(w.src_lum))
    e = ctx.tree_export(tree)
    cells = _oracle_cells(O.Tree(H.obox_of(w), w.src_xyz, w.src_lum))
    geo, link, mom, perm = e["geo"], e["link"], e["mom"], e["perm"].astype(np.int64)
    m = geo.shape[0]
    kind = geo[:, 3] >> 8
    level = geo[:, 3] & 0xFF
    seen = set()
    for p in range(m):
        key = (int(level[p]), int(geo[p, 0]), int(geo[p, 1]), int(geo[p, 2]))
        mem, nchild, lum, com = cells[key]
        first, count = link[p, 1], link[p, 2]
        assert np.array_equal(np.sort(perm[first:first + count]), mem)
        if kind[p] == 2:      # single source: used as itself
            assert count == 1 and link[p, 3] == mem[0]
            j = mem[0]
            assert mom[p, 3] == w.src_lum[j]
            assert np.array_equal(mom[p, :3], w.src_xyz[:, j])
        else:
            assert (nchild >= 2) if kind[p] == 0 else (key[0] == 21)
            n = len(mem)
            assert abs(mom[p, 3] - lum) <= 4e-16 * n * lum
            assert np.all(np.abs(mom[p, :3] - com) <= (4e-16 * n + 2e-16) * w.box_size)
            seen.add(key)
        # depth-first order: the subtree ends at skip
        sk = link[p, 0]
        assert p < sk <= m
        if sk < m:
            assert link[sk, 1] >= first + count
        if p + 1 < sk:
            assert link[p + 1, 1] >= first and link[sk - 1, 1] + link[sk - 1, 2] <= first + count
    canon = {k for k, v in cells.items() if len(v[0]) >= 2 and (v[1] >= 2 or k[0] == 21)}
    assert canon == seen
    assert (kind == 2).sum() == sum(1 for v in cells.values() if len(v[0]) == 1)


# --------------------------------------------------------------- lists ---

@pytest.mark.parametrize("theta", [0.0, 0.5, 1.0])
def test_lists_bit_exact_small(ctx, theta):
    w = H.workload("small")
    print(f"[case] lists small theta={theta}", flush=True)
    oc = H.oracle_case("small")
    tree = ctx.build_source_tree(H.box_of(w), dev(w.src_xyz), dev(w.src_lum))
    geo = ctx.tree_export(tree)["geo"]
    off, ent = ctx.interaction_lists(tree, dev(w.tgt_xyz), None, theta)
    ooff, oent = oc.tree.lists(w.tgt_xyz, None, theta)
    assert np.array_equal(off, ooff)
    assert np.array_equal(H.gpu_entries_as_cells(ent, geo), oent)


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.8, 1.0])
def test_lists_bit_exact_clumpy_subset(ctx, theta):
    w = H.workload("clumpy")
    print(f"[case] lists clumpy theta={theta}", flush=True)
    idx = H.W.sample_indices(w.n_tgt, 3000, seed=11)
    tgt = np.ascontiguousarray(w.tgt_xyz[:, idx])
    tree = ctx.build_source_tree(H.box_of(w), dev(w.src_xyz), dev(w.src_lum))
    geo = ctx.tree_export(tree)["geo"]
    off, ent = ctx.interaction_lists(tree, dev(tgt), None, theta)
    ot = O.Tree(H.obox_of(w), w.src_xyz, w.src_lum)
    ooff, oent = ot.lists(tgt, None, theta)
    assert np.array_equal(off, ooff)
    assert np.array_equal(H.gpu_entries_as_cells(ent, geo), oent)


def test_lists_diffuse_self_excluded(ctx):
    """Every particle an emitter: lists of sampled targets are exact and never
    hold the target's own source."""
    w = H.workload("small")
    # small diffuse case: 4096 emitters + star, self = own index
    d = H.W.make_diffuse(seed=5, n_gas=4096)
    idx = H.W.sample_indices(d.n_tgt, 500, seed=3)
    tgt = np.ascontiguousarray(d.tgt_xyz[:, idx])
    ss = d.self_src[idx]
    tree = ctx.build_source_tree(H.box_of(d), dev(d.src_xyz), dev(d.src_lum))
    geo = ctx.tree_export(tree)["geo"]
    off, ent = ctx.interaction_lists(tree, dev(tgt), dev(ss), 1.0)
    ooff, oent = O.Tree(H.obox_of(d), d.src_xyz, d.src_lum).lists(tgt, ss, 1.0)
    assert np.array_equal(off, ooff)
    rows = H.gpu_entries_as_cells(ent, geo)
    assert np.array_equal(rows, oent)
    for i in range(len(idx)):
        r = rows[off[i]:off[i + 1]]
        assert not np.any((r[:, 0] == -1) & (r[:, 1] == ss[i]))
    del w


# ---------------------------------------------------------------- grid ---

@pytest.mark.parametrize("name", ["small", "clumpy"])
def test_grid_parity(ctx, name):
    w = H.workload(name)
    print(f"[case] grid {name} G={1 << w.grid_log2}", flush=True)
    grid = ctx.build_gas_grid(H.box_of(w), dev(w.gas_xyz), dev(w.gas_h), dev(w.gas_nhi), w.grid_log2)
    got = ctx.grid_export(grid)
    want = H.oracle_case(name).grid if name == "small" else O.grid(H.obox_of(w), w.gas_xyz, w.gas_h,
                                                                     w.gas_nhi, w.grid_log2)
    assert np.array_equal(got == 0, want == 0)
    nz = want != 0
    assert np.max(np.abs(got[nz] / want[nz] - 1)) <= 1e-12


@pytest.mark.parametrize("case", ["log_h", "bin_edges"])
def test_grid_parity_wide_smoothing_lengths(ctx, case):
    """Smoothing lengths spread over a factor ~20 (several reach classes of
    the binning), and particles on cell faces with 2h on the quarter-cell
    class edges: every cell still sees every particle whose support reaches
    it (same zero pattern, rel 1e-12)."""
    rng = np.random.default_rng(61)
    G = 32
    size = 6.6
    delta = size / G
    n = 700                 # sparse enough to leave cells uncovered
    if case == "log_h":
        xyz = rng.random((3, n)) * size
        h = delta * np.exp(rng.uniform(np.log(0.15), np.log(3.0), n))
    else:
        # positions on cell faces and corners, 2h = k/4 cells exactly
        xyz = rng.integers(0, G + 1, (3, n)) * delta
        h = 0.5 * delta * rng.integers(1, 17, n) / 4.0
    nhi = 10 ** rng.uniform(-5, -2, n)
    print(f"[case] grid {case} G={G}", flush=True)
    box = O.make_box([0.0, 0.0, 0.0], size, 3.0856775814913673e21)
    from paper_1005_5312_amd import Box
    grid = ctx.build_gas_grid(Box((0.0, 0.0, 0.0), size, 3.0856775814913673e21), dev(xyz), dev(h), dev(nhi), 5)
    got = ctx.grid_export(grid)
    want = O.grid(box, xyz, h, nhi, 5)
    assert np.array_equal(got == 0, want == 0)
    nz = want != 0
    assert 0.5 < nz.mean() < 0.95
    assert np.max(np.abs(got[nz] / want[nz] - 1)) <= 1e-12


# --------------------------------------------------------------- rates ---

@pytest.mark.parametrize("theta", [0.0, 0.5, 1.0])
@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_rates_small(ctx, theta, prec):
    w = H.workload("small")
    print(f"[case] rates small theta={theta} {prec}", flush=True)
    oc = H.oracle_case("small")
    tree, grid = build(ctx, w)
    got = ctx.compute_rates(tree, grid, dev(w.tgt_xyz), None, theta, w.sigma, prec)
    ctx.synchronize()
    want = oc.rates(theta)
    rel, ab, nbig = H.rel_errors(got.cpu().numpy(), want)
    print(f"  max rel {rel:.3e} over {nbig}, max abs below floor {ab:.3e}")
    assert rel <= (H.TOL_FP64 if prec == "fp64" else H.TOL_FP32C)
    assert ab <= H.ABS_FLOOR


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.8, 1.0])
@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_rates_clumpy_sampled(ctx, theta, prec):
    w = H.workload("clumpy")
    print(f"[case] rates clumpy theta={theta} {prec}", flush=True)
    tree, grid = build(ctx, w)
    got = ctx.compute_rates(tree, grid, dev(w.tgt_xyz), None, theta, w.sigma, prec)
    ctx.synchronize()
    idx = H.W.sample_indices(w.n_tgt, 1500, seed=7)
    ot = O.Tree(H.obox_of(w), w.src_xyz, w.src_lum)
    want = O.rates(ot, w.grid_log2, O.grid(H.obox_of(w), w.gas_xyz, w.gas_h, w.gas_nhi, w.grid_log2),
                   w.tgt_xyz[:, idx], None, theta, w.sigma)
    rel, ab, nbig = H.rel_errors(got.cpu().numpy()[idx], want)
    print(f"  max rel {rel:.3e} over {nbig}, max abs below floor {ab:.3e}")
    assert rel <= (H.TOL_FP64 if prec == "fp64" else H.TOL_FP32C)
    assert ab <= H.ABS_FLOOR


def test_theta_sweep_error_grows_with_theta(ctx):
    """Clumpy medium, all 2^18 particles: theta = 0 sums every source on its
    own and matches the oracle's exact sum on sampled particles; the error
    of the tree approximation against it grows with theta."""
    w = H.workload("clumpy")
    print("[case] theta sweep clumpy", flush=True)
    tree, grid = build(ctx, w)
    tgt = dev(w.tgt_xyz)
    g0 = ctx.compute_rates(tree, grid, tgt, None, 0.0, w.sigma, "fp64").cpu().numpy()
    idx = H.W.sample_indices(w.n_tgt, 400, seed=3)
    want = O.rates(O.Tree(H.obox_of(w), w.src_xyz, w.src_lum), w.grid_log2,
                   O.grid(H.obox_of(w), w.gas_xyz, w.gas_h, w.gas_nhi, w.grid_log2), w.tgt_xyz[:, idx], None, 0.0,
                   w.sigma)
    rel, ab, _ = H.rel_errors(g0[idx], want)
    assert rel <= H.TOL_FP64 and ab <= H.ABS_FLOOR
    med = []
    for theta in (0.3, 0.5, 0.8, 1.0):
        g = ctx.compute_rates(tree, grid, tgt, None, theta, w.sigma, "fp32c").cpu().numpy().astype(np.float64)
        e = np.abs(g / g0 - 1)
        med.append(float(np.median(e)))
        print(f"  theta {theta}: median rel err vs theta 0 {med[-1]:.2e}, p99 {np.percentile(e, 99):.2e}")
    assert all(a < b for a, b in zip(med, med[1:]))


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_rates_diffuse_small_self(ctx, prec):
    """Diffuse emitters with self exclusion and a central star on grid planes."""
    d = H.W.make_diffuse(seed=5, n_gas=1 << 14)
    print(f"[case] rates diffuse 2^14 {prec}", flush=True)
    tree, grid = build(ctx, d)
    got = ctx.compute_rates(tree, grid, dev(d.tgt_xyz), dev(d.self_src), 1.0, d.sigma, prec)
    ctx.synchronize()
    idx = H.W.sample_indices(d.n_tgt, 2000, seed=2)
    oc = H.OracleCase(d)
    want = oc.rates(1.0, idx)
    rel, ab, nbig = H.rel_errors(got.cpu().numpy()[idx], want)
    print(f"  max rel {rel:.3e} over {nbig}, max abs below floor {ab:.3e}")
    assert rel <= (H.TOL_FP64 if prec == "fp64" else H.TOL_FP32C)
    assert ab <= H.ABS_FLOOR


def test_counters_match_oracle(ctx):
    w = H.workload("small")
    print("[case] counters small", flush=True)
    oc = H.oracle_case("small")
    tree, grid = build(ctx, w)
    for theta in (0.5, 1.0):
        got = ctx.rate_counters(tree, grid, dev(w.tgt_xyz), None, theta, "fp64")
        _, want = O.rates(oc.tree, w.grid_log2, oc.grid, w.tgt_xyz, None, theta, w.sigma, counters=True)
        assert np.array_equal(got[:, 0], want[:, 0])     # opening tests
        assert np.array_equal(got[:, 1], want[:, 1])     # entries
        assert np.array_equal(got[:, 3], want[:, 3])     # zero-distance skips
        # grid cells crossed: equal up to crossings that coincide in rounding
        assert np.abs(got[:, 2] - want[:, 2]).max() <= 2 + want[:, 2].max() // 1000


# ---------------------------------------------------------- edge cases ---

def test_ragged_tail_and_empty(ctx):
    """Target counts that are not multiples of the 64-lane tile, n = 0, and
    trees with no or one source."""
    w = H.workload("small")
    oc = H.oracle_case("small")
    tree, grid = build(ctx, w)
    for n in (1, 63, 65, 130, 1001):
        print(f"[case] ragged n={n}", flush=True)
        got = ctx.compute_rates(tree, grid, dev(w.tgt_xyz[:, :n]), None, 1.0, w.sigma, "fp64")
        ctx.synchronize()
        want = oc.rates(1.0, np.arange(n))
        assert H.rel_errors(got.cpu().numpy(), want)[0] <= H.TOL_FP64
    out = ctx.compute_rates(tree, grid, dev(np.zeros((3, 0))), None, 1.0, w.sigma, "fp64")
    assert out.numel() == 0
    box = H.box_of(w)
    empty = ctx.build_source_tree(box, dev(np.zeros((3, 0))), dev(np.zeros(0)))
    got = ctx.compute_rates(empty, grid, dev(w.tgt_xyz[:, :100]), None, 1.0, w.sigma, "fp32c")
    ctx.synchronize()
    assert torch.all(got == 0)
    one = ctx.build_source_tree(box, dev(w.src_xyz[:, :1]), dev(w.src_lum[:1]))
    ot = O.Tree(H.obox_of(w), w.src_xyz[:, :1], w.src_lum[:1])
    for prec, tol in (("fp64", H.TOL_FP64), ("fp32c", H.TOL_FP32C)):
        got = ctx.compute_rates(one, grid, dev(w.tgt_xyz), None, 0.7, w.sigma, prec)
        ctx.synchronize()
        want = O.rates(ot, w.grid_log2, oc.grid, w.tgt_xyz, None, 0.7, w.sigma)
        rel, ab, _ = H.rel_errors(got.cpu().numpy(), want)
        assert rel <= tol and ab <= H.ABS_FLOOR


def test_coincident_sources_and_faces(ctx):
    """Coincident sources form a level-21 bucket; targets on the box faces,
    corners and grid planes."""
    w = H.workload("small")
    oc = H.oracle_case("small")
    src = np.concatenate([w.src_xyz, np.repeat(w.src_xyz[:, :1], 3, axis=1),
                          np.array([[0.0, 6.6, 3.3], [0.0, 6.6, 3.3], [3.3, 3.3, 3.3]])], axis=1)
    lum = np.concatenate([w.src_lum, [1e48, 2e48, 0.0], [3e48, 4e48, 1e49]])
    tgt = np.array([[0.0, 6.6, 3.3, 0.0, 6.6, 3.3, 0.4125, 1.2],
                    [0.0, 6.6, 3.3, 6.6, 0.0, 0.0, 0.4125, 2.475],
                    [0.0, 6.6, 3.3, 3.3, 6.6, 1.0, 0.825, 6.6]])
    tree = ctx.build_source_tree(H.box_of(w), dev(src), dev(lum))
    geo = ctx.tree_export(tree)["geo"]
    ot = O.Tree(H.obox_of(w), src, lum)
    for theta in (0.0, 1.0):
        off, ent = ctx.interaction_lists(tree, dev(tgt), None, theta)
        ooff, oent = ot.lists(tgt, None, theta)
        assert np.array_equal(off, ooff)
        assert np.array_equal(H.gpu_entries_as_cells(ent, geo), oent)
        for prec, tol in (("fp64", H.TOL_FP64), ("fp32c", H.TOL_FP32C)):
            got = ctx.compute_rates(tree, ctx.build_gas_grid(H.box_of(w), dev(w.gas_xyz), dev(w.gas_h),
                                                             dev(w.gas_nhi), w.grid_log2),
                                    dev(tgt), None, theta, w.sigma, prec)
            ctx.synchronize()
            want = O.rates(ot, w.grid_log2, oc.grid, tgt, None, theta, w.sigma)
            rel, ab, _ = H.rel_errors(got.cpu().numpy(), want)
            assert rel <= tol and ab <= H.ABS_FLOOR


def test_input_errors(ctx):
    import paper_1005_5312_amd as S
    w = H.workload("small")
    tree, grid = build(ctx, w)
    bad = w.tgt_xyz[:, :10].copy()
    bad[1, 3] = np.nan
    ctx.compute_rates(tree, grid, dev(bad), None, 1.0, w.sigma, "fp64")
    with pytest.raises(S.StartError) as e:
        ctx.synchronize()
    assert e.value.code == S.binding.ENONFINITE
    bad[1, 3] = 7.0
    ctx.compute_rates(tree, grid, dev(bad), None, 1.0, w.sigma, "fp64")
    with pytest.raises(S.StartError) as e:
        ctx.synchronize()
    assert e.value.code == S.binding.EOUTOFBOX
    ctx.compute_rates(tree, grid, dev(w.tgt_xyz[:, :10]), dev(np.full(10, 99, np.int64)), 1.0, w.sigma, "fp64")
    with pytest.raises(S.StartError) as e:
        ctx.synchronize()
    assert e.value.code == S.binding.EINVAL
    with pytest.raises(S.StartError) as e:
        ctx.compute_rates(tree, grid, dev(w.tgt_xyz[:, :10]), None, -1.0, w.sigma, "fp64")
    assert e.value.code == S.binding.EINVAL
    with pytest.raises(S.StartError) as e:
        ctx.build_source_tree(H.box_of(w), dev(w.src_xyz), dev(-w.src_lum))
    assert e.value.code == S.binding.EINVAL
    srcb = w.src_xyz.copy()
    srcb[0, 0] = -1.0
    with pytest.raises(S.StartError) as e:
        ctx.build_source_tree(H.box_of(w), dev(srcb), dev(w.src_lum))
    assert e.value.code == S.binding.EOUTOFBOX
    with pytest.raises(S.StartError) as e:
        ctx.build_gas_grid(H.box_of(w), dev(w.gas_xyz), dev(-w.gas_h), dev(w.gas_nhi), 4)
    assert e.value.code == S.binding.EINVAL
    # still usable afterwards
    ctx.compute_rates(tree, grid, dev(w.tgt_xyz[:, :10]), None, 1.0, w.sigma, "fp64")
    ctx.synchronize()


def test_batched_equals_single(ctx):
    w = H.workload("small")
    d = H.W.make_diffuse(seed=9, n_gas=3000)
    t1, g1 = build(ctx, w)
    t2, g2 = build(ctx, d)
    single = [ctx.compute_rates(t1, g1, dev(w.tgt_xyz), None, 1.0, w.sigma, "fp32c"),
              ctx.compute_rates(t2, g2, dev(d.tgt_xyz), dev(d.self_src), 1.0, d.sigma, "fp64")]
    ctx.synchronize()
    outs = [torch.empty(w.n_tgt, dtype=torch.float32, device="cuda"),
            torch.empty(d.n_tgt, dtype=torch.float64, device="cuda")]
    ctx.compute_rates_batched([
        dict(tree=t1, grid=g1, tgt_xyz=dev(w.tgt_xyz), self_src=None, theta=1.0, sigma=w.sigma, prec="fp32c",
             out=outs[0]),
        dict(tree=t2, grid=g2, tgt_xyz=dev(d.tgt_xyz), self_src=dev(d.self_src), theta=1.0, sigma=d.sigma,
             prec="fp64", out=outs[1])])
    ctx.synchronize()
    for a, b in zip(single, outs):
        assert torch.equal(a, b)


def test_deterministic(ctx):
    w = H.workload("small")
    tree, grid = build(ctx, w)
    a = ctx.compute_rates(tree, grid, dev(w.tgt_xyz), None, 1.0, w.sigma, "fp32c").clone()
    b = ctx.compute_rates(tree, grid, dev(w.tgt_xyz), None, 1.0, w.sigma, "fp32c")
    ctx.synchronize()
    assert torch.equal(a, b)


def test_batched_many_uneven_items_bitwise(ctx):
    """One persistent launch over many uneven items (sizes, thetas, both
    precisions, shared and separate trees) gives each item exactly what a
    call of its own gives."""
    rng = np.random.default_rng(3)
    base = H.workload("small")
    d = H.W.make_diffuse(seed=13, n_gas=5000)
    t1, g1 = build(ctx, base)
    t2, g2 = build(ctx, d)
    items, singles = [], []
    for k in range(23):
        use_d = k % 3 == 0
        w, t, g = (d, t2, g2) if use_d else (base, t1, g1)
        n = int(rng.integers(1, 700))
        idx = np.sort(rng.choice(w.n_tgt, size=n, replace=False))
        tgt = dev(w.tgt_xyz[:, idx])
        ss = dev(w.self_src[idx]) if use_d else None
        theta = float(rng.choice([0.0, 0.4, 1.0, 1.3]))
        prec = "fp64" if k % 2 else "fp32c"
        dt = torch.float64 if prec == "fp64" else torch.float32
        out = torch.empty(n, dtype=dt, device="cuda")
        items.append(dict(tree=t, grid=g, tgt_xyz=tgt, self_src=ss, theta=theta, sigma=w.sigma, prec=prec, out=out))
        singles.append(ctx.compute_rates(t, g, tgt, ss, theta, w.sigma, prec).clone())
    ctx.synchronize()
    ctx.compute_rates_batched(items)
    ctx.synchronize()
    for it, ref in zip(items, singles):
        assert torch.equal(it["out"], ref)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_tile_size_does_not_change_results(ctx, prec):
    """Targets per wavefront from 1 (the wave on one target's rays) to 64:
    every target's terms are summed in its own depth-first order, so the
    rates are identical bit for bit."""
    w = H.workload("clumpy", n_gas=1 << 14, n_src=256)
    dev = ctx.device
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    box = H.box_of(w)
    tree = ctx.build_source_tree(box, d(w.src_xyz), d(w.src_lum))
    grid = ctx.build_gas_grid(box, d(w.gas_xyz), d(w.gas_h), d(w.gas_nhi), w.grid_log2)
    tgt = d(w.tgt_xyz[:, :3001])
    outs = {}
    try:
        for t in (64, 32, 7, 4, 1):
            ctx.set_tile_targets(t)
            outs[t] = ctx.compute_rates(tree, grid, tgt, None, 1.0, w.sigma, prec).cpu().numpy()
    finally:
        ctx.set_tile_targets(0)
    for t in outs:
        assert np.array_equal(outs[t], outs[64]), t


def test_autotune_picks_a_tile_and_keeps_results(ctx):
    w = H.workload("clumpy", n_gas=1 << 14, n_src=256)
    dev = ctx.device
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    box = H.box_of(w)
    tree = ctx.build_source_tree(box, d(w.src_xyz), d(w.src_lum))
    grid = ctx.build_gas_grid(box, d(w.gas_xyz), d(w.gas_h), d(w.gas_nhi), w.grid_log2)
    items = [dict(tree=tree, grid=grid, tgt_xyz=d(w.tgt_xyz[:, :2000]), self_src=None, theta=1.0, sigma=w.sigma,
                  prec="fp32c", out=torch.empty(2000, dtype=torch.float32, device=dev))]
    ref = ctx.compute_rates(tree, grid, items[0]["tgt_xyz"], None, 1.0, w.sigma, "fp32c").cpu().numpy()
    best, ms = ctx.autotune_rates(items, reps=2)
    print(f"  autotune 2000 targets: tile {best}, {ms:.3f} ms")
    assert best in (1, 4, 8, 16, 32, 64) and ms > 0
    assert np.array_equal(items[0]["out"].cpu().numpy(), ref)
    again = ctx.compute_rates(tree, grid, items[0]["tgt_xyz"], None, 1.0, w.sigma, "fp32c").cpu().numpy()
    assert np.array_equal(again, ref)


def _on_faces_edges_planes(rng, n, size, G):
    """n points whose coordinates are each, at random, on the lower or upper
    face of the box, on a grid plane, or anywhere."""
    p = rng.uniform(0.0, size, (3, n))
    kind = rng.integers(0, 4, (3, n))
    plane = np.floor(rng.uniform(0.0, size, (3, n)) / size * G) * (size / G)
    p = np.where(kind == 0, 0.0, np.where(kind == 1, size, np.where(kind == 2, plane, p)))
    return np.ascontiguousarray(p)


@pytest.mark.parametrize("grid_log2", [4, 6, 7])
def test_rays_ending_on_faces_edges_and_planes(ctx, grid_log2):
    """Sources and targets on the box's faces, edges and corners and on grid
    planes, so that rays end on the grid's boundary and the last turn of a
    march runs past it (into the grid's guard band), theta 0 and 1, both
    precisions, against the oracle."""
    rng = np.random.default_rng(100 + grid_log2)
    w = H.W.make_clumpy(seed=40 + grid_log2, n_gas=4096, n_src=8)
    G = 1 << grid_log2
    print(f"[case] faces, edges and planes, G = {G}", flush=True)
    src = np.concatenate([w.src_xyz, _on_faces_edges_planes(rng, 40, w.box_size, G)], axis=1)
    lum = 10.0 ** rng.uniform(47.0, 50.0, src.shape[1])
    tgt = _on_faces_edges_planes(rng, 400, w.box_size, G)
    box, obox = H.box_of(w), H.obox_of(w)
    tree = ctx.build_source_tree(box, dev(src), dev(lum))
    grid = ctx.build_gas_grid(box, dev(w.gas_xyz), dev(w.gas_h), dev(w.gas_nhi), grid_log2)
    ot = O.Tree(obox, src, lum)
    og = O.grid(obox, w.gas_xyz, w.gas_h, w.gas_nhi, grid_log2)
    for theta in (0.0, 1.0):
        want = O.rates(ot, grid_log2, og, tgt, None, theta, w.sigma)
        for prec, tol in (("fp64", H.TOL_FP64), ("fp32c", H.TOL_FP32C)):
            got = ctx.compute_rates(tree, grid, dev(tgt), None, theta, w.sigma, prec)
            ctx.synchronize()
            rel, ab, _ = H.rel_errors(got.cpu().numpy(), want)
            print(f"  theta {theta} {prec}: max rel {rel:.2e}", flush=True)
            assert rel <= tol and ab <= H.ABS_FLOOR


@pytest.mark.parametrize("grid_log2", [4, 6])
def test_rays_through_grid_edges_and_corners(ctx, grid_log2):
    """Sources and targets on grid vertices of a box of side 8, exact in both
    precisions' coordinates, so that the rays between them pass exactly
    through grid edges and corners: two or three plane parameters are equal
    at many crossings (at every one along the (1, 1, 0) and (1, 1, 1)
    diagonals), where the march moves one axis per step and the others
    follow with chords of length 0 (a reading of the paper's ray
    integration: the exact integral is unchanged).  Theta 0 and 1, both
    precisions, against the oracle, which sorts all crossings."""
    import dataclasses
    G = 1 << grid_log2
    side = 8.0
    print(f"[case] rays through grid edges and corners, G = {G}", flush=True)
    w0 = H.W.make_clumpy(seed=60 + grid_log2, n_gas=4096, n_src=8)
    k = side / w0.box_size
    w = dataclasses.replace(w0, box_size=side, gas_xyz=w0.gas_xyz * k, gas_h=w0.gas_h * k)
    rng = np.random.default_rng(70 + grid_log2)
    d = side / G
    src = rng.integers(1, G, (3, 12)).astype(np.float64) * d
    lum = 10.0 ** rng.uniform(47.0, 50.0, src.shape[1])
    dirs = np.array([[1, 1, 0], [1, 1, 1], [1, -1, 2], [2, 2, 1], [-1, 1, 1], [0, 1, 1]], np.float64)
    tg = [src[:, j] + m * v * d for j in range(4) for v in dirs for m in (1, 2, 3)]
    tg = [p for p in tg if np.all(p >= 0.0) and np.all(p <= side)]
    tgt = np.concatenate([np.array(tg).T, rng.integers(0, G + 1, (3, 64)).astype(np.float64) * d], axis=1)
    tgt = np.ascontiguousarray(tgt)
    box, obox = H.box_of(w), H.obox_of(w)
    tree = ctx.build_source_tree(box, dev(src), dev(lum))
    grid = ctx.build_gas_grid(box, dev(w.gas_xyz), dev(w.gas_h), dev(w.gas_nhi), grid_log2)
    ot = O.Tree(obox, src, lum)
    og = O.grid(obox, w.gas_xyz, w.gas_h, w.gas_nhi, grid_log2)
    for theta in (0.0, 1.0):
        want = O.rates(ot, grid_log2, og, tgt, None, theta, w.sigma)
        assert np.count_nonzero(want > H.FLOOR) > tgt.shape[1] // 2
        for prec, tol in (("fp64", H.TOL_FP64), ("fp32c", H.TOL_FP32C)):
            got = ctx.compute_rates(tree, grid, dev(tgt), None, theta, w.sigma, prec)
            ctx.synchronize()
            rel, ab, _ = H.rel_errors(got.cpu().numpy(), want)
            print(f"  theta {theta} {prec}: max rel {rel:.2e}", flush=True)
            assert rel <= tol and ab <= H.ABS_FLOOR


def test_largest_grids(ctx):
    """The largest grids: G = 512 (the largest with a guard band) against the
    oracle, on a sparse field (65536 particles with kernels of 0.6 cells, so
    the gather stays cheap at 512^3 centres; ~25 optical depths per filled
    cell), and G = 1024 (no band: the march clamps its offsets) in gas without
    neutral hydrogen, where the rate has the optically thin closed form
    L sigma / (4 pi d^2).  Targets also on faces, edges and grid planes."""
    rng = np.random.default_rng(7)
    w = H.W.make_small(seed=17, n_gas=1 << 16, n_src=1)
    src = np.concatenate([np.array([[1.7], [4.1], [2.9]]), np.array([[0.0], [6.6], [6.6]]),
                          _on_faces_edges_planes(rng, 1, w.box_size, 512)], axis=1)
    lum = np.array([5e48, 1e49, 2e48])
    tgt = np.concatenate([rng.uniform(0.0, w.box_size, (3, 300)), _on_faces_edges_planes(rng, 100, w.box_size, 512)],
                         axis=1)
    box, obox = H.box_of(w), H.obox_of(w)
    tree = ctx.build_source_tree(box, dev(src), dev(lum))
    ot = O.Tree(obox, src, lum)
    print("[case] G = 512, sparse field", flush=True)
    h = np.full(w.n_gas, 0.6 * w.box_size / 512)
    nhi = rng.uniform(0.05, 0.2, w.n_gas)
    grid = ctx.build_gas_grid(box, dev(w.gas_xyz), dev(h), dev(nhi), 9)
    og = O.grid(obox, w.gas_xyz, h, nhi, 9)
    want = O.rates(ot, 9, og, tgt, None, 0.0, w.sigma)
    del og
    for prec, tol in (("fp64", H.TOL_FP64), ("fp32c", H.TOL_FP32C)):
        got = ctx.compute_rates(tree, grid, dev(tgt), None, 0.0, w.sigma, prec)
        ctx.synchronize()
        rel, ab, nbig = H.rel_errors(got.cpu().numpy(), want)
        print(f"  {prec}: max rel {rel:.2e} over {nbig} targets", flush=True)
        assert rel <= tol and ab <= H.ABS_FLOOR
    grid.free()
    print("[case] G = 1024, no neutral gas", flush=True)
    grid = ctx.build_gas_grid(box, dev(w.gas_xyz), dev(h * 0.5), dev(np.zeros(w.n_gas)), 10)
    d = np.sqrt(((tgt[:, :, None] - src[:, None, :]) ** 2).sum(axis=0)) * w.length_unit_cm
    with np.errstate(divide="ignore"):
        want = np.where(d > 0, lum * w.sigma / (4 * np.pi * d * d), 0.0).sum(axis=1)   # a source at 0 is skipped
    for prec, tol in (("fp64", 1e-12), ("fp32c", 1e-5)):
        got = ctx.compute_rates(tree, grid, dev(tgt), None, 0.0, w.sigma, prec)
        ctx.synchronize()
        rel = float(np.max(np.abs(got.cpu().numpy().astype(np.float64) / want - 1)))
        print(f"  {prec}: max rel {rel:.2e}", flush=True)
        assert rel <= tol
    grid.free()
