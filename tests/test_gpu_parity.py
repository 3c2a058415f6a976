"""GPU parity: the HIP library through its C ABI against the FP64 oracle.

Bars: tree topology, keys, flags, integer fields and walk counts bit-exact; node FP32
fields bit-exact except those carrying the in-cell star extinction exp(-tau/2) (1 ulp);
J within 1e-4 relative; F per component within 1e-4 * 4 pi J; a_RP per component within
1e-4 (kappa / c) phi_RP 4 pi J of its cell; T_dust within 1e-5 relative of the FP64
bracketed root.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from workloads.synth import cell_centres

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_09072_amd as T
    return T


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


def say(*a):
    print(*a, flush=True)


# The one-block-per-target trace kernel (kernel = 2) is withdrawn: it was slower than the
# one-wave kernel on every workload measured, and a variant of its walk stopped making
# progress on the GPU without a cause that could be shown.  Its cases stay, skipped.
WITHDRAWN = "kernel 2 (one block per target) is withdrawn; the library rejects it"


def _k(*args):
    """A parameter set, skipped when its kernel (the last value) is the withdrawn one."""
    return pytest.param(*args, marks=pytest.mark.skip(reason=WITHDRAWN)) if args[-1] == 2 else pytest.param(*args)


def _amr_small(seed=3, stars=True):
    rng = np.random.default_rng(seed)
    blocks = []
    for bk in range(2):
        for bj in range(2):
            for bi in range(2):
                if (bi, bj, bk) in ((1, 1, 0), (0, 1, 1)):
                    for k in range(2):
                        for j in range(2):
                            for i in range(2):
                                blocks.append((1, 2 * bi + i, 2 * bj + j, 2 * bk + k))
                else:
                    blocks.append((0, bi, bj, bk))
    blocks = np.array(blocks, np.int32)
    n = blocks.shape[0] * 512
    st = np.array([[0.7, 0.7, 0.2, 3.0], [0.1, 0.2, 0.3, 1.0], [0.5, 0.5, 0.5, 2.0]]) if stars else np.zeros((0, 4))
    return W.Workload(name="amr-small", nb=2, max_level=1, blocks=blocks, x0=(0, 0, 0), box_len=1.0,
                      rho=(10 ** rng.uniform(-1, 1.7, n)).astype(np.float32),
                      t_dust=rng.uniform(0.5, 1.5, n).astype(np.float32),
                      kappa=np.ones(n, np.float32), stars=st, units=W.CODE_UNITS, n_side=2, theta=(1, 4))


def _padded(n=40, seed=5):
    """Non-power-of-two domain (root padded) with stars, lognormal density."""
    ss = np.random.SeedSequence(seed).spawn(3)
    g = W.grf(n, np.random.default_rng(ss[0]))
    rho = W.lognormal(g, 1.5)
    kap = 10.0 ** np.random.default_rng(ss[1]).uniform(-1, 1, rho.shape)
    t = np.random.default_rng(ss[2]).uniform(0.05, 0.2, rho.shape) ** 0.25
    from workloads.synth import _uniform_workload
    return _uniform_workload(f"pad{n}", rho, t, kap, n // 8, 1.0, W.CODE_UNITS, 2,
                             [[0.31, 0.62, 0.5, 1.0], [0.9, 0.1, 0.05, 0.5]])


TREE_CASES = {
    "sphere16": lambda: W.c1_sphere16(),
    "turb32": lambda: W.c2_turb64(n=32, n_side=2),
    "amr_small": lambda: _amr_small(),
    "padded40": lambda: _padded(),
    "core32": lambda: W.c3_core128(n=32, n_side=2),
}


# ----------------------------------------------------------------------------------
@pytest.mark.parametrize("ns", [1, 2, 4, 8])
def test_ray_tables_equal_oracle(lib, ctx, ns):
    say("ray tables n_side", ns)
    tab, dirs = lib.ray_tables(ctx, ns)
    assert np.array_equal(tab, oracle.cube_table(ns))
    assert np.abs(dirs - oracle.ray_dirs(ns)).max() < 1e-6


@pytest.mark.parametrize("ns", [1, 2, 4, 8])
def test_alpha_table_equal_oracle(lib, ctx, ns):
    """The tabulated angular kernel of distant nodes, built by the library from its pixel
    table in exact integers: every pixel, count and overflow flag equal to the oracle's."""
    say("alpha table n_side", ns)
    assert np.array_equal(lib.alpha_table(ctx, ns), oracle.alpha_table(ns))


@pytest.mark.parametrize("case", list(TREE_CASES))
def test_tree_bit_exact(lib, ctx, case):
    from paper_2204_09072_amd.run import tree_of, upload
    w = TREE_CASES[case]()
    say("tree", case, w.n_cells)
    dev = upload(w)
    tree = tree_of(ctx, w, dev)
    ot = oracle.Tree(w)
    assert (tree.n_node, tree.n_leaf, tree.depth, tree.root_edge, tree.n_bins) == \
           (ot.n_node, ot.n_leaf, ot.depth, ot.root_edge, ot.n_bins)
    assert tree.u_len == ot.u_len
    g = lib.tree_export(ctx, tree)
    o = ot.export()
    for k in ("geo", "meta", "leaf_cell"):
        assert np.array_equal(g[k], o[k]), k
    leaf = (o["meta"] >> 12) & 1 == 1
    # S-free fields bit-exact; the star term (exp(-tau/2)) may differ by one ulp
    has_src = np.zeros(len(leaf), bool)
    if w.stars.shape[0]:
        has_src = o["q"][:, 2] != 0
    q_g, q_o = g["q"], o["q"]
    exact = leaf & ~has_src
    assert np.array_equal(q_g[exact].view(np.uint32), q_o[exact].view(np.uint32))
    ulp = np.abs(q_g.view(np.int32).astype(np.int64) - q_o.view(np.int32).astype(np.int64))
    assert ulp[leaf].max() <= 1
    assert np.array_equal(g["vthick"].view(np.uint32), o["vthick"].view(np.uint32))
    if not w.stars.shape[0]:
        assert np.array_equal(q_g.view(np.uint32), q_o.view(np.uint32))
        assert np.array_equal(g["pcol"], o["pcol"])
    else:
        # h-node sums carry the star light: within 1 ulp; positions within one fixed-point step
        assert ulp[~leaf].max() <= 1
        assert np.abs(g["pcol"] - o["pcol"]).max() <= 1


@pytest.mark.parametrize("case", ["sphere16", "amr_small", "padded40"])
def test_walk_counts_equal_oracle(lib, ctx, case):
    import torch
    from paper_2204_09072_amd.run import params_of, tree_of, upload
    w = TREE_CASES[case]()
    say("walk counts", case)
    tree = tree_of(ctx, w, upload(w))
    cnt = torch.zeros((tree.n_cells, 3), dtype=torch.int32, device="cuda")
    lib.walk_counts(ctx, tree, params_of(w), cnt)
    ctx.sync()
    ot = oracle.Tree(w)
    _, _, oc = ot.trace(oracle.params(w.n_side, theta=w.theta), counters=True)
    assert np.array_equal(cnt.cpu().numpy(), oc.astype(np.int32))


def _check_trace(J, F, Jo, Fo):
    J = np.asarray(J, np.float64)
    rel = np.abs(J - Jo) / np.maximum(np.abs(Jo), 1e-300)
    bad = rel > 1e-4
    assert not bad.any(), f"J: {bad.sum()} cells off, worst rel {rel.max():.3e}"
    tolF = 1e-4 * 4 * np.pi * np.abs(Jo)[:, None]
    dF = np.abs(np.asarray(F, np.float64) - Fo)
    assert (dF <= tolF + 1e-30).all(), f"F: worst {np.max(dF / (tolF + 1e-30)):.3e} x tolerance"


# kernel 1: one wave per target (segments in passes); kernel 2: one block per target
@pytest.mark.parametrize("case,bpp,kernel", [_k(*c) for c in [
    ("sphere16", 0, 1), ("turb32", 0, 1), ("turb32", 3, 1), ("amr_small", 0, 1), ("amr_small", 2, 1),
    ("padded40", 0, 1), ("core32", 1, 1),
    ("sphere16", 0, 2), ("turb32", 0, 2), ("turb32", 5, 2), ("amr_small", 0, 2), ("amr_small", 3, 2),
    ("padded40", 0, 2), ("core32", 0, 2)]])
def test_trace_parity_all_targets(lib, ctx, case, bpp, kernel):
    from paper_2204_09072_amd.run import trace
    w = TREE_CASES[case]()
    say("trace", case, "bins_per_pass", bpp, "kernel", kernel)
    tree, J, F, U = trace(ctx, w, bins_per_pass=bpp, kernel=kernel)
    ctx.sync()
    ot = oracle.Tree(w)
    Jo, Fo = ot.trace(oracle.params(w.n_side, theta=w.theta))
    _check_trace(J.cpu().numpy(), F.cpu().numpy().T, Jo, Fo)
    assert np.allclose(U.cpu().numpy(), 4 * np.pi * J.cpu().numpy() / w.units[1], rtol=1e-6)


@pytest.mark.parametrize("case,kernel", [_k(*c) for c in [("turb32", 1), ("amr_small", 2), ("padded40", 1),
                                                          ("amr_small", 1)]])
def test_trace_parity_per_node_kernel(lib, ctx, case, kernel):
    """The per-node 8-point kernel for every node (no table) against the oracle run the
    same way."""
    from paper_2204_09072_amd.run import trace
    w = TREE_CASES[case]()
    say("trace per-node kernel", case, "kernel", kernel)
    tree, J, F, U = trace(ctx, w, kernel=kernel, per_node_kernel=True)
    ctx.sync()
    Jo, Fo = oracle.Tree(w).trace(oracle.params(w.n_side, theta=w.theta, alpha_table=False))
    _check_trace(J.cpu().numpy(), F.cpu().numpy().T, Jo, Fo)


EDGE_CASES = {
    # one 8^3 block: the smallest tree the builder accepts
    "single_block": lambda: W.small_uniform(8, 1.0, 1.0, 1.0, n_side=1),
    # every leaf optically thick (tau_b = 6.25): thick sums, merged runs carried across passes
    "thick_box": lambda: W.small_uniform(16, 100.0, 1.0, 1.0, n_side=2),
    # one thick blob in an empty box: zero content almost everywhere
    "thick_blob": lambda: W.thick_blob(16, 2),
    # dark absorbing medium lit by one star (Sec. 5.1 set-up)
    "point_source": lambda: W.point_source_box(16, 0.5, n_side=2),
}


@pytest.mark.parametrize("case", list(EDGE_CASES))
@pytest.mark.parametrize("kernel,bpp", [_k(1, 0), _k(1, 1), pytest.param(2, 0, marks=pytest.mark.skip(reason=WITHDRAWN))])
def test_trace_parity_edge_cases(lib, ctx, case, kernel, bpp):
    """Degenerate grids, every target against the oracle, both kernels (one radial point per
    pass for the one-wave kernel as well: every merge run crosses passes)."""
    from paper_2204_09072_amd.run import trace
    w = EDGE_CASES[case]()
    say("trace edge case", case, "kernel", kernel, "bins_per_pass", bpp)
    tree, J, F, U = trace(ctx, w, kernel=kernel, bins_per_pass=bpp)
    ctx.sync()
    Jo, Fo = oracle.Tree(w).trace(oracle.params(w.n_side, theta=w.theta))
    _check_trace(J.cpu().numpy(), F.cpu().numpy().T, Jo, Fo)


def test_trace_parity_merge_off_and_background(lib, ctx):
    from paper_2204_09072_amd.run import trace
    w = TREE_CASES["amr_small"]()
    w.j_bg = 0.37
    say("trace merge off + background")
    tree, J, F, U = trace(ctx, w, merge=False)
    ctx.sync()
    ot = oracle.Tree(w)
    Jo, Fo = ot.trace(oracle.params(w.n_side, theta=w.theta, merge=False, j_bg=0.37))
    _check_trace(J.cpu().numpy(), F.cpu().numpy().T, Jo, Fo)


def test_trace_bitwise_reproducible(lib, ctx):
    """Every target is traced by one wave whose additions into its bins run in program order,
    so for a given pass width the result is the same bit for bit from run to run and under
    any work split (targets per grab, waves per block).  A different pass width prunes other
    subtrees per pass and changes the order of the sums, within the J bar."""
    from paper_2204_09072_amd.run import trace, tree_of, upload
    w = W.c2_turb64()
    dev = upload(w)
    tree = tree_of(ctx, w, dev)
    runs = {}
    for tag, kw in (("auto", {}), ("again", {}), ("chunk8", dict(chunk=8)), ("four_waves", dict(waves_per_block=4)),
                    ("two_points", dict(bins_per_pass=2))):
        say("reproducibility run", tag)
        _, J, F, _ = trace(ctx, w, dev, tree=tree, **kw)
        ctx.sync()
        runs[tag] = (J.cpu().numpy().view(np.uint32).copy(), F.cpu().numpy().view(np.uint32).copy())
    for tag in ("again", "chunk8", "four_waves"):
        assert np.array_equal(runs[tag][0], runs["auto"][0]) and np.array_equal(runs[tag][1], runs["auto"][1]), tag
    Ja, Jb = runs["auto"][0].view(np.float32), runs["two_points"][0].view(np.float32)
    assert np.max(np.abs(Ja - Jb) / np.maximum(np.abs(Ja), 1e-30)) < 1e-5
    tree.free()


@pytest.mark.parametrize("name,n_sample,kernel", [("turb64", 1500, 0), ("core128", 160, 0),
                                                  ("core128", 80, 1), ("amr256", 400, 0)])
def test_trace_parity_full_size_sampled(lib, ctx, name, n_sample, kernel):
    from paper_2204_09072_amd.run import trace
    w = W.CONFIGS[name]()
    say("trace full size", name, w.n_cells, "kernel", kernel)
    tree, J, F, U = trace(ctx, w, kernel=kernel)
    ctx.sync()
    rng = np.random.default_rng(11)
    cells = np.sort(rng.choice(w.n_cells, n_sample, replace=False))
    ot = oracle.Tree(w)
    Jo, Fo = ot.trace(oracle.params(w.n_side, theta=w.theta), cells=cells)
    _check_trace(J.cpu().numpy()[cells], F.cpu().numpy().T[cells], Jo, Fo)


def test_trace_parity_nside8_sampled(lib, ctx):
    """768 rays (N_side = 8, opening angle 1/16): the wide-ray kernel (12 rays per lane,
    direction tables in global memory) on a 32^3 turbulent box with a star."""
    from paper_2204_09072_amd.run import trace
    w = W.c2_turb64(n=32, n_side=8)
    say("trace n_side 8", w.n_cells)
    tree, J, F, U = trace(ctx, w)
    ctx.sync()
    cells = np.sort(np.random.default_rng(12).choice(w.n_cells, 400, replace=False))
    ot = oracle.Tree(w)
    Jo, Fo = ot.trace(oracle.params(8, theta=w.theta), cells=cells)
    _check_trace(J.cpu().numpy()[cells], F.cpu().numpy().T[cells], Jo, Fo)


def _force_factor(ot, c):
    """(kappa / c) phi_RP(tau) of every cell: the oracle's force for a unit flux (Sec. 4.5)."""
    return ot.rad_force(np.ones((ot.n_cells, 3)), c)[0][:, 0]


def _check_force(a, ps, ao, po, fac, Jo, cells=None):
    """a_RP per cell and component within 1e-4 (kappa / c) phi_RP 4 pi J of that cell (the
    flux bar carried through the force); P_src per cell within 1e-5 relative."""
    sel = slice(None) if cells is None else cells
    tol = 1e-4 * fac[sel, None] * 4 * np.pi * np.abs(Jo)[:, None]
    d = np.abs(np.asarray(a, np.float64) - ao[sel])
    assert (d <= tol + 1e-37).all(), f"a_RP: worst {np.max(d / (tol + 1e-37)):.3e} x tolerance"
    po = po[sel]
    assert (np.abs(np.asarray(ps, np.float64) - po) <= 1e-5 * np.abs(po)).all()


def test_rad_force_parity(lib, ctx):
    """The whole path (trace, then force) against the oracle's whole path, per cell and
    component; and the force step alone on the library's own flux, per element."""
    from paper_2204_09072_amd.run import force, trace
    w = TREE_CASES["padded40"]()
    say("rad force")
    tree, J, F, U = trace(ctx, w)
    a, ps = force(ctx, tree, F)
    ctx.sync()
    ot = oracle.Tree(w)
    Jo, Fo = ot.trace(oracle.params(w.n_side, theta=w.theta))
    ao, po = ot.rad_force(Fo, w.units[1])
    fac = _force_factor(ot, w.units[1])
    a = a.cpu().numpy().T
    ps = ps.cpu().numpy()
    _check_force(a, ps, ao, po, fac, Jo)
    assert (po > 0).sum() == 2
    # the force step alone, given the same flux: a = kappa F / c phi_RP per element
    ag, pg = ot.rad_force(F.cpu().numpy().T.astype(np.float64), w.units[1])
    assert (np.abs(a - ag) <= 1e-5 * np.abs(ag) + 1e-37).all()
    assert (np.abs(ps - pg) <= 1e-5 * pg).all()


@pytest.mark.parametrize("name,n_sample", [("core128", 120), ("amr256", 200)])
def test_rad_force_parity_full_size_sampled(lib, ctx, name, n_sample):
    """a_RP of sampled cells of the full-size core and AMR grid, trace and force on the GPU
    against the oracle's trace and force, per cell and component."""
    from paper_2204_09072_amd.run import force, trace
    w = W.CONFIGS[name]()
    say("rad force full size", name, w.n_cells)
    tree, J, F, U = trace(ctx, w)
    a, ps = force(ctx, tree, F)
    ctx.sync()
    cells = np.sort(np.random.default_rng(13).choice(w.n_cells, n_sample, replace=False))
    ot = oracle.Tree(w)
    Jo, Fo = ot.trace(oracle.params(w.n_side, theta=w.theta), cells=cells)
    Ff = np.zeros((w.n_cells, 3))
    Ff[cells] = Fo
    ao, po = ot.rad_force(Ff, w.units[1])
    fac = _force_factor(ot, w.units[1])
    _check_force(a.cpu().numpy().T[cells], ps.cpu().numpy()[cells], ao, po, fac, Jo, cells)


def test_build_tree_validates_cells_on_request(lib, ctx):
    """With validation on, a NaN, infinite or negative density, opacity or dust temperature
    makes the build fail with TR_EINVAL; off (the default), the same arrays build."""
    import torch
    from paper_2204_09072_amd.run import upload
    w = W.small_uniform(16, 1.0, 1.0, 1.0)
    dev = upload(w)
    say("build validation")
    args = lambda d: (ctx, w.nb, 0, w.blocks, w.x0, 1.0, d["rho"], d["kappa"], d["t_dust"], w.stars, np.pi, 1.0)
    ctx.set_validation(True)
    try:
        lib.build_tree(*args(dev)).free()
        for field, val in (("rho", float("nan")), ("rho", -1.0), ("kappa", float("inf")), ("t_dust", -0.5)):
            d = dict(dev)
            d[field] = dev[field].clone()
            d[field][777] = val
            with pytest.raises(lib.TreerayError) as e:
                lib.build_tree(*args(d))
            assert e.value.code == lib.TR_EINVAL
            assert {"rho": "density", "kappa": "opacity", "t_dust": "dust temperature"}[field] in str(e.value)
    finally:
        ctx.set_validation(False)
    d = dict(dev)
    d["rho"] = dev["rho"].clone()
    d["rho"][777] = -1.0
    lib.build_tree(*args(d)).free()


def test_build_tree_rejects_bad_grids(lib, ctx):
    import torch
    w = W.small_uniform(16, 1.0, 1.0, 1.0)
    from paper_2204_09072_amd.run import upload
    dev = upload(w)
    bad = w.blocks.copy()
    bad[1] = bad[0]                      # two blocks on the same spot
    with pytest.raises(lib.TreerayError) as e:
        lib.build_tree(ctx, w.nb, 0, bad, w.x0, 1.0, dev["rho"], dev["kappa"], dev["t_dust"],
                       w.stars, np.pi, 1.0)
    assert e.value.code == lib.TR_EINVAL
    bad = w.blocks.copy()
    bad[0, 1] = 7                        # out of range
    with pytest.raises(lib.TreerayError):
        lib.build_tree(ctx, w.nb, 0, bad, w.x0, 1.0, dev["rho"], dev["kappa"], dev["t_dust"],
                       w.stars, np.pi, 1.0)
    tree = lib.build_tree(ctx, w.nb, 0, w.blocks, w.x0, 1.0, dev["rho"], dev["kappa"], dev["t_dust"],
                          w.stars, np.pi, 1.0)
    with pytest.raises(lib.TreerayError):
        lib.trace_rays(ctx, tree, lib.trace_params(3), torch.empty(4096, device="cuda"),
                       torch.empty((3, 4096), device="cuda"))
    # the withdrawn one-block kernel is refused with a message, before any launch
    with pytest.raises(lib.TreerayError) as e:
        lib.trace_rays(ctx, tree, lib.trace_params(1, kernel=2), torch.empty(4096, device="cuda"),
                       torch.empty((3, 4096), device="cuda"))
    assert e.value.code == lib.TR_EINVAL and "withdrawn" in str(e.value)


# ----------------------------------------------------------------------------------
# dust equilibrium and the guess network
# ----------------------------------------------------------------------------------
def test_dust_plain_parity(lib, ctx):
    import torch
    from paper_2204_09072_amd.run import dust
    s = W.dust_samples(200_000, seed=21).astype(np.float32).astype(np.float64)
    say("dust plain", s.shape)
    dev = [torch.from_numpy(s[:, k].astype(np.float32)).cuda() for k in range(3)]
    T, it = dust(ctx, *dev, W.SIGMA_SB, W.C_LIGHT)
    ctx.sync()
    To, _ = oracle.dust_eq(s[:, 0], s[:, 1], s[:, 2], W.SIGMA_SB, W.C_LIGHT, 3.8e-33)
    rel = np.abs(T.cpu().numpy() - To) / To
    assert rel.max() < 1e-5, rel.max()
    it = it.cpu().numpy()
    say("newton iterations: mean %.2f max %d" % (it.mean(), it.max()))
    assert it.max() < 50


def _bf16(a):
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def test_mlp_grad_parity(lib, ctx):
    import torch
    H = lib.MLP_HIDDEN
    prm = lib.init_mlp_params(3)
    prm[3 * H:4 * H] = np.random.default_rng(1).normal(scale=0.2, size=H)
    prm = _bf16(prm)
    rng = np.random.default_rng(4)
    n = 4099                                  # several 32-sample tiles and a ragged tail
    x = _bf16(rng.normal(size=(n, 3)).astype(np.float32))
    y = rng.normal(size=n).astype(np.float32)
    say("mlp grad", n)
    m = lib.Mlp(ctx, prm)
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    g = torch.zeros(lib.MLP_NPARAM, device="cuda")
    loss = torch.zeros(1, device="cuda")
    m.grad(xd, yd, g, loss)
    out = torch.zeros(n, device="cuda")
    m.forward(xd, out)
    ctx.sync()
    lo, oo, go = oracle.mlp(H, prm.astype(np.float64), x.astype(np.float64), y.astype(np.float64),
                            round_bf16=True)
    d = np.abs(out.cpu().numpy() - oo) / np.abs(oo).max()
    say("forward |dy|/max|y|: median %.2e p99 %.2e max %.2e" % (np.median(d), np.quantile(d, 0.99), d.max()))
    # the FP32 and FP64 activations can round to different bfloat16 neighbours (2^-8
    # relative) near a rounding boundary; away from those the outputs agree to 1e-5
    assert np.median(d) < 1e-5 and np.quantile(d, 0.99) < 1e-3 and d.max() < 1e-2
    assert loss.item() == pytest.approx(lo, rel=1e-3)
    # many 32-sample steps per wave (the inference loop keeps three steps' inputs in flight):
    # every sample against the FP64 network
    nb = 300_001
    xb = _bf16(np.random.default_rng(5).normal(size=(nb, 3)).astype(np.float32))
    ob = torch.zeros(nb, device="cuda")
    m.forward(torch.from_numpy(xb).cuda(), ob)
    ctx.sync()
    _, oob, _ = oracle.mlp(H, prm.astype(np.float64), xb.astype(np.float64), round_bf16=True, grad=False)
    db = np.abs(ob.cpu().numpy() - oob) / np.abs(oob).max()
    say("forward %d: median %.2e max %.2e" % (nb, np.median(db), db.max()))
    assert np.median(db) < 1e-5 and db.max() < 1e-2
    g = g.cpu().numpy()
    offs = [0, 3 * H, 4 * H, 4 * H + H * H, 5 * H + H * H, 6 * H + H * H, 6 * H + H * H + 1]
    for a, b in zip(offs[:-1], offs[1:]):
        err = np.linalg.norm(g[a:b] - go[a:b]) / max(np.linalg.norm(go[a:b]), 1e-30)
        say("grad block", a, b, "rel frobenius err %.2e" % err)
        assert err < 1e-2, (a, b, err)


def test_mlp_adam_steps_match_closed_form(lib, ctx):
    """Two training steps against Adam's update written out in numpy (beta1 0.9, beta2 0.999,
    eps 1e-8, bias-corrected moments), each fed the gradient the library computes for the
    same parameters and batch."""
    import torch
    prm = lib.init_mlp_params(5)
    rng = np.random.default_rng(6)
    m = lib.Mlp(ctx, prm)
    lr = 1e-2
    p = prm.astype(np.float64)
    mom = np.zeros_like(p)
    vel = np.zeros_like(p)
    say("adam steps")
    for step in (1, 2):
        x = torch.from_numpy(rng.normal(size=(3000, 3)).astype(np.float32)).cuda()
        y = torch.from_numpy(rng.normal(size=3000).astype(np.float32)).cuda()
        g = torch.zeros(lib.MLP_NPARAM, device="cuda")
        loss = torch.zeros(1, device="cuda")
        m.grad(x, y, g, loss)
        ctx.sync()
        g = g.cpu().numpy().astype(np.float64)
        m.train_step(x, y, lr)
        ctx.sync()
        mom = 0.9 * mom + 0.1 * g
        vel = 0.999 * vel + 0.001 * g * g
        upd = lr * (mom / (1 - 0.9 ** step)) / (np.sqrt(vel / (1 - 0.999 ** step)) + 1e-8)
        p = p - upd
        got = m.params().astype(np.float64)
        err = np.abs(got - p)
        # the step size is lr * O(1); the gradient's own rounding (atomic order) moves it by
        # far less except where |g| ~ eps
        assert (err <= 1e-3 * lr + 1e-6 * np.abs(p)).all(), (step, err.max())
        assert np.abs(upd).max() > 0.5 * lr
    m.free()


def test_mlp_checkpoint_resume(lib, ctx, tmp_path):
    """Training state through a checkpoint file: parameters, Adam moments and step count
    come back bit for bit, and a resumed network takes the same next Adam step (with the
    restored step's bias correction) as the one that kept training."""
    import torch
    from paper_2204_09072_amd.guess import load_checkpoint, save_checkpoint
    rng = np.random.default_rng(8)
    norm = np.array([1, 2, 3, 0.5, 0.25, 2, -1, 3], np.float32)
    a = lib.Mlp(ctx, lib.init_mlp_params(9), norm)
    lr = 1e-2
    batches = [(torch.from_numpy(rng.normal(size=(2000, 3)).astype(np.float32)).cuda(),
                torch.from_numpy(rng.normal(size=2000).astype(np.float32)).cuda()) for _ in range(4)]
    say("checkpoint: three steps, save, load")
    for x, y in batches[:3]:
        a.train_step(x, y, lr)
    ctx.sync()
    path = str(tmp_path / "guess.ckpt")
    save_checkpoint(a, path)
    b = load_checkpoint(ctx, path)
    sa, sb = a.get_state(), b.get_state()
    assert sa["steps"] == sb["steps"] == 3
    for k in ("params", "adam_m", "adam_v", "norm"):
        assert np.array_equal(sa[k], sb[k]), k
    assert np.array_equal(sb["norm"], norm)
    # forward passes agree exactly (same parameters, same bfloat16 rounding)
    ya, yb = torch.zeros(2000, device="cuda"), torch.zeros(2000, device="cuda")
    a.forward(batches[3][0], ya)
    b.forward(batches[3][0], yb)
    ctx.sync()
    assert torch.equal(ya, yb)
    # the fourth step on both; a restart at step 0 would move the parameters ~10x further
    x, y = batches[3]
    a.train_step(x, y, lr)
    b.train_step(x, y, lr)
    ctx.sync()
    pa, pb = a.params().astype(np.float64), b.params().astype(np.float64)
    assert (np.abs(pa - pb) <= 1e-3 * lr + 1e-6 * np.abs(pa)).all(), np.abs(pa - pb).max()
    c = lib.Mlp(ctx, sa["params"], norm)  # same parameters, fresh Adam state
    c.train_step(x, y, lr)
    ctx.sync()
    assert np.abs(c.params().astype(np.float64) - pa).max() > 10 * (1e-3 * lr)
    with pytest.raises(lib.TreerayError):
        b.set_state(sa["params"], None, None, -1)
    for m in (a, b, c):
        m.free()


def test_walk_stack_overflow_is_reported(lib, ctx):
    """Failure detection: a walk stack too small for the tree (the stack_limit test hook)
    makes the walk drop subtrees, latch the overflow and tr_sync report TR_EOVERFLOW, for the
    trace and for the walk counters; the flag is then clear and a normal trace matches the
    oracle again.  The kernel itself never writes past its stack (pushes beyond it are
    dropped), so the condition is forced without any out-of-bounds access."""
    import torch
    from paper_2204_09072_amd.run import trace, tree_of, upload
    w = TREE_CASES["turb32"]()
    dev = upload(w)
    tree = tree_of(ctx, w, dev)
    say("stack overflow forced: trace")
    trace(ctx, w, dev, tree=tree, stack_limit=9)
    with pytest.raises(lib.TreerayError) as e:
        ctx.sync()
    assert e.value.code == lib.TR_EOVERFLOW
    say("stack overflow forced: walk counts")
    cnt = torch.zeros((tree.n_cells, 3), dtype=torch.int32, device="cuda")
    lib.walk_counts(ctx, tree, lib.trace_params(w.n_side, theta=w.theta, stack_limit=9), cnt)
    with pytest.raises(lib.TreerayError) as e:
        ctx.sync()
    assert e.value.code == lib.TR_EOVERFLOW
    with pytest.raises(lib.TreerayError):
        trace(ctx, w, dev, tree=tree, stack_limit=-1)
    say("normal trace after the overflow")
    _, J, F, _ = trace(ctx, w, dev, tree=tree)
    ctx.sync()
    Jo, Fo = oracle.Tree(w).trace(oracle.params(w.n_side, theta=w.theta))
    _check_trace(J.cpu().numpy(), F.cpu().numpy().T, Jo, Fo)
    tree.free()
