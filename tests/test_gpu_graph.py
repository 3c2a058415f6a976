"""Tree refill and the whole hot path in one HIP graph, through the C ABI.

tr_tree_refill must leave exactly the node arrays that tr_build_tree makes from the same
inputs (same blocks), and a graph that captures refill -> trace -> force -> dust must give,
on every replay, exactly the results of the same calls made directly."""
import copy

import numpy as np
import pytest

import workloads as W

from test_gpu_parity import TREE_CASES, say

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


def _other_fields(w, seed):
    """The same blocks with new densities (some cells crossing rho kappa dx = 1 either way),
    dust temperatures and moved stars."""
    rng = np.random.default_rng(seed)
    w2 = copy.copy(w)
    w2.rho = (w.rho * 10.0 ** rng.uniform(-1.0, 1.0, w.rho.shape)).astype(w.rho.dtype)
    w2.t_dust = (w.t_dust * rng.uniform(0.8, 1.25, w.t_dust.shape)).astype(w.t_dust.dtype)
    if w.stars.shape[0]:
        st = np.array(w.stars, np.float64, copy=True)
        st[:, :3] = np.clip(st[:, :3] + rng.uniform(-0.2, 0.2, st[:, :3].shape) * w.box_len,
                            w.x0, np.asarray(w.x0) + 0.999 * w.box_len)
        st[:, 3] *= rng.uniform(0.5, 2.0, st.shape[0])
        w2.stars = st
    return w2


def _dev_stars(w):
    import torch
    if not w.stars.shape[0]:
        return None
    return torch.from_numpy(np.ascontiguousarray(w.stars, np.float64)).cuda()


@pytest.mark.parametrize("case", ["turb32", "amr_small", "padded40", "core32"])
def test_tree_refill_equals_build(lib, ctx, case):
    from paper_2204_09072_amd.run import tree_of, trace, upload
    w1 = TREE_CASES[case]()
    w2 = _other_fields(w1, seed=17)
    say("tree refill", case, w1.n_cells, "cells", w1.stars.shape[0], "stars")
    d1, d2 = upload(w1), upload(w2)
    a = tree_of(ctx, w1, d1)
    b = tree_of(ctx, w2, d2)
    thick_before = (lib.tree_export(ctx, a)["meta"] >> 13) & 1
    a.refill(d2["rho"], d2["kappa"], d2["t_dust"], _dev_stars(w2))
    ctx.sync()
    ga, gb = lib.tree_export(ctx, a), lib.tree_export(ctx, b)
    for k in ("geo", "meta", "leaf_cell", "pcol"):
        assert np.array_equal(ga[k], gb[k]), k
    for k in ("q", "vthick"):
        assert np.array_equal(ga[k].view(np.uint32), gb[k].view(np.uint32)), k
    # the case really changed: thick flags moved and the content differs from the first fields
    assert ((gb["meta"] >> 13) & 1 != thick_before).any()
    _, Ja, Fa, _ = trace(ctx, w2, d2, tree=a)
    _, Jb, Fb, _ = trace(ctx, w2, d2, tree=b)
    ctx.sync()
    assert np.array_equal(Ja.cpu().numpy().view(np.uint32), Jb.cpu().numpy().view(np.uint32))
    a.free()
    b.free()


def test_whole_step_in_one_graph(lib, ctx):
    """Refill, trace, radiation force and dust equilibrium captured once in a HIP graph on the
    context's stream and replayed three times, with other work on the stream between the
    replays; every replay equals the direct calls bit for bit."""
    import torch
    from paper_2204_09072_amd.run import params_of, tree_of, upload
    w1 = TREE_CASES["turb32"]()
    w2 = _other_fields(w1, seed=23)
    d1, d2 = upload(w1), upload(w2)
    t_gas = torch.from_numpy(np.ascontiguousarray(w2.t_dust * 1.3, np.float32)).cuda()
    stars2 = _dev_stars(w2)
    n = w1.n_cells
    s = torch.cuda.Stream()
    old = torch.cuda.current_stream().cuda_stream
    ctx.set_stream(s.cuda_stream)
    try:
        with torch.cuda.stream(s):
            tree = tree_of(ctx, w1, d1)
            p = params_of(w1)
            dp = lib.dust_params(w1.units[0], w1.units[1])
            J = torch.empty(n, device="cuda")
            F = torch.empty((3, n), device="cuda")
            U = torch.empty(n, device="cuda")
            a = torch.empty((3, n), device="cuda")
            ps = torch.empty(n, device="cuda")
            T = torch.empty(n, device="cuda")

            def step():
                tree.refill(d2["rho"], d2["kappa"], d2["t_dust"], stars2)
                lib.trace_rays(ctx, tree, p, J, F, U)
                lib.rad_force(ctx, tree, F, a, ps)
                lib.dust_equilibrium(ctx, d2["rho"], U, t_gas, dp, T)

            say("whole step: direct calls (also the warm-up: tables and workspaces)")
            step()
            ctx.sync()
            ref = [x.clone() for x in (J, F, a, ps, T)]
            for x in (J, F, a, ps, T):
                x.fill_(-1.0)
            torch.cuda.synchronize()
            say("whole step: capture")
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                step()
            other = tree_of(ctx, w1, d1)  # a different tree, traced directly between replays
            for rep in range(3):
                for x in (J, F, a, ps, T):
                    x.fill_(-1.0)
                torch.cuda.synchronize()
                say("whole step: replay", rep)
                g.replay()
                torch.cuda.synchronize()
                for got, want in zip((J, F, a, ps, T), ref):
                    assert torch.equal(got, want), rep
                Jo = torch.empty(n, device="cuda")
                Fo = torch.empty((3, n), device="cuda")
                lib.trace_rays(ctx, other, params_of(w1), Jo, Fo, None)
                ctx.sync()
            other.free()
            tree.free()
            del g
    finally:
        ctx.set_stream(old)


def test_batch_replay_after_refill(lib, ctx):
    """A captured batch reads its trees' node arrays at every replay: after a refill of one
    instance the next replay gives, bit for bit, what the same batch over a tree built
    directly from the new fields gives."""
    import torch
    from paper_2204_09072_amd.run import params_of, tree_of, upload
    wa, wb = TREE_CASES["turb32"](), TREE_CASES["amr_small"]()
    wa2 = _other_fields(wa, seed=31)
    da, db, da2 = upload(wa), upload(wb), upload(wa2)
    ta, tb = tree_of(ctx, wa, da), tree_of(ctx, wb, db)
    J = [torch.empty(w.n_cells, device="cuda") for w in (wa, wb)]
    F = [torch.empty((3, w.n_cells), device="cuda") for w in (wa, wb)]
    b = lib.Batch(ctx, [ta, tb], [params_of(wa), params_of(wb)], J, F, None)
    b.launch()
    ctx.sync()
    say("batch after refill: refill and replay")
    ta.refill(da2["rho"], da2["kappa"], da2["t_dust"], _dev_stars(wa2))
    b.launch()
    ctx.sync()
    got = [j.cpu().numpy().copy() for j in J]
    say("batch after refill: the same batch over a fresh build")
    ta2 = tree_of(ctx, wa2, da2)
    J2 = [torch.empty(w.n_cells, device="cuda") for w in (wa, wb)]
    F2 = [torch.empty((3, w.n_cells), device="cuda") for w in (wa, wb)]
    b2 = lib.Batch(ctx, [ta2, tb], [params_of(wa2), params_of(wb)], J2, F2, None)
    b2.launch()
    ctx.sync()
    for g_, w_ in zip(got, J2):
        assert np.array_equal(g_.view(np.uint32), w_.cpu().numpy().view(np.uint32))
    b.free()
    b2.free()
    for t in (ta, tb, ta2):
        t.free()
