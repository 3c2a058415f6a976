"""Dust equilibrium on the GPU: every starting rule and iteration form against the FP64
bracketed root of the oracle (rel 1e-5), and what the trained guess network gains over
the solve without it."""
import numpy as np
import pytest

import oracle
import workloads as W

from test_gpu_parity import say

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


@pytest.mark.parametrize("start,linear", [(0, False), (1, False), (0, True), (1, True), (2, False)])
def test_dust_every_start_parity(lib, ctx, start, linear):
    import torch
    from paper_2204_09072_amd.run import dust
    s = W.dust_samples(100_000, seed=22).astype(np.float32).astype(np.float64)
    say("dust start", start, "linear", linear)
    dev = [torch.from_numpy(s[:, k].astype(np.float32)).cuda() for k in range(3)]
    T, it = dust(ctx, *dev, W.SIGMA_SB, W.C_LIGHT, start=start, linear=linear, max_iter=250)
    ctx.sync()
    To, _ = oracle.dust_eq(s[:, 0], s[:, 1], s[:, 2], W.SIGMA_SB, W.C_LIGHT, 3.8e-33)
    rel = np.abs(T.cpu().numpy() - To) / To
    it = it.cpu().numpy()
    say("  max rel %.2e, iterations mean %.2f max %d" % (rel.max(), it.mean(), it.max()))
    assert rel.max() < 1e-5
    assert it.max() < 250


def _cloud(ctx, seed):
    """u_rad of a 32^3 collapsing core from the GPU trace, with rho and T_gas."""
    from paper_2204_09072_amd.run import trace, upload
    w = W.c3_core128(n=32, seed=seed, n_side=2)
    dev = upload(w)
    tree, J, F, U = trace(ctx, w, dev)
    ctx.sync()
    tree.free()
    return w, dev["rho"], U, dev["t_gas"]


def test_learned_guess_gain(lib, ctx):
    """Train the guess network on log-uniform (rho, u_rad, T_gas) states (labels from the
    library's own solve), use it on a held-out draw: same T_dust as the FP64 oracle, fewer
    Newton steps than plain Newton on the residual started at the bracket end nearer the
    root.  States inside the bracket are where a guess can help: in the collapsing core
    most cells have T_dust at a bracket end (T_gas or T_J) and every start finds it in
    about one step (reported, not asserted)."""
    import torch
    from paper_2204_09072_amd.guess import train_guess
    from paper_2204_09072_amd.run import dust
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    s1 = W.dust_samples(200_000, seed=31).astype(np.float32)
    r1, u1, t1 = d(s1[:, 0]), d(s1[:, 1]), d(s1[:, 2])
    lab, _ = dust(ctx, r1, u1, t1, W.SIGMA_SB, W.C_LIGHT)
    ctx.sync()
    say("training on", r1.numel(), "states")
    mlp, losses = train_guess(ctx, s1[:, 0], s1[:, 1], s1[:, 2], lab.cpu().numpy(), steps=1500, batch=8192,
                              log_every=500)
    say("losses", losses)
    assert losses[-1][1] < 0.01 * losses[0][1]
    s2 = W.dust_samples(100_000, seed=32).astype(np.float32)
    r2, u2, t2 = d(s2[:, 0]), d(s2[:, 1]), d(s2[:, 2])
    To, _ = oracle.dust_eq(s2[:, 0].astype(np.float64), s2[:, 1].astype(np.float64), s2[:, 2].astype(np.float64),
                           W.SIGMA_SB, W.C_LIGHT, 3.8e-33)
    res = {}
    for name, kw in (("learned", dict(mlp=mlp)), ("learned_lin", dict(mlp=mlp, linear=True)),
                     ("end_linear", dict(start=1, linear=True, max_iter=250)),
                     ("end_log", dict(start=1)), ("secant_log", dict(start=0))):
        T, it = dust(ctx, r2, u2, t2, W.SIGMA_SB, W.C_LIGHT, **kw)
        ctx.sync()
        rel = np.abs(T.cpu().numpy() - To) / To
        res[name] = float(it.float().mean().item())
        res[name + "_max"] = int(it.max().item())
        say("  %-11s max rel %.2e  mean iterations %.3f  max %d" % (name, rel.max(), res[name], res[name + "_max"]))
        assert rel.max() < 1e-5, name
    # the network's guess saves steps over the plain Newton start it replaces
    assert res["learned"] < res["end_linear"] and res["learned_lin"] < res["end_linear"]
    # and has no tail: a step that lands on a bracket end not yet evaluated tries that end
    # (roots at T_J or T_gas to FP32 precision) instead of being replaced by bisection,
    # which took such cells 10-16 steps
    assert res["learned_max"] <= 8 and res["learned_lin_max"] <= 8
    # the collapsing core, for the record
    w, rc, uc, tc = _cloud(ctx, 2)
    for name, kw in (("learned", dict(mlp=mlp)), ("end_linear", dict(start=1, linear=True, max_iter=250))):
        T, it = dust(ctx, rc, uc, tc, W.SIGMA_SB, W.C_LIGHT, **kw)
        ctx.sync()
        say("  core %-10s mean iterations %.3f" % (name, float(it.float().mean().item())))
    mlp.free()


@pytest.mark.parametrize("n", [0, 1, 33])
def test_dust_and_network_tiny_inputs(lib, ctx, n):
    """Empty and ragged inputs: nothing launched for n = 0; for a single state and for one
    32-state step plus one, the solve against the oracle and the network's forward pass
    against the oracle's bfloat16-rounded evaluation."""
    import torch
    from paper_2204_09072_amd.run import dust
    s = W.dust_samples(max(n, 1), seed=40)[:n].astype(np.float32)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    say("tiny inputs", n)
    T, it = dust(ctx, d(s[:, 0]), d(s[:, 1]), d(s[:, 2]), W.SIGMA_SB, W.C_LIGHT)
    H = lib.MLP_HIDDEN
    prm = lib.init_mlp_params(5)
    u = prm.view(np.uint32).astype(np.uint64)
    prm = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32).view(np.float32)
    m = lib.Mlp(ctx, prm)
    x = np.random.default_rng(41).normal(size=(n, 3)).astype(np.float32)
    xu = x.view(np.uint32).astype(np.uint64)
    x = ((xu + 0x7FFF + ((xu >> 16) & 1)) & 0xFFFF0000).astype(np.uint32).view(np.float32).reshape(n, 3)
    y = torch.zeros(n, device="cuda")
    m.forward(d(x), y)
    ctx.sync()
    if n:
        To, _ = oracle.dust_eq(s[:, 0].astype(np.float64), s[:, 1].astype(np.float64), s[:, 2].astype(np.float64),
                               W.SIGMA_SB, W.C_LIGHT, 3.8e-33)
        assert np.all(np.abs(T.cpu().numpy() - To) / To < 1e-5)
        _, yo, _ = oracle.mlp(H, prm.astype(np.float64), x.astype(np.float64), np.zeros(n), round_bf16=True)
        assert np.allclose(y.cpu().numpy(), yo, rtol=1e-2, atol=1e-2 * np.abs(yo).max())
    m.free()


def test_learned_one_kernel_equals_staged(lib, ctx):
    """The learned start in one kernel (guesses kept in registers) and staged (inference into a
    buffer, then the solve) take the same starting points: identical T_dust and step counts
    on every state, including a ragged last group of 64."""
    import torch
    from paper_2204_09072_amd.guess import features
    s = W.dust_samples(100_003, seed=44).astype(np.float32)
    f = features(*(s[:, k].astype(np.float64) for k in range(3)))
    norm = np.array([*f.mean(0), *(1.0 / f.std(0)), 1.3, 2.0], np.float32)
    mlp = lib.Mlp(ctx, lib.init_mlp_params(11), norm)
    rho, u, tg = (torch.from_numpy(np.ascontiguousarray(s[:, k])).cuda() for k in range(3))
    out = {}
    for staged in (False, True):
        t = torch.empty(len(s), device="cuda")
        it = torch.empty(len(s), dtype=torch.uint8, device="cuda")
        lib.dust_equilibrium(ctx, rho, u, tg, lib.dust_params(W.SIGMA_SB, W.C_LIGHT, staged=staged), t, it, mlp)
        ctx.sync()
        out[staged] = (t.cpu().numpy(), it.cpu().numpy())
    assert np.array_equal(out[False][0], out[True][0])
    assert np.array_equal(out[False][1], out[True][1])
    mlp.free()


def test_poisoned_network_falls_back_to_the_bracket(lib, ctx):
    """Failure recovery: a network whose output is NaN (NaN weights) or absurd (a huge
    output bias) still gives every state its equilibrium temperature within 1e-5, since a
    guess outside the bracket (or NaN) is clamped to it before Newton starts."""
    import torch
    from paper_2204_09072_amd.run import dust
    s = W.dust_samples(20_000, seed=44).astype(np.float32)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    To, _ = oracle.dust_eq(*[s[:, k].astype(np.float64) for k in range(3)], W.SIGMA_SB, W.C_LIGHT, 3.8e-33)
    for tag, prm in (("nan", np.full(lib.MLP_NPARAM, np.nan, np.float32)),
                     ("huge", np.concatenate([np.zeros(lib.MLP_NPARAM - 1), [1e4]]).astype(np.float32))):
        say("poisoned network", tag)
        m = lib.Mlp(ctx, prm)
        for staged in (False, True):
            T, it = dust(ctx, d(s[:, 0]), d(s[:, 1]), d(s[:, 2]), W.SIGMA_SB, W.C_LIGHT, mlp=m, staged=staged)
            ctx.sync()
            Tg = T.cpu().numpy()
            assert np.isfinite(Tg).all(), (tag, staged)
            assert np.max(np.abs(Tg - To) / To) < 1e-5, (tag, staged)
        m.free()
