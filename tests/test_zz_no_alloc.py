"""The allocation-free dust solve (tr_dust_equilibrium_noalloc) against the allocating entry
point, through the C ABI: the same starting points and results on two calls in a row (the
largest input it takes, then a smaller ragged one, which must not see the first call's
scratch), and a clear error beyond its size limit."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_noalloc_dust_matches_allocating_entry_point():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_09072_amd as T
    from paper_2204_09072_amd.guess import features
    ctx = T.Context(0)
    s0 = W.dust_samples(20_000, seed=41)
    f = features(s0[:, 0], s0[:, 1], s0[:, 2])
    norm = np.array([*f.mean(0), *(1.0 / f.std(0)), 1.3, 2.0], np.float32)
    mlp = T.Mlp(ctx, T.init_mlp_params(9), norm)
    dp = T.dust_params(W.SIGMA_SB, W.C_LIGHT)
    for n, seed in ((T.NOALLOC_DUST_STATES, 42), (70_001, 43)):
        print("no-alloc dust solve", n, flush=True)
        s = W.dust_samples(n, seed=seed).astype(np.float32)
        rho, u, tg = (torch.from_numpy(np.ascontiguousarray(s[:, k])).cuda() for k in range(3))
        ta = torch.empty(n, device="cuda")
        tb = torch.full((n,), -1.0, device="cuda")
        ia = torch.empty(n, dtype=torch.uint8, device="cuda")
        ib = torch.empty(n, dtype=torch.uint8, device="cuda")
        T.dust_equilibrium(ctx, rho, u, tg, dp, ta, ia, mlp)
        T.dust_equilibrium_noalloc(ctx, rho, u, tg, dp, tb, ib, mlp)
        ctx.sync()
        a, b = ta.cpu().numpy().astype(np.float64), tb.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(b - a) <= 1e-5 * a), np.max(np.abs(b - a) / a)
        assert np.array_equal(ia.cpu().numpy(), ib.cpu().numpy())
        # without a network the variant takes the plain start, no scratch involved
        T.dust_equilibrium(ctx, rho, u, tg, dp, ta, ia, None)
        T.dust_equilibrium_noalloc(ctx, rho, u, tg, dp, tb, ib, None)
        ctx.sync()
        assert torch.equal(ta, tb) and torch.equal(ia, ib)
    # beyond the limit: TR_EINVAL before any work (the arrays are never read)
    one = torch.zeros(1, device="cuda")
    rc = T._lib.tr_dust_equilibrium_noalloc(ctx.h, T.NOALLOC_DUST_STATES + 1, T._ptr(one), T._ptr(one),
                                            T._ptr(one), ctypes.byref(dp), mlp.h, T._ptr(one), None)
    assert rc == T.TR_EINVAL
    assert b"at most" in T._lib.tr_last_error(ctx.h)
    mlp.free()
    ctx.close()
