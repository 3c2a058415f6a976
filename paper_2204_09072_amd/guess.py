"""Training of the dust-equilibrium guess network on the GPU (tr_mlp_train_step).

Features are (log10 rho, log10 u_rad, log10 T_gas), standardised; the target is
log10 T_dust, standardised.  The normalisation travels with the network
(tr_mlp_create's ``norm``) so the dust solve can feed raw fields.
"""
from __future__ import annotations

import numpy as np

from . import Context, Mlp, init_mlp_params


def features(rho, u_rad, t_gas):
    return np.stack([np.log10(np.maximum(rho, 1e-37)), np.log10(np.maximum(u_rad, 1e-37)),
                     np.log10(np.maximum(t_gas, 1e-37))], axis=1)


def train_guess(ctx: Context, rho, u_rad, t_gas, t_dust, steps=3000, batch=8192, lr=3e-3,
                seed=0, log_every=0):
    """Fit the network to (rho, u_rad, T_gas) -> T_dust samples (host arrays).

    Mini-batches are consecutive slices of the samples in an order drawn on the host once
    per pass over the data (a fresh permutation, uploaded whole); every training step runs
    in the library (tr_mlp_train_step).  Returns (mlp, losses).  The learning rate decays
    by 10x over the run."""
    import torch
    f = features(np.asarray(rho, np.float64), np.asarray(u_rad, np.float64),
                 np.asarray(t_gas, np.float64))
    y = np.log10(np.asarray(t_dust, np.float64))
    shift = f.mean(axis=0)
    scale = 1.0 / np.maximum(f.std(axis=0), 1e-6)
    oshift, oscale = y.mean(), 1.0 / max(y.std(), 1e-6)
    norm = np.array([*shift, *scale, oshift, oscale], np.float32)
    xs = ((f - shift) * scale).astype(np.float32)
    ys = ((y - oshift) * oscale).astype(np.float32)
    mlp = Mlp(ctx, init_mlp_params(seed), norm)
    rng = np.random.default_rng(seed)
    loss = torch.zeros(1, device="cuda")
    losses = []
    n = ys.shape[0]
    batch = min(batch, n)
    per_pass = n // batch
    x = t = None
    for s in range(steps):
        k = s % per_pass
        if k == 0:
            order = rng.permutation(n)
            x = torch.from_numpy(np.ascontiguousarray(xs[order])).cuda()
            t = torch.from_numpy(np.ascontiguousarray(ys[order])).cuda()
        a = lr * (0.1 ** (s / max(steps - 1, 1)))
        mlp.train_step(x[k * batch:(k + 1) * batch], t[k * batch:(k + 1) * batch], a, loss)
        if log_every and (s % log_every == 0 or s == steps - 1):
            ctx.sync()
            losses.append((s, float(loss.item())))
    ctx.sync()
    return mlp, losses
