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


# Checkpoints of the guess network: a flat little-endian float32 file holding the
# parameters, Adam's first moments and Adam's second moments (n_params each, in that
# order), and beside it a JSON header (<path>.json) with the layout, the Adam step count,
# the normalisation and the file's SHA-256.
CHECKPOINT_FORMAT = "treeray-guess-network"
_ARRAYS = ("params", "adam_m", "adam_v")


def write_checkpoint(path, state: dict):
    """Write a training state (as returned by Mlp.get_state) to `path` and `path`.json."""
    import hashlib
    import json
    import os
    from . import MLP_NPARAM
    arrs = [np.ascontiguousarray(state[k], "<f4") for k in _ARRAYS]
    for a in arrs:
        if a.shape != (MLP_NPARAM,):
            raise ValueError(f"checkpoint arrays must hold {MLP_NPARAM} floats")
    blob = b"".join(a.tobytes() for a in arrs)
    header = {"format": CHECKPOINT_FORMAT, "version": 1, "n_params": MLP_NPARAM,
              "layout": "W1[64][3] b1[64] W2[64][64] b2[64] W3[64] b3",
              "arrays": list(_ARRAYS), "dtype": "float32 little-endian",
              "adam": {"beta1": 0.9, "beta2": 0.999, "eps": 1e-8},
              "adam_steps": int(state["steps"]),
              "norm": [float(v) for v in np.asarray(state["norm"], np.float32)],
              "sha256": hashlib.sha256(blob).hexdigest()}
    for name, data, mode in ((path, blob, "wb"), (str(path) + ".json", json.dumps(header, indent=1), "w")):
        tmp = str(name) + ".tmp"
        with open(tmp, mode) as f:
            f.write(data)
        os.replace(tmp, name)


def read_checkpoint(path) -> dict:
    """Read a checkpoint written by write_checkpoint; raises ValueError on a wrong format,
    size or checksum."""
    import hashlib
    import json
    from . import MLP_NPARAM
    with open(str(path) + ".json") as f:
        header = json.load(f)
    if header.get("format") != CHECKPOINT_FORMAT or header.get("version") != 1:
        raise ValueError(f"{path}: not a version-1 {CHECKPOINT_FORMAT} checkpoint")
    if header.get("n_params") != MLP_NPARAM:
        raise ValueError(f"{path}: {header.get('n_params')} parameters, this network has {MLP_NPARAM}")
    with open(path, "rb") as f:
        blob = f.read()
    if len(blob) != 3 * 4 * MLP_NPARAM or hashlib.sha256(blob).hexdigest() != header.get("sha256"):
        raise ValueError(f"{path}: size or checksum does not match its header")
    flat = np.frombuffer(blob, "<f4").astype(np.float32)
    state = {k: flat[i * MLP_NPARAM:(i + 1) * MLP_NPARAM].copy() for i, k in enumerate(_ARRAYS)}
    state["steps"] = int(header["adam_steps"])
    state["norm"] = np.asarray(header["norm"], np.float32)
    return state


def save_checkpoint(mlp: Mlp, path):
    write_checkpoint(path, mlp.get_state())


def load_checkpoint(ctx: Context, path) -> Mlp:
    """A network in the state a checkpoint holds; training continues with Adam step
    adam_steps + 1."""
    st = read_checkpoint(path)
    mlp = Mlp(ctx, st["params"], st["norm"])
    mlp.set_state(st["params"], st["adam_m"], st["adam_v"], st["steps"])
    return mlp
