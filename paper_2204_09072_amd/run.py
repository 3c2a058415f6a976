"""Convenience wrappers: upload a workload's cell arrays and run the hot path through the C ABI.

A workload is any object with the attributes of ``workloads.synth.Workload`` (nb,
max_level, blocks, x0, box_len, rho, kappa, t_dust, t_gas, stars, units, n_side, theta,
j_bg).  Only argument marshalling happens here.
"""
from __future__ import annotations

import numpy as np

from . import (Context, build_tree, dust_equilibrium, dust_params, rad_force, trace_params,
               trace_rays)


def upload(w, device="cuda"):
    import torch
    f = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
    return dict(rho=f(w.rho), kappa=f(w.kappa), t_dust=f(w.t_dust), t_gas=f(w.t_gas))


def tree_of(ctx: Context, w, dev):
    return build_tree(ctx, w.nb, w.max_level, w.blocks, w.x0, w.box_len, dev["rho"], dev["kappa"],
                      dev["t_dust"], w.stars, w.units[0], w.units[1])


def params_of(w, **kw):
    return trace_params(w.n_side, theta=w.theta, j_bg=getattr(w, "j_bg", 0.0), **kw)


def trace(ctx: Context, w, dev=None, tree=None, **kw):
    """Build the tree and trace every cell; returns (tree, J [n], F [3, n], u_rad [n])."""
    import torch
    dev = upload(w) if dev is None else dev
    tree = tree_of(ctx, w, dev) if tree is None else tree
    n = tree.n_cells
    J = torch.empty(n, dtype=torch.float32, device="cuda")
    F = torch.empty((3, n), dtype=torch.float32, device="cuda")
    U = torch.empty(n, dtype=torch.float32, device="cuda")
    trace_rays(ctx, tree, params_of(w, **kw), J, F, U)
    return tree, J, F, U


def force(ctx: Context, tree, F):
    import torch
    n = tree.n_cells
    a = torch.empty((3, n), dtype=torch.float32, device="cuda")
    p = torch.empty(n, dtype=torch.float32, device="cuda")
    rad_force(ctx, tree, F, a, p)
    return a, p


def dust(ctx: Context, rho, u_rad, t_gas, sigma, c, c_gd=3.8e-33, mlp=None, **kw):
    import torch
    n = rho.numel()
    T = torch.empty(n, dtype=torch.float32, device="cuda")
    it = torch.empty(n, dtype=torch.uint8, device="cuda")
    dust_equilibrium(ctx, rho, u_rad, t_gas, dust_params(sigma, c, c_gd, **kw), T, it, mlp)
    return T, it
