#!/usr/bin/env python3
"""Benchmark of the TreeRay/RadPressure hot path on one MI355X.

One step = the whole path over one synthetic cloud with inputs resident in HBM:
tree build (b-nodes, h-nodes, centres of luminosity) -> ray tracing (walk, mapping,
integration, finalisation, u_rad) -> radiation-pressure force -> dust equilibrium with
the learned Newton guess.  Prints one JSON line.

Default workload: the AMR cloud, 256^3-equivalent (64^3 base grid of 8^3 blocks refined
twice on density, ~2.5 M leaf cells, 10 stars, T_gas log-uniform 10-300 K), N_side = 4
(192 rays), opening angle 1/8: the full pipeline.  The guess network is trained before
timing, on the GPU by the library's own kernels, on 10^6 states: cells of another
realisation of the cloud (seed 1) traced by the library, plus 20 % log-uniform states,
labelled with the FP64 oracle's bracketed equilibrium solve (the oracle leg, which also
times the oracle for `cpu_baseline`).  The same line carries `batch_c4`: the batch of 64
uneven instances in one autotuned, graph-replayed persistent launch.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "core128": "128^3 collapsing core (0.4 pc, 150 Msun, rho ~ r^-2 x lognormal sigma=1), "
               "T_gas 10-300 K, kappa = kappa_P(T_d), N_side=4 (192 rays), theta=1/8, "
               "dust equilibrium with learned guess",
    "turb64": "64^3 lognormal turbulent box (sigma_ln=1.5, k^-4), kappa 0.1-10, one star, "
              "N_side=2 (48 rays), theta=1/4, code units",
    "sphere16": "16^3 uniform sphere, N_side=1 (12 rays), theta=1/2, code units",
    "amr256": "AMR 256^3-equivalent (64^3 base, 2 extra levels, ~2.5M leaves), 10 stars, "
              "N_side=4 (192 rays), theta=1/8, dust equilibrium with learned guess",
}

B_LEAF, B_HNODE = 12, 36   # algorithmic bytes per accepted b-node / visited h-node
B_ALPHA = 8                # angular-kernel entry per accepted node (up to 4 (ray, alpha) pairs)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2204_09072_amd", "csrc", "trace.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def make_workload(name, seed=0):
    import workloads as W
    if name == "core128":
        return W.c3_core128(seed=seed)
    if name == "turb64":
        return W.c2_turb64(seed=seed)
    if name == "sphere16":
        return W.c1_sphere16()
    if name == "amr256":
        return W.c5_amr256(seed=seed)
    raise SystemExit(f"unknown workload {name}")


def training_states(ctx, name, n_total=1_000_000, aug_frac=0.2, seed=1):
    """(rho, u_rad, T_gas) host arrays for the guess network: random cells of another
    realisation of the workload, their u_rad traced by the library, plus log-uniform states
    over the same ranges (untimed setup)."""
    import workloads as W
    from paper_2204_09072_amd.run import trace, upload
    w = make_workload(name, seed=seed)
    dev = upload(w)
    tree, J, F, U = trace(ctx, w, dev)
    ctx.sync()
    u = U.cpu().numpy()
    tree.free()
    n_aug = int(n_total * aug_frac)
    pick = np.random.default_rng(seed).choice(w.n_cells, min(w.n_cells, n_total - n_aug), replace=False)
    aug = W.dust_samples(n_aug, seed=7, rho_range=(float(w.rho.min()), float(w.rho.max())),
                         u_range=(max(float(u.min()), 1e-30), float(u.max())),
                         t_range=(10.0, 300.0)).astype(np.float32)
    return (np.concatenate([w.rho[pick], aug[:, 0]]), np.concatenate([u[pick], aug[:, 1]]),
            np.concatenate([w.t_gas[pick], aug[:, 2]]))


def library_labels(T, ctx, states, units):
    """Labels from the library's own bracketed solve (only when the oracle leg is off)."""
    import torch
    from paper_2204_09072_amd.run import dust
    dv = [torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda() for a in states]
    Td, _ = dust(ctx, *dv, units[0], units[1])
    ctx.sync()
    return Td.cpu().numpy()


def train_on(ctx, states, labels, steps):
    from paper_2204_09072_amd.guess import train_guess
    t0 = time.perf_counter()
    mlp, losses = train_guess(ctx, *states, labels, steps=steps, batch=8192, log_every=max(steps // 5, 1))
    return mlp, {"steps": steps, "samples": int(len(labels)), "seconds": round(time.perf_counter() - t0, 2),
                 "loss": [round(l, 6) for _, l in losses]}


def interior_states(n, seed):
    """Log-uniform (rho, u_rad, T_gas) on the device (the dust solve's interior states)."""
    import torch
    import workloads as W
    smp = W.dust_samples(n, seed=seed).astype(np.float32)
    return tuple(torch.from_numpy(np.ascontiguousarray(smp[:, k])).cuda() for k in range(3))


DUST_VARIANTS = (("learned", True, {}), ("learned_linear_newton", True, dict(linear=True)),
                 ("learned_staged", True, dict(staged=True)),
                 ("plain", False, dict(start=1, linear=True, max_iter=250)),
                 ("plain_log_newton", False, dict(start=1)), ("secant_log_newton", False, dict(start=0)),
                 ("plain_bisection", False, dict(start=2, max_iter=250)))


def dust_compare(T, ctx, mlp, rho, u_rad, t_gas, units, reps=20):
    """Every start on the same fields with the same stopping rule: time (HIP events, the
    network's inference included for the learned starts), Newton steps, solutions."""
    import torch
    n = rho.numel()
    stats, sol = {}, {}
    for name, learned, kw in DUST_VARIANTS:
        m = mlp if learned else None
        out = torch.empty(n, device="cuda")
        it = torch.empty(n, dtype=torch.uint8, device="cuda")
        dpv = T.dust_params(units[0], units[1], **kw)
        T.dust_equilibrium(ctx, rho, u_rad, t_gas, dpv, out, it, m)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            T.dust_equilibrium(ctx, rho, u_rad, t_gas, dpv, out, it, m)
        e1.record()
        torch.cuda.synchronize()
        ms_v = e0.elapsed_time(e1) / reps
        itf = it.float()
        stats[name] = {"ms": round(ms_v, 4), "solves_per_s": n / (ms_v / 1000.0),
                       "mean_iters": round(float(itf.mean().item()), 3), "max_iters": int(it.max().item()),
                       "iter_hist": [int(v) for v in torch.bincount(it.long()).cpu().numpy()]}
        sol[name] = out.cpu().numpy()
    ref = sol["plain"]
    for name in stats:
        stats[name]["max_rel_diff_vs_plain"] = float(np.max(np.abs(sol[name] - ref) / ref))
    return stats, sol


def dust_summary(stats):
    best_analytic = min(stats[k]["ms"] for k in stats if not k.startswith("learned"))
    best_learned = min(stats[k]["ms"] for k in stats if k.startswith("learned"))
    return {"unit": "T_dust solves/s",
            "learned_solves_per_s": stats["learned"]["solves_per_s"],
            "plain_solves_per_s": stats["plain"]["solves_per_s"],
            "speedup_learned_over_plain": round(stats["plain"]["ms"] / stats["learned"]["ms"], 3),
            "speedup_best_learned_over_plain": round(stats["plain"]["ms"] / best_learned, 3),
            "speedup_learned_over_best_analytic_start": round(best_analytic / stats["learned"]["ms"], 3),
            "variants": stats,
            "stop_rule": "Newton step |dT| <= 1e-6 T (taken before the bracket test) or bracket width "
                         "<= 1e-6 T; bisection when a step leaves the bracket, except that a step reaching an end not yet "
                         "evaluated tries that end once"}


def oracle_labels(states, units, c_gd=3.8e-33):
    """The oracle leg's first part: FP64 bracketed equilibrium temperatures of the guess
    network's training states (host arrays)."""
    import oracle
    T, _ = oracle.dust_eq(*[np.asarray(a, np.float64) for a in states], units[0], units[1], c_gd)
    return T.astype(np.float32)


def cpu_baseline(w, n_pix, stride, u_rad=None, gpu_t_dust=None, gpu_counts=None):
    """FP64 oracle on the host cores: tree, every `stride`-th target, force and dust.  With
    the GPU's walk counters (int [n_cells, 3]) also checks that the oracle's walk of every
    traced target accepts and opens the same numbers of nodes."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    ot = oracle.Tree(w)
    t_tree = time.perf_counter() - t0
    cells = np.arange(0, w.n_cells, stride, dtype=np.int64)
    t0 = time.perf_counter()
    J, F, ocnt = ot.trace(oracle.params(w.n_side, theta=w.theta), cells=cells, n_threads=threads,
                          counters=True)
    t_trace = time.perf_counter() - t0
    walk_check = None
    if gpu_counts is not None:
        same = np.array_equal(np.asarray(gpu_counts)[cells].astype(np.int64), ocnt)
        walk_check = {"targets": int(len(cells)), "equal": bool(same)}
        if not same:
            raise SystemExit("walk counters of the GPU differ from the oracle's")
    t_dust = 0.0
    errs = None
    if w.cgs and w.t_gas is not None:
        m = min(w.n_cells, 200_000)
        rho = w.rho[:m].astype(np.float64)
        u = np.full(m, 1e-10) if u_rad is None else np.asarray(u_rad[:m], np.float64)
        t0 = time.perf_counter()
        To, _ = oracle.dust_eq(rho, u, w.t_gas[:m].astype(np.float64), w.units[0], w.units[1], 3.8e-33)
        t_dust = (time.perf_counter() - t0) * w.n_cells / m
        if gpu_t_dust:
            errs = {k: float(np.max(np.abs(v[:m] - To) / To)) for k, v in gpu_t_dust.items()}
    t_step = t_tree + t_trace * (w.n_cells / len(cells)) + t_dust
    # the same on one thread, over a sample 16 times sparser
    cells1 = np.arange(0, w.n_cells, 16 * stride, dtype=np.int64)
    t0 = time.perf_counter()
    ot.trace(oracle.params(w.n_side, theta=w.theta), cells=cells1, n_threads=1)
    t_trace1 = time.perf_counter() - t0
    t_step1 = t_tree + t_trace1 * (w.n_cells / len(cells1)) + t_dust
    out = {
        "value": w.n_cells * n_pix / t_step,
        "unit": "target-ray evaluations/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"FP64 oracle: full tree build ({t_tree:.2f} s), ray tracing of every "
                   f"{stride}th target ({len(cells)} targets, {t_trace:.2f} s) scaled to all "
                   f"{w.n_cells} targets, dust equilibrium timed on {min(w.n_cells, 200_000)} cells "
                   f"and scaled; estimated step {t_step:.1f} s"),
    }
    out["single_thread"] = {
        "value": w.n_cells * n_pix / t_step1, "cores": 1,
        "sample": (f"ray tracing of every {16 * stride}th target ({len(cells1)} targets, {t_trace1:.2f} s) "
                   f"on one thread, tree build and dust as above (the dust solve, {t_dust:.2f} s, on all threads); "
                   f"estimated step {t_step1:.1f} s")}
    if errs:
        out["dust_max_rel_err"] = errs
    if walk_check:
        out["walk_counts_vs_oracle"] = walk_check
    return out


def _rocpd(paths):
    """Open every rocprofv3 result database under the given paths (rocpd SQLite)."""
    import glob
    import sqlite3
    dbs = []
    for p in paths:
        dbs += sorted(glob.glob(os.path.join(p, "**", "*.db"), recursive=True)) if os.path.isdir(p) else [p]
    if not dbs:
        raise SystemExit(f"no rocprofv3 database under {paths}")
    return [sqlite3.connect(d) for d in dbs]


def summarize_kernels(paths):
    """Text summary of a `rocprofv3 --kernel-trace --stats` run: per-kernel calls and durations
    (the database's top_kernels view holds microseconds)."""
    rows = {}
    for c in _rocpd(paths):
        for name, calls, total, avg, _ in c.execute("select * from top_kernels"):
            r = rows.setdefault(name, [0, 0.0])
            r[0] += calls
            r[1] += total
    tot = sum(r[1] for r in rows.values()) or 1.0
    out = [f"{'calls':>6} {'total ms':>12} {'avg ms':>12} {'share':>7}  kernel"]
    for name, (calls, total) in sorted(rows.items(), key=lambda kv: -kv[1][1]):
        out.append(f"{calls:6d} {total / 1e3:12.3f} {total / calls / 1e3:12.3f} {100 * total / tot:6.2f}%  {name[:110]}")
    return "\n".join(out)


def pmc_per_dispatch(paths):
    """{(kernel, dispatch): {counter: value}} from `rocprofv3 --pmc` runs."""
    res = {}
    for c in _rocpd(paths):
        for kname, disp, cname, val in c.execute(
                "select kernel_name, dispatch_id, counter_name, value from counters_collection"):
            res.setdefault((kname, disp), {})
            res[(kname, disp)][cname] = res[(kname, disp)].get(cname, 0.0) + val
    return res


def trace_counters(paths):
    """Counters of the trace launch (not the walk-count launch) from `rocprofv3 --pmc` runs of
    --traffic-probe, one line per counter."""
    rows = {}
    for (k, _), v in pmc_per_dispatch(paths).items():
        if "k_trace" in k and "<" in k and "true" not in k.split(",")[1]:
            for c, x in v.items():
                rows.setdefault(c, []).append(x)
    return {c: float(np.mean(x)) for c, x in sorted(rows.items())}


def write_traffic(workload, fetch_paths, write_paths, calib_bytes, out_paths, tcc_paths=None):
    """HBM bytes per trace launch from FETCH_SIZE and WRITE_SIZE runs of --traffic-probe,
    each scaled by the same counter's reading for a plain copy of known size; with a
    TCC_HIT_sum / TCC_MISS_sum run also the launch's L2 hit rate."""
    def pick(paths, counter):
        d = pmc_per_dispatch(paths)
        trace = [v[counter] for (k, _), v in d.items() if "k_trace<" in k and "true" not in k.split(",")[1]]
        other = [v[counter] for (k, _), v in d.items() if "k_trace" not in k]
        if not trace or not other:
            raise SystemExit(f"{counter}: trace or calibration dispatch missing")
        return float(np.mean(trace)), float(max(other))
    f_trace, f_copy = pick(fetch_paths, "FETCH_SIZE")
    w_trace, w_copy = pick(write_paths, "WRITE_SIZE")
    kf, kw = calib_bytes / (f_copy * 1024.0), calib_bytes / (w_copy * 1024.0)
    info = {"workload": workload, "kernel": "k_trace", "trace_hip_sha": kernel_source_hash(),
            "fetch_kib_per_launch": f_trace, "write_kib_per_launch": w_trace,
            "copy_bytes": calib_bytes, "copy_fetch_kib": f_copy, "copy_write_kib": w_copy,
            "fetch_scale": kf, "write_scale": kw,
            "bytes_per_launch": f_trace * 1024.0 * kf + w_trace * 1024.0 * kw}
    if tcc_paths:
        cs = trace_counters(tcc_paths)
        info["l2_hit_rate"] = cs["TCC_HIT_sum"] / (cs["TCC_HIT_sum"] + cs["TCC_MISS_sum"])
    for p in out_paths:
        with open(p, "w") as f:
            json.dump(info, f, indent=1)
    return info


CALIB_BYTES = 1 << 30   # plain device-to-device copy used to scale the byte counters


def traffic_probe(name):
    """One trace launch of the workload preceded by a plain 1 GiB device copy (run under
    rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)."""
    import torch
    import paper_2204_09072_amd as T
    from paper_2204_09072_amd.run import params_of, upload
    w = make_workload(name)
    ctx = T.Context(0)
    dev = upload(w)
    src = torch.ones(CALIB_BYTES // 4, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    tree = T.build_tree(ctx, w.nb, w.max_level, w.blocks, w.x0, w.box_len, dev["rho"], dev["kappa"],
                        dev["t_dust"], w.stars, w.units[0], w.units[1])
    n = w.n_cells
    J = torch.empty(n, device="cuda")
    F = torch.empty((3, n), device="cuda")
    T.trace_rays(ctx, tree, params_of(w), J, F, None)
    ctx.sync()
    log(f"traffic probe {name}: one trace launch done")


def mlp_probe(n=2_097_152, steps=20, reps=3):
    """The learned-start solve on n log-uniform interior states, `reps` times in one kernel
    (k_dust_learned: inference and Newton together) and `reps` times staged (k_mlp_infer,
    then k_dust from the stored guesses), then `steps` training steps of 8192 samples
    (k_mlp_train + k_adam): for rocprofv3 runs of the matrix-core counters."""
    import torch
    import paper_2204_09072_amd as T
    import workloads as W
    from paper_2204_09072_amd.guess import features
    ctx = T.Context(0)
    r, u, t = interior_states(n, seed=32)
    f = features(*(x.cpu().numpy().astype(np.float64) for x in (r, u, t)))
    norm = np.array([*f.mean(0), *(1.0 / f.std(0)), 1.3, 2.0], np.float32)
    mlp = T.Mlp(ctx, T.init_mlp_params(0), norm)
    out = torch.empty(n, device="cuda")
    for staged in (False, True):
        dp = T.dust_params(W.SIGMA_SB, W.C_LIGHT, staged=staged)
        for _ in range(reps):
            T.dust_equilibrium(ctx, r, u, t, dp, out, None, mlp)
    rng = np.random.default_rng(5)
    x = torch.from_numpy(rng.normal(size=(8192, 3)).astype(np.float32)).cuda()
    y = torch.from_numpy(rng.normal(size=8192).astype(np.float32)).cuda()
    for _ in range(steps):
        mlp.train_step(x, y, 1e-3)
    ctx.sync()
    log(f"mlp probe: {reps} fused and {reps} staged learned solves of {n} states, {steps} training steps of 8192")
    mlp.free()


def ray_count_study(name):
    """Cost and accuracy of 48, 192 and 768 rays on one workload (the paper's Sec. 7.6
    comparison): trace time per N_side (opening angle 1/(2 N_side)), cost relative to 48
    rays, and the radiation temperature T_J = (pi J / sigma)^(1/4) against 768 rays over
    the whole domain and over its central half."""
    import torch
    import paper_2204_09072_amd as T
    from paper_2204_09072_amd.run import params_of, upload
    import workloads as W
    w = make_workload(name)
    ctx = T.Context(0)
    dev = upload(w)
    tree = T.build_tree(ctx, w.nb, w.max_level, w.blocks, w.x0, w.box_len, dev["rho"], dev["kappa"],
                        dev["t_dust"], w.stars, w.units[0], w.units[1])
    n = w.n_cells
    J = torch.empty(n, device="cuda")
    F = torch.empty((3, n), device="cuda")
    res, tj = {}, {}
    for ns in (2, 4, 8):
        w.n_side, w.theta = ns, (1, 2 * ns)
        p = params_of(w)
        T.trace_rays(ctx, tree, p, J, F, None)   # warm-up (builds the ray tables)
        ctx.sync()
        best = 1e30
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            T.trace_rays(ctx, tree, p, J, F, None)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        ctx.sync()
        tj[ns] = (np.pi * np.maximum(J.cpu().numpy().astype(np.float64), 0) / w.units[0]) ** 0.25
        # accepted nodes per target (the walk counters): the opening angle follows the ray
        # count, so the work per target grows faster than the rays
        cnt = torch.zeros((n, 3), dtype=torch.int32, device="cuda")
        T.walk_counts(ctx, tree, p, cnt)
        ctx.sync()
        acc = float(cnt[:, :2].to(torch.float64).sum().item()) / n
        del cnt
        res[ns] = {"rays": 12 * ns * ns, "trace_ms": round(best, 3),
                   "target_rays_per_s": n * 12 * ns * ns / (best / 1000.0),
                   "accepted_nodes_per_target": round(acc, 1),
                   "ns_per_accepted_node_and_target": round(best * 1e6 / (acc * n), 4)}
        log(f"ray study {name}: N_side {ns}: {best:.1f} ms")
    x = W.synth.cell_centres(w)
    c = np.asarray(w.x0) + 0.5 * w.box_len
    half = np.all(np.abs(x - c) < 0.25 * w.box_len, axis=1)
    for ns in (2, 4):
        r = tj[ns] / np.maximum(tj[8], 1e-300) - 1.0
        res[ns]["t_j_residual_vs_768_full"] = {"mean": float(r.mean()), "std": float(r.std())}
        res[ns]["t_j_residual_vs_768_half"] = {"mean": float(r[half].mean()), "std": float(r[half].std())}
    base = res[2]["trace_ms"]
    out = {"study": "ray count", "workload": f"{name}: {WORKLOADS[name]}", "n_cells": n,
           "cost_ratio_48_192_768": [round(res[k]["trace_ms"] / base, 3) for k in (2, 4, 8)],
           "accepted_node_ratio_48_192_768": [round(res[k]["accepted_nodes_per_target"] /
                                                    res[2]["accepted_nodes_per_target"], 3) for k in (2, 4, 8)],
           "paper_cost_ratio_48_192_768": [1.0, 4.39, 15.98],
           "paper_t_j_residual_vs_768_half": {"48": "-15.4% +- 14%", "192": "-3.77% +- 5.31%"},
           "paper_t_j_residual_vs_768_full": {"48": "-31.0% +- 17.9%", "192": "-13.2% +- 10.5%"},
           "by_n_side": res}
    print(json.dumps(out), flush=True)
    tree.free()


def batch_c4(T, ctx, reps):
    """The 64 uneven instances (edges 32-96, N_side 2 or 4, 0-4 stars; 24.1 M cells) in one
    persistent launch: trees built, the launch autotuned on a sample of targets and captured
    in a HIP graph, then `reps` graph replays timed with HIP events on the library's stream."""
    import torch
    import workloads as W
    from paper_2204_09072_amd.run import params_of, tree_of, upload
    log("batch of 64 instances ...")
    t0 = time.perf_counter()
    ws = W.c4_batch64()
    trees, J, F = [], [], []
    for w in ws:
        trees.append(tree_of(ctx, w, upload(w)))
        J.append(torch.empty(w.n_cells, device="cuda"))
        F.append(torch.empty((3, w.n_cells), device="cuda"))
    ctx.sync()
    b = T.Batch(ctx, trees, [params_of(w) for w in ws], J, F, None)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    tun = b.tune(sample_stride=16)
    t_tune = time.perf_counter() - t0
    b.launch()                      # warm-up replay
    ctx.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.launch()
    e1.record()
    torch.cuda.synchronize()
    ctx.sync()
    ms = e0.elapsed_time(e1) / reps
    cells = sum(w.n_cells for w in ws)
    rays = sum(w.n_cells * 12 * w.n_side ** 2 for w in ws)
    b.free()
    for t in trees:
        t.free()
    return {"value": rays / (ms / 1000.0), "unit": "target-ray evaluations/s", "ms_per_launch": round(ms, 2),
            "replays": reps, "instances": len(ws), "cells": int(cells), "target_rays": int(rays),
            "tuned": {"bins_per_pass": tun.bins_per_pass, "waves_per_block": tun.waves_per_block,
                      "chunk": tun.chunk, "widest_pass": tun.widest_pass, "waves_used": tun.waves_used,
                      "sample_ms": round(tun.sample_ms, 3), "tune_seconds": round(t_tune, 2)},
            "setup_seconds": round(t_setup, 2),
            "workload": "64 instances, edge uniform over {32, 40, ..., 96} (8^3 blocks), lognormal sigma=1.5, "
                        "kappa 0.1-10, 0-4 stars of L=1, N_side 2 or 4, code units; one autotuned persistent "
                        "launch replayed from a HIP graph"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="amr256", choices=sorted(WORKLOADS))
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--cpu-stride", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (timing, training labels and walk-count check)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance batch (batch_c4)")
    ap.add_argument("--batch-reps", type=int, default=2)
    ap.add_argument("--bins-per-pass", type=int, default=0)
    ap.add_argument("--waves-per-block", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--traffic-probe", action="store_true",
                    help="one calibration copy and one trace launch, for rocprofv3 --pmc runs")
    ap.add_argument("--summarize", nargs="+", metavar="DIR",
                    help="print the per-kernel summary of rocprofv3 --kernel-trace --stats output")
    ap.add_argument("--counters", nargs="+", metavar="DIR",
                    help="print the trace launch's counters from rocprofv3 --pmc runs of --traffic-probe")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/trace_<workload>_traffic.json from two --pmc runs")
    ap.add_argument("--traffic-out", nargs="*", default=None)
    ap.add_argument("--tcc", nargs="*", default=None, metavar="DIR",
                    help="with --write-traffic: a TCC_HIT_sum TCC_MISS_sum run for the L2 hit rate")
    ap.add_argument("--mlp-probe", action="store_true",
                    help="guess-network inference and training only, for rocprofv3 --pmc runs")
    ap.add_argument("--ray-study", action="store_true",
                    help="trace cost and T_J accuracy at 48, 192 and 768 rays (prints one JSON line)")
    args = ap.parse_args()
    if args.summarize:
        print(summarize_kernels(args.summarize))
        return
    if args.counters:
        cs = trace_counters(args.counters)
        for c, v in cs.items():
            print(f"{c:24s} {v:.4e}")
        if "TCC_HIT_sum" in cs and "TCC_MISS_sum" in cs:
            print(f"L2 hit rate              {cs['TCC_HIT_sum'] / (cs['TCC_HIT_sum'] + cs['TCC_MISS_sum']):.4f}")
        if "TCP_TOTAL_CACHE_ACCESSES_sum" in cs and "TCP_TCC_READ_REQ_sum" in cs:
            print(f"L1 hit rate (reads)      "
                  f"{1.0 - cs['TCP_TCC_READ_REQ_sum'] / cs['TCP_TOTAL_CACHE_ACCESSES_sum']:.4f}")
        return
    if args.write_traffic:
        outs = args.traffic_out or [os.path.join(ROOT, "profiles", f"trace_{args.workload}_traffic.json")]
        print(json.dumps(write_traffic(args.workload, [args.write_traffic[0]], [args.write_traffic[1]],
                                       CALIB_BYTES, outs, args.tcc)))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run it with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if args.traffic_probe:
        traffic_probe(args.workload)
        return
    if args.ray_study:
        ray_count_study(args.workload)
        return
    if args.mlp_probe:
        mlp_probe()
        return

    import torch
    import paper_2204_09072_amd as T
    from paper_2204_09072_amd.run import params_of, upload

    w = make_workload(args.workload)
    n_pix = 12 * w.n_side * w.n_side
    ctx = T.Context(0)
    dev = upload(w)
    log(f"workload {args.workload}: {w.n_cells} cells, {n_pix} rays")
    oracle_leg = not args.no_cpu_baseline

    # guess network (untimed setup): trained by the library on 10^6 states labelled by the
    # oracle leg's FP64 equilibrium solve (the library's own solve when that leg is off)
    mlp = None
    train_info = None
    if w.cgs:
        states = training_states(ctx, args.workload)
        t0 = time.perf_counter()
        labels = oracle_labels(states, w.units) if oracle_leg else library_labels(T, ctx, states, w.units)
        t_lab = time.perf_counter() - t0
        mlp, train_info = train_on(ctx, states, labels, args.train_steps)
        train_info["labels"] = ("FP64 oracle, bracketed solve (%.2f s)" % t_lab) if oracle_leg else \
            "library's bracketed solve (oracle leg off)"
        log("guess network trained", train_info)

    p = params_of(w, bins_per_pass=args.bins_per_pass, waves_per_block=args.waves_per_block,
                  chunk=args.chunk)
    n = w.n_cells
    J = torch.empty(n, device="cuda")
    F = torch.empty((3, n), device="cuda")
    U = torch.empty(n, device="cuda")
    A = torch.empty((3, n), device="cuda")
    PS = torch.empty(n, device="cuda")
    TD = torch.empty(n, device="cuda")
    IT = torch.empty(n, dtype=torch.uint8, device="cuda")
    dp = T.dust_params(w.units[0], w.units[1])

    ev = {k: [torch.cuda.Event(enable_timing=True) for _ in range(2)]
          for k in ("build", "trace", "force", "dust")}
    times = {k: [] for k in ev}

    def step(record):
        e = ev if record else None
        if e: e["build"][0].record()
        tree = T.build_tree(ctx, w.nb, w.max_level, w.blocks, w.x0, w.box_len, dev["rho"],
                            dev["kappa"], dev["t_dust"], w.stars, w.units[0], w.units[1])
        if e: e["build"][1].record(); e["trace"][0].record()
        T.trace_rays(ctx, tree, p, J, F, U)
        if e: e["trace"][1].record(); e["force"][0].record()
        T.rad_force(ctx, tree, F, A, PS)
        if e: e["force"][1].record()
        if w.cgs:
            if e: e["dust"][0].record()
            T.dust_equilibrium(ctx, dev["rho"], U, dev["t_gas"], dp, TD, IT, mlp)
            if e: e["dust"][1].record()
        return tree

    for i in range(args.warmup):
        step(False).free()
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    trees = []
    for i in range(args.steps):
        tr = step(True)
        torch.cuda.synchronize()
        for k in ev:
            if k == "dust" and not w.cgs:
                continue
            times[k].append(ev[k][0].elapsed_time(ev[k][1]))
        trees.append(tr)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.sync()
    for tr in trees[:-1]:
        tr.free()
    tree = trees[-1]
    ms = (t1 - t0) * 1000.0 / args.steps

    # the allocation-free refill of the same tree (what a graph-captured step runs in place of
    # the build); reported beside the step, which keeps the build
    st_dev = (torch.from_numpy(np.ascontiguousarray(np.asarray(w.stars, np.float64).reshape(-1, 4)))
              .cuda() if len(w.stars) else None)
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tree.refill(dev["rho"], dev["kappa"], dev["t_dust"], st_dev)
    refill_ms = []
    for i in range(3):
        r0.record()
        tree.refill(dev["rho"], dev["kappa"], dev["t_dust"], st_dev)
        r1.record()
        torch.cuda.synchronize()
        refill_ms.append(r0.elapsed_time(r1))
    ctx.sync()
    times["refill"] = refill_ms
    value = n * n_pix / (ms / 1000.0)
    log(f"timed {args.steps} steps: {ms:.1f} ms per step")

    # roofline of the dominant kernel (the ray-tracing walk): algorithmic bytes from the walk
    # counters (checked against the oracle's on the oracle leg's targets)
    cnt = torch.zeros((n, 3), dtype=torch.int32, device="cuda")
    T.walk_counts(ctx, tree, params_of(w), cnt)
    ctx.sync()
    cnt_h = cnt.cpu().numpy()
    c = cnt_h.astype(np.int64).sum(0)
    node_bytes = float(B_LEAF * c[0] + B_HNODE * (c[1] + c[2]))
    alpha_bytes = float(B_ALPHA * (c[0] + c[1]))
    alg_bytes = node_bytes + alpha_bytes
    t_trace = float(np.mean(times["trace"])) / 1000.0
    achieved = alg_bytes / t_trace / 1e9
    traffic = l2_hit = None
    tj = os.path.join(ROOT, "profiles", f"trace_{args.workload}_traffic.json")
    if os.path.exists(tj):
        with open(tj) as f:
            tr_info = json.load(f)
        if tr_info.get("trace_hip_sha") == kernel_source_hash():
            traffic = tr_info.get("bytes_per_launch")
            l2_hit = tr_info.get("l2_hit_rate")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
            "frac": round(achieved / 8000.0, 4), "traffic": traffic,
            "l2_hit_rate": None if l2_hit is None else round(l2_hit, 4),
            "kernel": "k_trace", "algorithmic_bytes_per_launch": alg_bytes,
            "algorithmic_bytes": ("12 B per accepted leaf + 36 B per accepted or opened h-node (node "
                                  "records) + 8 B per accepted node (its angular-kernel entry of up to "
                                  "4 (ray, alpha) pairs)"),
            "node_bytes_per_launch": node_bytes, "alpha_bytes_per_launch": alpha_bytes,
            "kernel_ms": round(t_trace * 1000, 3),
            "walk_totals": {"b_nodes_accepted": int(c[0]), "h_nodes_accepted": int(c[1]),
                            "h_nodes_opened": int(c[2])}}

    # dust: the learned start against the solve without the network, same stopping rule;
    # "plain" is Newton on the residual from the bracket end nearer the root (bisection
    # safeguarded); the log-space variants are this library's stronger analytic starts
    dust = None
    dust_T = {}
    if w.cgs:
        stats, dust_T = dust_compare(T, ctx, mlp, dev["rho"], U, dev["t_gas"], w.units)
        dust = dust_summary(stats)
        dust["network"] = train_info
        # states inside the bracket (log-uniform over the dense-cloud range), where a guess
        # can help: in the cloud most cells have T_dust at a bracket end (T_gas or T_J)
        log("dust on interior states ...")
        t0 = time.perf_counter()
        st_tr = interior_states(200_000, seed=31)
        st_tr = tuple(x.cpu().numpy() for x in st_tr)
        lab = oracle_labels(st_tr, w.units) if oracle_leg else library_labels(T, ctx, st_tr, w.units)
        mlp_i, info_i = train_on(ctx, st_tr, lab, args.train_steps)
        ri, ui, ti = interior_states(n, seed=32)
        st_i, _ = dust_compare(T, ctx, mlp_i, ri, ui, ti, w.units)
        dust["interior_states"] = dict(dust_summary(st_i), network=info_i,
                                       states="%d log-uniform (rho 1e-24..1e-14 g/cm^3, u_rad 1e-16..1e-6 "
                                              "erg/cm^3, T_gas 5..2000 K), network trained on another "
                                              "draw of 200 000" % n,
                                       seconds=round(time.perf_counter() - t0, 2))
        mlp_i.free()

    batch = None if args.no_batch else batch_c4(T, ctx, args.batch_reps)

    base = None
    if oracle_leg:
        log("cpu baseline (oracle) ...")
        base = cpu_baseline(w, n_pix, args.cpu_stride, U.cpu().numpy(), dust_T, gpu_counts=cnt_h)
        if dust is not None and base.get("dust_max_rel_err"):
            for k, v in base.pop("dust_max_rel_err").items():
                dust["variants"][k]["max_rel_err_vs_oracle"] = v

    out = {
        "metric": "target-ray evaluations/s + T_dust solves/s, learned vs plain at fixed error",
        "value": value,
        "unit": "target-ray evaluations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}",
                   "n_cells": n, "n_pix": n_pix, "n_bins": tree.n_bins, "n_nodes": tree.n_node,
                   "bins_per_pass": args.bins_per_pass, "parallelism": "single GPU"},
        "kernels_ms": {k: round(float(np.mean(v)), 3) for k, v in times.items() if v},
        "dust": dust,
        "roofline": roof,
        "batch_c4": batch,
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)
    tree.free()


if __name__ == "__main__":
    main()
