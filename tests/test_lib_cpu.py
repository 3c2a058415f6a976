"""Host-side checks that need no GPU: the C-ABI library loads and exports every symbol
its header declares, the binding's structures match the header, the input layout helpers
are consistent, and the benchmark refuses multi-GPU runs."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "treeray.h")
LIB = os.path.join(ROOT, "paper_2204_09072_amd", "libtreeray.so")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tr_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_binding_structs_match_header(tmp_path):
    """Compile a host probe against the header and compare struct sizes and offsets with
    the ctypes mirrors of the binding."""
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    import paper_2204_09072_amd as T
    probe = r'''
#include <stdio.h>
#include <stddef.h>
#include "treeray.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(tr_grid), sizeof(tr_units), sizeof(tr_tree_info),
         sizeof(tr_trace_params), sizeof(tr_dust_params), sizeof(tr_star), sizeof(tr_batch_tuning),
         sizeof(tr_uv_params));
  printf("%zu %zu %zu %zu %zu\n", offsetof(tr_grid, box_len), offsetof(tr_trace_params, j_bg),
         offsetof(tr_dust_params, rel_tol), offsetof(tr_tree_info, u_len),
         offsetof(tr_batch_tuning, waves_used));
  return 0;
}
'''
    src = str(tmp_path / "abi_probe.c")
    exe = str(tmp_path / "abi_probe")
    with open(src, "w") as f:
        f.write(probe)
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
    out = subprocess.check_output([exe]).decode().split()
    sizes = [int(v) for v in out[:8]]
    offs = [int(v) for v in out[8:]]
    assert sizes == [ctypes.sizeof(T.Grid), ctypes.sizeof(T.Units), ctypes.sizeof(T.TreeInfo),
                     ctypes.sizeof(T.TraceParams), ctypes.sizeof(T.DustParams), 32,
                     ctypes.sizeof(T.BatchTuning), ctypes.sizeof(T.UvParams)]
    assert offs == [T.Grid.box_len.offset, T.TraceParams.j_bg.offset, T.DustParams.rel_tol.offset,
                    T.TreeInfo.u_len.offset, T.BatchTuning.waves_used.offset]


def test_dense_block_layout_roundtrip():
    rng = np.random.default_rng(0)
    a = rng.normal(size=(24, 24, 24))
    b = W.uniform_blocks(3)
    cells = W.dense_to_blocks(a, b)
    assert np.array_equal(W.blocks_to_dense(cells, b, 3), a)
    # local index ci + 8 cj + 64 ck
    assert cells[1] == a[1, 0, 0] and cells[8] == a[0, 1, 0] and cells[64] == a[0, 0, 1]


def test_grf_is_unit_gaussian_with_steep_spectrum():
    g = W.grf(32, np.random.default_rng(1))
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1) < 1e-12
    p = np.abs(np.fft.fftn(g)) ** 2
    k = np.sqrt(sum(np.meshgrid(*(np.fft.fftfreq(32) ** 2,) * 3, indexing="ij")))
    lo, hi = p[(k > 0.05) & (k < 0.1)].mean(), p[(k > 0.2) & (k < 0.4)].mean()
    assert lo / hi > 100          # ~k^-4


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_guess_checkpoint_file_roundtrip(tmp_path):
    """The network's checkpoint files (flat float32 arrays + JSON header) read back exactly,
    and a corrupted or foreign file is refused."""
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    import json
    import paper_2204_09072_amd as T
    from paper_2204_09072_amd.guess import read_checkpoint, write_checkpoint
    rng = np.random.default_rng(3)
    st = {"params": rng.normal(size=T.MLP_NPARAM).astype(np.float32),
          "adam_m": rng.normal(size=T.MLP_NPARAM).astype(np.float32),
          "adam_v": rng.random(T.MLP_NPARAM).astype(np.float32),
          "steps": 1234, "norm": np.arange(8, dtype=np.float32)}
    path = str(tmp_path / "net.ckpt")
    write_checkpoint(path, st)
    back = read_checkpoint(path)
    for k in ("params", "adam_m", "adam_v", "norm"):
        assert np.array_equal(back[k], st[k]), k
    assert back["steps"] == 1234
    assert os.path.getsize(path) == 3 * 4 * T.MLP_NPARAM
    raw = bytearray(open(path, "rb").read())
    raw[100] ^= 1
    open(path, "wb").write(bytes(raw))
    with pytest.raises(ValueError):
        read_checkpoint(path)
    write_checkpoint(path, st)
    hdr = json.load(open(path + ".json"))
    hdr["n_params"] = 17
    json.dump(hdr, open(path + ".json", "w"))
    with pytest.raises(ValueError):
        read_checkpoint(path)


def test_tuning_cache_store_and_key(tmp_path):
    """The autotune cache keeps one setting per (architecture, N_side set, radial points,
    instances, grid class) and applies a stored one instead of searching again."""
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from types import SimpleNamespace as NS
    from paper_2204_09072_amd import tuning
    trees = [NS(n_bins=21, n_cells=32768), NS(n_bins=29, n_cells=262144)]
    params = [NS(n_side=4), NS(n_side=2)]
    key = tuning.cache_key("gfx950:sramecc+:xnack-", trees, params)
    assert key == "gfx950|n_side=2,4|n_bins=29|instances=2|cells~2^18"
    path = str(tmp_path / "tune.json")
    assert tuning.load(path) == {}

    class FakeBatch:
        def __init__(self):
            self.searched = 0
            self.applied = None

        def tune(self, stride):
            self.searched += 1
            return NS(bins_per_pass=0, waves_per_block=8, chunk=2, sample_ms=1.25, widest_pass=14, waves_used=8)

        def set_tuning(self, bp, waves, chunk):
            self.applied = (bp, waves, chunk)

        def get_tuning(self):
            return NS(bins_per_pass=self.applied[0], waves_per_block=self.applied[1], chunk=self.applied[2])

    b = FakeBatch()
    t, hit = tuning.tune_cached(b, path, key)
    assert not hit and b.searched == 1 and t.waves_per_block == 8
    b2 = FakeBatch()
    t2, hit2 = tuning.tune_cached(b2, path, key)
    assert hit2 and b2.searched == 0 and b2.applied == (0, 8, 2)
    assert tuning.load(path)[key]["widest_pass"] == 14


def test_binding_rejects_host_arrays_for_device_arguments():
    """The refill's arrays are dereferenced in kernels: the binding refuses host arrays and
    wrong dtypes before anything reaches the library."""
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    import torch
    import paper_2204_09072_amd as T
    with pytest.raises(TypeError):
        T._check_device("stars", np.zeros((1, 4)), "float64")
    with pytest.raises(TypeError):
        T._check_device("rho", torch.zeros(4), "float32")   # a host tensor
    with pytest.raises(ValueError):
        T._check_device("rho", None, "float32")
    T._check_device("kappa", None, "float32", optional=True)


def test_entry_points_refuse_null_handles():
    """Every call that takes a context, tree, batch or network returns TR_EINVAL (-1) for a
    null one before anything reaches the GPU (runs on a host without one)."""
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    calls = {
        "tr_build_tree": [None] * 9,
        "tr_tree_refill": [None, None, None, None, None, None, 0],
        "tr_trace_rays": [None] * 6,
        "tr_walk_counts": [None] * 4,
        "tr_rad_force": [None] * 5,
        "tr_dust_equilibrium": [None, 0] + [None] * 7,
        "tr_dust_equilibrium_noalloc": [None, 0] + [None] * 7,
        "tr_dust_fixed_point": [None] * 10 + [1, 0.0] + [None] * 6,
        "tr_trace_rays_batched": [None, 1] + [None] * 5,
        "tr_batch_create": [None, 1] + [None] * 6,
        "tr_batch_launch": [None],
        "tr_batch_launch_eager": [None],
        "tr_batch_tune": [None, 16, None],
        "tr_batch_set_tuning": [None, None],
        "tr_mlp_create": [None] * 4,
        "tr_mlp_forward": [None, None, 0, None, None],
        "tr_mlp_train_step": [None, None, 0, None, None, 0.0, None],
        "tr_ray_tables": [None, 4, 64, None, None],
        "tr_alpha_table": [None, 4, 64, None],
        "tr_star_luminosity_split": [None, 0, None, None, None, 0.1, 1.0, 1.0, None, None],
        "tr_uv_rad_pressure": [None, 0] + [None] * 7,
        "tr_sync": [None],
        "tr_ctx_set_stream": [None, None],
        "tr_ctx_set_validation": [None, 1],
        "tr_tree_get_info": [None, None],
        "tr_tree_export": [None] * 8,
    }
    for name, args in calls.items():
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        conv = [ctypes.c_double(a) if isinstance(a, float) else (ctypes.c_int(a) if isinstance(a, int) else P(a))
                for a in args]
        assert f(*conv) == -1, name
