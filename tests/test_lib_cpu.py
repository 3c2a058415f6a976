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
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(tr_grid), sizeof(tr_units), sizeof(tr_tree_info),
         sizeof(tr_trace_params), sizeof(tr_dust_params), sizeof(tr_star));
  printf("%zu %zu %zu %zu\n", offsetof(tr_grid, box_len), offsetof(tr_trace_params, j_bg),
         offsetof(tr_dust_params, rel_tol), offsetof(tr_tree_info, u_len));
  return 0;
}
'''
    src = str(tmp_path / "abi_probe.c")
    exe = str(tmp_path / "abi_probe")
    with open(src, "w") as f:
        f.write(probe)
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
    out = subprocess.check_output([exe]).decode().split()
    sizes = [int(v) for v in out[:6]]
    offs = [int(v) for v in out[6:]]
    assert sizes == [ctypes.sizeof(T.Grid), ctypes.sizeof(T.Units), ctypes.sizeof(T.TreeInfo),
                     ctypes.sizeof(T.TraceParams), ctypes.sizeof(T.DustParams), 32]
    assert offs == [T.Grid.box_len.offset, T.TraceParams.j_bg.offset, T.DustParams.rel_tol.offset,
                    T.TreeInfo.u_len.offset]


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
