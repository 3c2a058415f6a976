"""Python binding of the MI355X TreeRay/RadPressure library (libtreeray.so).

Argument marshalling only: every step of the hot path runs in the HIP kernels behind
the C ABI declared in ``include/treeray.h``.  Device buffers are torch tensors on the
HIP device (torch provides memory and streams); the library never sees torch types.
Importing this module fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtreeray.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2204_09072_amd.build` "
                      "(hipcc, gfx950)")

_lib = C.CDLL(LIB_PATH)
_P = C.c_void_p

TR_OK, TR_EINVAL, TR_ENOMEM, TR_EHIP, TR_EOVERFLOW = 0, -1, -2, -3, -4


class TreerayError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"treeray error {code}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nb", C.c_int32), ("max_level", C.c_int32), ("n_blk", C.c_int32),
                ("blocks", _P), ("x0", C.c_double * 3), ("box_len", C.c_double)]


class Units(C.Structure):
    _fields_ = [("sigma", C.c_double), ("c", C.c_double)]


class TreeInfo(C.Structure):
    _fields_ = [("n_node", C.c_int64), ("n_leaf", C.c_int64), ("n_cells", C.c_int64),
                ("depth", C.c_int32), ("root_edge", C.c_int32), ("n_bins", C.c_int32),
                ("u_len", C.c_double)]


class TraceParams(C.Structure):
    _fields_ = [("n_side", C.c_int32), ("theta_num", C.c_int32), ("theta_den", C.c_int32),
                ("cube_m", C.c_int32), ("merge", C.c_int32), ("j_bg", C.c_float),
                ("bins_per_pass", C.c_int32), ("chunk", C.c_int32), ("waves_per_block", C.c_int32),
                ("kernel", C.c_int32), ("per_node_kernel", C.c_int32), ("orientation", C.c_int32),
                ("orient_seed", C.c_uint32), ("stack_limit", C.c_int32)]


class BatchTuning(C.Structure):
    _fields_ = [("bins_per_pass", C.c_int32), ("waves_per_block", C.c_int32), ("chunk", C.c_int32),
                ("sample_ms", C.c_float), ("widest_pass", C.c_int32), ("waves_used", C.c_int32)]


class UvParams(C.Structure):
    _fields_ = [("e_ph", C.c_double), ("sigma_d", C.c_double), ("sigma_h", C.c_double),
                ("alpha_b", C.c_double), ("mu_mh", C.c_double), ("c", C.c_double)]


class DustParams(C.Structure):
    _fields_ = [("sigma", C.c_double), ("c", C.c_double), ("c_gd", C.c_double), ("xi", C.c_double),
                ("rel_tol", C.c_float), ("max_iter", C.c_int32), ("start", C.c_int32), ("linear", C.c_int32),
                ("staged", C.c_int32)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_I = C.c_int
_sig("tr_ctx_create", _I, [C.POINTER(_P), _I, _P])
_sig("tr_ctx_destroy", None, [_P])
_sig("tr_ctx_set_stream", _I, [_P, _P])
_sig("tr_ctx_set_validation", _I, [_P, _I])
_sig("tr_last_error", C.c_char_p, [_P])
_sig("tr_sync", _I, [_P])
_sig("tr_build_tree", _I, [_P, C.POINTER(Grid), _P, _P, _P, _P, _I, C.POINTER(Units), C.POINTER(_P)])
_sig("tr_tree_free", None, [_P])
_sig("tr_tree_refill", _I, [_P, _P, _P, _P, _P, _P, _I])
_sig("tr_tree_get_info", _I, [_P, C.POINTER(TreeInfo)])
_sig("tr_tree_export", _I, [_P, _P, _P, _P, _P, _P, _P, _P])
_sig("tr_trace_rays", _I, [_P, _P, C.POINTER(TraceParams), _P, _P, _P])
_sig("tr_walk_counts", _I, [_P, _P, C.POINTER(TraceParams), _P])
_sig("tr_batch_create", _I, [_P, _I, _P, _P, _P, _P, _P, C.POINTER(_P)])
_sig("tr_batch_launch", _I, [_P])
_sig("tr_batch_launch_eager", _I, [_P])
_sig("tr_batch_tune", _I, [_P, _I, C.POINTER(BatchTuning)])
_sig("tr_batch_get_tuning", _I, [_P, C.POINTER(BatchTuning)])
_sig("tr_batch_set_tuning", _I, [_P, C.POINTER(BatchTuning)])
_sig("tr_batch_free", None, [_P])
_sig("tr_trace_rays_batched", _I, [_P, _I, _P, _P, _P, _P, _P])
_sig("tr_ray_tables", _I, [_P, _I, _I, _P, _P])
_sig("tr_alpha_table", _I, [_P, _I, _I, _P])
_sig("tr_rad_force", _I, [_P, _P, _P, _P, _P])
_sig("tr_dust_fixed_point", _I, [_P, C.POINTER(Grid), _P, _P, _P, _I, C.POINTER(Units), C.POINTER(TraceParams),
                                  C.POINTER(DustParams), _P, _I, C.c_float, _P, _P, _P, _P,
                                  C.POINTER(C.c_int32), C.POINTER(C.c_float)])
_sig("tr_star_luminosity_split", _I, [_P, _I, _P, _P, _P, C.c_double, C.c_double, C.c_double, _P, _P])
_sig("tr_uv_rad_pressure", _I, [_P, C.c_int64, _P, _P, _P, _P, C.POINTER(UvParams), _P, _P])
_sig("tr_dust_equilibrium", _I, [_P, C.c_int64, _P, _P, _P, C.POINTER(DustParams), _P, _P, _P])
_sig("tr_dust_equilibrium_noalloc", _I, [_P, C.c_int64, _P, _P, _P, C.POINTER(DustParams), _P, _P, _P])
_sig("tr_mlp_n_params", _I, [])
_sig("tr_mlp_create", _I, [_P, _P, _P, C.POINTER(_P)])
_sig("tr_mlp_free", None, [_P])
_sig("tr_mlp_get_params", _I, [_P, _P, _P])
_sig("tr_mlp_get_state", _I, [_P, _P, _P, _P, _P, _P, _P])
_sig("tr_mlp_set_state", _I, [_P, _P, _P, _P, _P, C.c_int64])
_sig("tr_mlp_forward", _I, [_P, _P, C.c_int64, _P, _P])
_sig("tr_mlp_grad", _I, [_P, _P, C.c_int64, _P, _P, _P, _P])
_sig("tr_mlp_train_step", _I, [_P, _P, C.c_int64, _P, _P, C.c_float, _P])

MLP_NPARAM = _lib.tr_mlp_n_params()
MLP_HIDDEN = 64


def _check_device(name, t, dtype, optional=False):
    """A device array argument must be a contiguous GPU tensor of the given dtype: the
    library dereferences it in kernels."""
    if t is None:
        if optional:
            return
        raise ValueError(f"{name}: required")
    if isinstance(t, np.ndarray) or not getattr(t, "is_cuda", False):
        raise TypeError(f"{name}: a GPU tensor is required (got {type(t).__name__})")
    if str(t.dtype) != f"torch.{dtype}" or not t.is_contiguous():
        raise TypeError(f"{name}: contiguous {dtype} required (got {t.dtype})")


def _ptr(t):
    """Device (or host numpy) address of a buffer, None for None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(_P)
    return _P(t.data_ptr())


class Context:
    """One HIP device and stream (tr_ctx)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        self._torch = torch
        h = _P()
        s = stream if stream is not None else torch.cuda.current_stream(device).cuda_stream
        rc = _lib.tr_ctx_create(C.byref(h), device, _P(s))
        if rc:
            raise TreerayError(rc, "tr_ctx_create failed")
        self.h = h

    def check(self, rc):
        if rc:
            raise TreerayError(rc, _lib.tr_last_error(self.h).decode())

    def set_stream(self, stream):
        self.check(_lib.tr_ctx_set_stream(self.h, _P(stream)))

    def set_validation(self, on: bool):
        self.check(_lib.tr_ctx_set_validation(self.h, int(bool(on))))

    def sync(self):
        self.check(_lib.tr_sync(self.h))

    def close(self, _destroy=_lib.tr_ctx_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Tree:
    """Library-owned octree (tr_tree)."""

    def __init__(self, ctx: Context, h):
        self.ctx = ctx
        self.h = h
        info = TreeInfo()
        ctx.check(_lib.tr_tree_get_info(h, C.byref(info)))
        self.n_node = info.n_node
        self.n_leaf = info.n_leaf
        self.n_cells = info.n_cells
        self.depth = info.depth
        self.root_edge = info.root_edge
        self.n_bins = info.n_bins
        self.u_len = info.u_len

    def refill(self, rho, kappa, t_dust, stars=None):
        """tr_tree_refill: new cell fields (device float32) and stars (device float64 [n, 4]
        or None) on the same blocks; asynchronous, allocation-free."""
        for name, t, dt in (("rho", rho, "float32"), ("kappa", kappa, "float32"), ("t_dust", t_dust, "float32"),
                            ("stars", stars, "float64")):
            _check_device(name, t, dt, optional=name in ("kappa", "stars"))
        if stars is not None and (stars.dim() != 2 or stars.shape[1] != 4):
            raise ValueError("stars: device float64 [n, 4] (x, y, z, L)")
        n = 0 if stars is None else int(stars.shape[0])
        self.ctx.check(_lib.tr_tree_refill(self.ctx.h, self.h, _ptr(rho), _ptr(kappa), _ptr(t_dust),
                                           _ptr(stars) if n else None, n))

    def free(self, _free=_lib.tr_tree_free):
        if getattr(self, "h", None):
            _free(self.h)
            self.h = None

    def __del__(self):
        self.free()


def build_tree(ctx: Context, nb, max_level, blocks, x0, box_len, rho, kappa, t_dust, stars,
               sigma, c) -> Tree:
    """tr_build_tree.  blocks: host int32 [n_blk, 4]; rho, kappa (or None), t_dust: device
    float32 [n_cells]; stars: host float64 [n, 4]."""
    blocks = np.ascontiguousarray(blocks, np.int32)
    g = Grid(int(nb), int(max_level), int(blocks.shape[0]), _ptr(blocks),
             (C.c_double * 3)(*[float(v) for v in x0]), float(box_len))
    st = np.ascontiguousarray(np.asarray(stars, np.float64).reshape(-1, 4))
    u = Units(float(sigma), float(c))
    h = _P()
    ctx.check(_lib.tr_build_tree(ctx.h, C.byref(g), _ptr(rho), _ptr(kappa), _ptr(t_dust),
                                 _ptr(st) if st.shape[0] else None, int(st.shape[0]), C.byref(u),
                                 C.byref(h)))
    return Tree(ctx, h)


def dust_fixed_point(ctx: Context, nb, max_level, blocks, x0, box_len, rho, t_gas, stars, sigma, c,
                     tp: TraceParams, dp: DustParams, t_dust, J, F, u_rad, max_iter=20, tol=1e-4, mlp=None):
    """tr_dust_fixed_point: t_dust (device float32) is the start and receives the result.
    Returns (sweeps, last largest relative change)."""
    blocks = np.ascontiguousarray(blocks, np.int32)
    g = Grid(int(nb), int(max_level), int(blocks.shape[0]), _ptr(blocks),
             (C.c_double * 3)(*[float(v) for v in x0]), float(box_len))
    st = np.ascontiguousarray(np.asarray(stars, np.float64).reshape(-1, 4))
    u = Units(float(sigma), float(c))
    it = C.c_int32(0)
    ch = C.c_float(0.0)
    ctx.check(_lib.tr_dust_fixed_point(ctx.h, C.byref(g), _ptr(rho), _ptr(t_gas),
                                       _ptr(st) if st.shape[0] else None, int(st.shape[0]), C.byref(u),
                                       C.byref(tp), C.byref(dp), None if mlp is None else mlp.h,
                                       int(max_iter), float(tol), _ptr(t_dust), _ptr(J), _ptr(F), _ptr(u_rad),
                                       C.byref(it), C.byref(ch)))
    return int(it.value), float(ch.value)


T_LYC = 13.6 * 1.602176634e-12 / 1.380649e-16   # h nu_LyC / k_B in K


def star_luminosity_split(ctx: Context, L_int, L_acc, r_star, sigma, L_uv, L_ir, f_fill=0.1, t_lyc=T_LYC):
    """tr_star_luminosity_split on device float64 arrays."""
    ctx.check(_lib.tr_star_luminosity_split(ctx.h, int(L_int.numel()), _ptr(L_int), _ptr(L_acc), _ptr(r_star),
                                            float(f_fill), float(sigma), float(t_lyc), _ptr(L_uv), _ptr(L_ir)))


def uv_params(e_ph, sigma_d=1.5e-21, sigma_h=6.3e-18, alpha_b=2.6e-13, mu_mh=1.4 * 1.6735575e-24,
              c=2.99792458e10) -> UvParams:
    return UvParams(float(e_ph), float(sigma_d), float(sigma_h), float(alpha_b), float(mu_mh), float(c))


def uv_rad_pressure(ctx: Context, rho, x_ion, n_ph, u_ph, p: UvParams, a_uv, parts=None):
    """tr_uv_rad_pressure: rho, x_ion, n_ph [n]; u_ph, a_uv, parts [3, n] (device float32)."""
    ctx.check(_lib.tr_uv_rad_pressure(ctx.h, int(rho.numel()), _ptr(rho), _ptr(x_ion), _ptr(n_ph), _ptr(u_ph),
                                      C.byref(p), _ptr(a_uv), _ptr(parts)))


def tree_export(ctx: Context, tree: Tree):
    n = tree.n_node
    out = dict(geo=np.zeros((n, 4), np.int32), meta=np.zeros(n, np.uint32),
               q=np.zeros((n, 4), np.float32), vthick=np.zeros(n, np.float32),
               pcol=np.zeros((n, 3), np.int32), leaf_cell=np.zeros(n, np.int64))
    ctx.check(_lib.tr_tree_export(ctx.h, tree.h, *[_ptr(out[k]) for k in
                                                   ("geo", "meta", "q", "vthick", "pcol", "leaf_cell")]))
    return out


def trace_params(n_side, theta=None, cube_m=0, merge=True, j_bg=0.0, bins_per_pass=0, chunk=0,
                 waves_per_block=0, kernel=0, per_node_kernel=False, orientation=0,
                 orient_seed=0, stack_limit=0) -> TraceParams:
    """kernel: 0 automatic, 1 one wave per target (2, one block per target, is withdrawn).
    per_node_kernel: the 8-point kernel for every node instead of the table for far ones.
    orientation: 0..47 signed axis permutation of the ray set, -1 drawn per target.
    stack_limit: test hook, a walk stack small enough to overflow (0 = one that cannot)."""
    th = (0, 0) if theta is None else theta
    return TraceParams(int(n_side), int(th[0]), int(th[1]), int(cube_m), int(bool(merge)),
                       float(j_bg), int(bins_per_pass), int(chunk), int(waves_per_block), int(kernel),
                       int(bool(per_node_kernel)), int(orientation), int(orient_seed), int(stack_limit))


def trace_rays(ctx: Context, tree: Tree, p: TraceParams, J, F, u_rad=None):
    """tr_trace_rays: J [n], F [3, n], u_rad [n] or None (device float32)."""
    ctx.check(_lib.tr_trace_rays(ctx.h, tree.h, C.byref(p), _ptr(J), _ptr(F), _ptr(u_rad)))


def _batch_arrays(trees, params, J, F, U):
    n = len(trees)
    assert len(params) == n and len(J) == n and len(F) == n
    th = (_P * n)(*[t.h for t in trees])
    pa = (TraceParams * n)(*params)
    ja = (_P * n)(*[_ptr(x) for x in J])
    fa = (_P * n)(*[_ptr(x) for x in F])
    ua = None if U is None else (_P * n)(*[_ptr(x) for x in U])
    return n, th, pa, ja, fa, ua


class Batch:
    """tr_batch: many trees traced by one persistent launch replayed from a HIP graph.
    trees, params, J, F, U: equal-length lists (U may be None or hold None entries)."""

    def __init__(self, ctx: Context, trees, params, J, F, U=None):
        self.ctx = ctx
        self._keep = (list(trees), list(J), list(F), None if U is None else list(U))
        n, th, pa, ja, fa, ua = _batch_arrays(trees, params, J, F, U)
        h = _P()
        ctx.check(_lib.tr_batch_create(ctx.h, n, th, pa, ja, fa, ua, C.byref(h)))
        self.h = h

    def launch(self):
        self.ctx.check(_lib.tr_batch_launch(self.h))

    def launch_eager(self):
        self.ctx.check(_lib.tr_batch_launch_eager(self.h))

    def tune(self, sample_stride=16) -> BatchTuning:
        out = BatchTuning()
        self.ctx.check(_lib.tr_batch_tune(self.h, int(sample_stride), C.byref(out)))
        return out

    def get_tuning(self) -> BatchTuning:
        out = BatchTuning()
        self.ctx.check(_lib.tr_batch_get_tuning(self.h, C.byref(out)))
        return out

    def set_tuning(self, bins_per_pass=0, waves_per_block=0, chunk=0):
        t = BatchTuning(int(bins_per_pass), int(waves_per_block), int(chunk), 0.0, 0, 0)
        self.ctx.check(_lib.tr_batch_set_tuning(self.h, C.byref(t)))

    def free(self, _free=_lib.tr_batch_free):
        if getattr(self, "h", None):
            _free(self.h)
            self.h = None

    def __del__(self):
        self.free()


def trace_rays_batched(ctx: Context, trees, params, J, F, U=None):
    """tr_trace_rays_batched: one persistent launch over all trees (synchronous)."""
    n, th, pa, ja, fa, ua = _batch_arrays(trees, params, J, F, U)
    ctx.check(_lib.tr_trace_rays_batched(ctx.h, n, th, pa, ja, fa, ua))


def walk_counts(ctx: Context, tree: Tree, p: TraceParams, counters):
    """tr_walk_counts: counters device int32 [n, 3]."""
    ctx.check(_lib.tr_walk_counts(ctx.h, tree.h, C.byref(p), _ptr(counters)))


def ray_tables(ctx: Context, n_side: int, cube_m: int = 0):
    M = cube_m or 16 * n_side
    tab = np.zeros(6 * M * M, np.int32)
    dirs = np.zeros((12 * n_side * n_side, 3), np.float32)
    ctx.check(_lib.tr_ray_tables(ctx.h, int(n_side), int(M), _ptr(tab), _ptr(dirs)))
    return tab, dirs


def alpha_table(ctx: Context, n_side: int, cube_m: int = 0):
    """tr_alpha_table: host int32 [6 M M, 15, 9]."""
    M = cube_m or 16 * n_side
    out = np.zeros((6 * M * M, 15, 9), np.int32)
    ctx.check(_lib.tr_alpha_table(ctx.h, int(n_side), int(M), _ptr(out)))
    return out


def rad_force(ctx: Context, tree: Tree, F, a_rp, p_src=None):
    """tr_rad_force: F, a_rp [3, n]; p_src [n] or None (device float32)."""
    ctx.check(_lib.tr_rad_force(ctx.h, tree.h, _ptr(F), _ptr(a_rp), _ptr(p_src)))


def dust_params(sigma, c, c_gd=3.8e-33, xi=1.0, rel_tol=0.0, max_iter=0, start=0, linear=False,
                staged=False) -> DustParams:
    """start 0: secant point of the bracket (log space); 1: the bracket end nearer the root;
    2: plain bisection (no Newton steps).  linear: Newton on the residual itself instead of
    on ln w against ln T.  staged (with a network): the inference into a buffer, then the
    solve, instead of one kernel."""
    return DustParams(float(sigma), float(c), float(c_gd), float(xi), float(rel_tol), int(max_iter),
                      int(start), int(bool(linear)), int(bool(staged)))


def dust_equilibrium(ctx: Context, rho, u_rad, t_gas, p: DustParams, t_dust, iters=None, mlp=None):
    """tr_dust_equilibrium on device float32 arrays; iters uint8 or None."""
    n = int(rho.numel())
    ctx.check(_lib.tr_dust_equilibrium(ctx.h, n, _ptr(rho), _ptr(u_rad), _ptr(t_gas), C.byref(p),
                                       None if mlp is None else mlp.h, _ptr(t_dust), _ptr(iters)))


NOALLOC_DUST_STATES = 1 << 22   # TR_NOALLOC_DUST_STATES


def dust_equilibrium_noalloc(ctx: Context, rho, u_rad, t_gas, p: DustParams, t_dust, iters=None, mlp=None):
    """tr_dust_equilibrium_noalloc (no device allocation; at most NOALLOC_DUST_STATES states)."""
    n = int(rho.numel())
    ctx.check(_lib.tr_dust_equilibrium_noalloc(ctx.h, n, _ptr(rho), _ptr(u_rad), _ptr(t_gas), C.byref(p),
                                               None if mlp is None else mlp.h, _ptr(t_dust), _ptr(iters)))


class Mlp:
    """Guess network (tr_mlp): parameters W1[64][3] b1 W2[64][64] b2 W3[64] b3 (float32)."""

    def __init__(self, ctx: Context, params: np.ndarray, norm=None):
        self.ctx = ctx
        prm = np.ascontiguousarray(params, np.float32)
        assert prm.shape == (MLP_NPARAM,)
        nrm = None if norm is None else np.ascontiguousarray(norm, np.float32)
        h = _P()
        ctx.check(_lib.tr_mlp_create(ctx.h, _ptr(prm), _ptr(nrm), C.byref(h)))
        self.h = h
        self.norm = nrm

    def params(self) -> np.ndarray:
        out = np.zeros(MLP_NPARAM, np.float32)
        self.ctx.check(_lib.tr_mlp_get_params(self.ctx.h, self.h, _ptr(out)))
        return out

    def get_state(self) -> dict:
        """Training state: params, adam_m, adam_v (float32 arrays), steps, norm."""
        prm, m1, m2 = (np.zeros(MLP_NPARAM, np.float32) for _ in range(3))
        norm = np.zeros(8, np.float32)
        steps = C.c_int64(0)
        self.ctx.check(_lib.tr_mlp_get_state(self.ctx.h, self.h, _ptr(prm), _ptr(m1), _ptr(m2),
                                             C.byref(steps), _ptr(norm)))
        return {"params": prm, "adam_m": m1, "adam_v": m2, "steps": int(steps.value), "norm": norm}

    def set_state(self, params, adam_m=None, adam_v=None, steps=0):
        arrs = [None if a is None else np.ascontiguousarray(a, np.float32) for a in (params, adam_m, adam_v)]
        for a in arrs:
            assert a is None or a.shape == (MLP_NPARAM,)
        self.ctx.check(_lib.tr_mlp_set_state(self.ctx.h, self.h, *[_ptr(a) for a in arrs], int(steps)))

    def forward(self, x, y):
        self.ctx.check(_lib.tr_mlp_forward(self.ctx.h, self.h, int(x.shape[0]), _ptr(x), _ptr(y)))

    def grad(self, x, y, grad, loss):
        self.ctx.check(_lib.tr_mlp_grad(self.ctx.h, self.h, int(x.shape[0]), _ptr(x), _ptr(y),
                                        _ptr(grad), _ptr(loss)))

    def train_step(self, x, y, lr, loss=None):
        self.ctx.check(_lib.tr_mlp_train_step(self.ctx.h, self.h, int(x.shape[0]), _ptr(x), _ptr(y),
                                              float(lr), _ptr(loss)))

    def free(self, _free=_lib.tr_mlp_free):
        if getattr(self, "h", None):
            _free(self.h)
            self.h = None

    def __del__(self):
        self.free()


def init_mlp_params(seed: int = 0) -> np.ndarray:
    """Random initial parameters (uniform, fan-in scaled)."""
    rng = np.random.default_rng(seed)
    H = MLP_HIDDEN
    parts = [rng.uniform(-1, 1, 3 * H) / np.sqrt(3), np.zeros(H),
             rng.uniform(-1, 1, H * H) / np.sqrt(H), np.zeros(H),
             rng.uniform(-1, 1, H) / np.sqrt(H), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)
