"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

The oracle is the plain reference the HIP library is checked against.  Only the
tests, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may
import this package; the library under ``paper_2204_09072_amd`` never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "treeray_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

NB_FIELDS = 6
DEFAULT_CUBE_PER_NSIDE = 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-Wno-unused-function", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.or_build_tree.restype = P
        L.or_build_tree.argtypes = [C.c_int, C.c_int, C.c_int, P, P, C.c_double, P, P, P,
                                    C.c_int, P, C.c_double]
        L.or_tree_free.argtypes = [P]
        L.or_tree_count.restype = C.c_int64
        L.or_tree_count.argtypes = [P, C.c_int]
        L.or_tree_u_len.restype = C.c_double
        L.or_tree_u_len.argtypes = [P]
        L.or_tree_export.argtypes = [P, P, P, P, P, P, P]
        L.or_tree_export_f64.argtypes = [P, P]
        L.or_pix2vec.argtypes = [C.c_int, C.c_int, P]
        L.or_vec2pix.restype = C.c_int
        L.or_vec2pix.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
        L.or_vec2pix_many.argtypes = [C.c_int, C.c_int64, P, P]
        L.or_march.restype = C.c_double
        L.or_march.argtypes = [C.c_int, C.c_double, P, P, P, P, C.c_int, P]
        L.or_march_mean.argtypes = [C.c_int, C.c_double, P, P, C.c_int64, P, C.c_int, C.c_int,
                                    C.c_int, P, P]
        L.or_cube_table.argtypes = [C.c_int, C.c_int, P]
        L.or_alpha_table.argtypes = [C.c_int, P, P]
        L.or_trace.restype = C.c_int
        L.or_trace.argtypes = [P, P, C.c_int64, P, P, P, P, C.c_int]
        L.or_trace_one.restype = C.c_int
        L.or_trace_one.argtypes = [P, P, C.c_int64, C.c_int, P, P, P, P, P, P]
        L.or_integrate_ray.restype = C.c_double
        L.or_integrate_ray.argtypes = [C.c_int, C.c_int, P, P, C.c_double]
        L.or_rad_force.argtypes = [P, P, P, P, P, C.c_double, P, P]
        L.or_dust_eq.argtypes = [C.c_int64, P, P, P, C.c_double, C.c_double, C.c_double,
                                 C.c_double, P, P]
        L.or_dust_residual.restype = C.c_double
        L.or_dust_residual.argtypes = [C.c_double] * 8
        L.or_lyman_fraction.restype = C.c_double
        L.or_lyman_fraction.argtypes = [C.c_double, C.c_double]
        L.or_luminosity_split.argtypes = [C.c_int, P, P, P, C.c_double, C.c_double, C.c_double, P, P]
        L.or_uv_rad_pressure.argtypes = [C.c_int64, P, P, P, P] + [C.c_double] * 6 + [P, P]
        L.or_mlp.restype = C.c_double
        L.or_mlp.argtypes = [C.c_int, P, C.c_int64, P, P, C.c_int, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _Params(C.Structure):
    _fields_ = [("n_side", C.c_int), ("theta_num", C.c_int), ("theta_den", C.c_int),
                ("cube_m", C.c_int), ("merge", C.c_int), ("j_bg", C.c_double),
                ("orient", C.c_int), ("orient_seed", C.c_uint), ("alpha_table", C.c_int)]


def params(n_side, theta=None, cube_m=None, merge=True, j_bg=0.0, orient=0, orient_seed=0, alpha_table=True):
    """orient: 0..47 signed axis permutation of the ray set, -1 drawn per target cell.
    alpha_table: tabulated angular kernel for nodes at least 8 edges away."""
    theta = (1, 2 * n_side) if theta is None else theta
    cube_m = DEFAULT_CUBE_PER_NSIDE * n_side if cube_m is None else cube_m
    return _Params(int(n_side), int(theta[0]), int(theta[1]), int(cube_m), int(bool(merge)),
                   float(j_bg), int(orient), int(orient_seed), int(bool(alpha_table)))


class Tree:
    """FP64 oracle tree over a workload (see workloads.synth.Workload)."""

    def __init__(self, w, t_dust=None, kappa="from_workload"):
        L = lib()
        self.w = w
        self._keep = []
        blocks = np.ascontiguousarray(w.blocks, np.int32)
        x0 = np.asarray(w.x0, np.float64)
        rho = np.ascontiguousarray(w.rho, np.float32)
        kap = w.kappa if kappa == "from_workload" else kappa
        kap = None if kap is None else np.ascontiguousarray(kap, np.float32)
        td = np.ascontiguousarray(w.t_dust if t_dust is None else t_dust, np.float32)
        st = np.ascontiguousarray(w.stars, np.float64).reshape(-1, 4)
        self.rho, self.kappa, self.t_dust = rho, kap, td
        h = L.or_build_tree(int(w.nb), int(w.max_level), int(blocks.shape[0]), _p(blocks),
                            _p(x0), float(w.box_len), _p(rho), _p(kap), _p(td),
                            int(st.shape[0]), _p(st), float(w.units[0]))
        if not h:
            raise ValueError("oracle rejected the grid")
        self.h = h
        self.n_node = L.or_tree_count(h, 0)
        self.n_leaf = L.or_tree_count(h, 1)
        self.depth = L.or_tree_count(h, 2)
        self.root_edge = L.or_tree_count(h, 3)
        self.n_bins = L.or_tree_count(h, 4)
        self.n_cells = L.or_tree_count(h, 5)
        self.u_len = L.or_tree_u_len(h)

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_tree_free(self.h)
            self.h = None

    def export(self):
        n = self.n_node
        geo = np.zeros((n, 4), np.int32)
        meta = np.zeros(n, np.uint32)
        q = np.zeros((n, 4), np.float32)
        vt = np.zeros(n, np.float32)
        pc = np.zeros((n, 3), np.int32)
        lc = np.zeros(n, np.int64)
        lib().or_tree_export(self.h, _p(geo), _p(meta), _p(q), _p(vt), _p(pc), _p(lc))
        return dict(geo=geo, meta=meta, q=q, vthick=vt, pcol=pc, leaf_cell=lc)

    def export_f64(self):
        out = np.zeros((self.n_node, 6))
        lib().or_tree_export_f64(self.h, _p(out))
        return out

    def trace(self, prm, cells=None, n_threads=0, counters=False):
        n = self.n_cells if cells is None else len(cells)
        c = None if cells is None else np.ascontiguousarray(cells, np.int64)
        J = np.zeros(n)
        F = np.zeros((n, 3))
        cnt = np.zeros((n, 3), np.int64) if counters else None
        rc = lib().or_trace(self.h, C.byref(prm), n, _p(c), _p(J), _p(F), _p(cnt), int(n_threads))
        if rc:
            raise ValueError("oracle trace failed")
        return (J, F, cnt) if counters else (J, F)

    def trace_one(self, prm, cell, brute=False):
        npix = 12 * prm.n_side * prm.n_side
        nb = self.n_bins
        bins = np.zeros((npix, nb + 1, NB_FIELDS))
        flags = np.zeros((npix, nb + 1), np.uint8)
        Fh = np.zeros(npix)
        tau = np.zeros(npix)
        J = np.zeros(1)
        F = np.zeros(3)
        rc = lib().or_trace_one(self.h, C.byref(prm), int(cell), int(bool(brute)), _p(bins),
                                _p(flags), _p(Fh), _p(tau), _p(J), _p(F))
        if rc:
            raise ValueError("oracle trace_one failed")
        return dict(bins=bins, flags=flags, Fh=Fh, tau=tau, J=J[0], F=F)

    def rad_force(self, F, c):
        n = self.n_cells
        F = np.ascontiguousarray(F, np.float64).reshape(n, 3)
        a = np.zeros((n, 3))
        ps = np.zeros(n)
        lib().or_rad_force(self.h, _p(self.rho), _p(self.kappa), _p(self.t_dust), _p(F),
                           float(c), _p(a), _p(ps))
        return a, ps


def pix2vec(n_side, pix):
    v = np.zeros(3)
    lib().or_pix2vec(int(n_side), int(pix), _p(v))
    return v


def ray_dirs(n_side):
    return np.stack([pix2vec(n_side, p) for p in range(12 * n_side * n_side)])


def vec2pix(n_side, v):
    return lib().or_vec2pix(int(n_side), float(v[0]), float(v[1]), float(v[2]))


def vec2pix_many(n_side, v):
    """Pixel ids of directions v [n, 3]."""
    v = np.ascontiguousarray(v, np.float64).reshape(-1, 3)
    out = np.zeros(v.shape[0], np.int32)
    lib().or_vec2pix_many(int(n_side), v.shape[0], _p(v), _p(out))
    return out


def march(kr, B, box, p, u, skip_own=False):
    """Direct ray marching (no tree) through dense [n, n, n] arrays (index [i, j, k] along
    x, y, z) of rho*kappa per length and source function: (intensity, optical depth)."""
    kr = np.ascontiguousarray(kr, np.float64)
    B = np.ascontiguousarray(B, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    tau = np.zeros(1)
    I = lib().or_march(int(kr.shape[0]), float(box), _p(kr), _p(B), _p(p), _p(u), int(bool(skip_own)),
                       _p(tau))
    return I, tau[0]


def march_mean(kr, B, box, pts, n_side, sub=3, skip_own=False):
    """Mean intensity J and mean absorbed fraction <1 - e^-tau> at each point of pts [m, 3]
    by direct marching along the 4^sub sub-pixels of every pixel of the N_side set."""
    kr = np.ascontiguousarray(kr, np.float64)
    B = np.ascontiguousarray(B, np.float64)
    pts = np.ascontiguousarray(pts, np.float64).reshape(-1, 3)
    m = pts.shape[0]
    J = np.zeros(m)
    A = np.zeros(m)
    lib().or_march_mean(int(kr.shape[0]), float(box), _p(kr), _p(B), m, _p(pts), int(n_side), int(sub),
                        int(bool(skip_own)), _p(J), _p(A))
    return J, A


def cube_table(n_side, M=None):
    M = DEFAULT_CUBE_PER_NSIDE * n_side if M is None else M
    out = np.zeros(6 * M * M, np.int32)
    lib().or_cube_table(int(n_side), int(M), _p(out))
    return out


A_NCLASS, A_WIDTH = 15, 9


def alpha_table(n_side, M=None):
    """Tabulated angular kernel [6 M M, 15, 9] (pixels 0..3, counts 0..3 of 64, flag)."""
    M = DEFAULT_CUBE_PER_NSIDE * n_side if M is None else M
    pix = cube_table(n_side, M)
    out = np.zeros((6 * M * M, A_NCLASS, A_WIDTH), np.int32)
    lib().or_alpha_table(int(M), _p(pix), _p(out))
    return out


def integrate_ray(n_side, bins, flags, j_bg=0.0):
    bins = np.ascontiguousarray(bins, np.float64)
    flags = np.ascontiguousarray(flags, np.uint8)
    return lib().or_integrate_ray(int(n_side), bins.shape[0] - 1, _p(bins), _p(flags), float(j_bg))


def dust_eq(rho, u_rad, t_gas, sigma, c, c_gd, xi=1.0):
    rho = np.ascontiguousarray(rho, np.float64)
    u = np.ascontiguousarray(u_rad, np.float64)
    tg = np.ascontiguousarray(t_gas, np.float64)
    n = rho.shape[0]
    T = np.zeros(n)
    it = np.zeros(n, np.int32)
    lib().or_dust_eq(n, _p(rho), _p(u), _p(tg), float(sigma), float(c), float(c_gd), float(xi),
                     _p(T), _p(it))
    return T, it


def dust_residual(T, rho, u_rad, t_gas, sigma, c, c_gd, xi=1.0):
    return lib().or_dust_residual(float(T), float(rho), float(u_rad), float(t_gas), float(sigma),
                                  float(c), float(c_gd), float(xi))


def mlp_n_params(H):
    return 3 * H + H + H * H + H + H + 1


def mlp(H, params_, x, y=None, round_bf16=False, grad=True):
    prm = np.ascontiguousarray(params_, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    n = x.shape[0]
    yy = None if y is None else np.ascontiguousarray(y, np.float64)
    out = np.zeros(n)
    g = np.zeros(mlp_n_params(H)) if (grad and y is not None) else None
    loss = lib().or_mlp(int(H), _p(prm), n, _p(x), _p(yy), int(bool(round_bf16)), _p(out), _p(g))
    return loss, out, g


def dust_fixed_point(w, n_iter, c_gd=3.8e-33, xi=1.0, tol=0.0, prm=None):
    """Self-consistent dust temperature (Sec. 2, 4.1, 4.6): the dust temperature gives each
    cell its Planck-mean opacity and emission, the traced field gives the dust temperature
    through the equilibrium; repeated from w.t_dust for n_iter sweeps or until the largest
    relative change is <= tol.  The tree reads the temperature in single precision, as the
    cell arrays are stored.  Returns (T_dust, J, F, changes)."""
    import copy
    sigma, c = w.units
    prm = params(w.n_side, theta=w.theta) if prm is None else prm
    T = np.asarray(w.t_dust, np.float64)
    rho = np.asarray(w.rho, np.float64)
    tg = np.asarray(w.t_gas, np.float64)
    changes = []
    J = F = None
    for _ in range(n_iter):
        wk = copy.copy(w)
        wk.kappa = None
        wk.t_dust = T.astype(np.float32)
        tree = Tree(wk)
        J, F = tree.trace(prm)
        Tn, _ = dust_eq(rho, 4.0 * np.pi * J / c, tg, sigma, c, c_gd, xi)
        ch = float(np.max(np.abs(Tn - T) / Tn))
        changes.append(ch)
        T = Tn
        if ch <= tol:
            break
    return T, J, F, changes


T_LYC = 13.6 * 1.602176634e-12 / 1.380649e-16   # h nu_LyC / k_B in K (13.6 eV)


def lyman_fraction(T, t_lyc=T_LYC):
    """Fraction of a black body's power above the Lyman limit (Sec. 7.2)."""
    return lib().or_lyman_fraction(float(T), float(t_lyc))


def luminosity_split(L_int, L_acc, r_star, sigma, f_fill=0.1, t_lyc=T_LYC):
    """(L_uv, L_ir) of stars with internal and accretion luminosities (Sec. 7.2)."""
    a = [np.ascontiguousarray(v, np.float64) for v in (L_int, L_acc, r_star)]
    n = a[0].shape[0]
    uv, ir = np.zeros(n), np.zeros(n)
    lib().or_luminosity_split(n, _p(a[0]), _p(a[1]), _p(a[2]), float(f_fill), float(sigma), float(t_lyc),
                              _p(uv), _p(ir))
    return uv, ir


def uv_rad_pressure(rho, x_ion, nph, uph, e_ph, sigma_d=1.5e-21, sigma_h=6.3e-18, alpha_b=2.6e-13,
                    mu_mh=1.4 * 1.6735575e-24, c=2.99792458e10):
    """App. C: acceleration [n, 3] and momentum rates per volume on dust, H, H+ [n, 3]."""
    rho, x, N = (np.ascontiguousarray(v, np.float64) for v in (rho, x_ion, nph))
    u = np.ascontiguousarray(uph, np.float64).reshape(-1, 3)
    n = rho.shape[0]
    a = np.zeros((n, 3))
    parts = np.zeros((n, 3))
    lib().or_uv_rad_pressure(n, _p(rho), _p(x), _p(N), _p(u), float(e_ph), float(sigma_d), float(sigma_h),
                             float(alpha_b), float(mu_mh), float(c), _p(a), _p(parts))
    return a, parts
