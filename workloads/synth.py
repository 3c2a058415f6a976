"""Synthetic AMR clouds for the TreeRay/RadPressure hot path.

Every workload is a set of *leaf blocks* of 8^3 cells on a cubic domain of
``nb`` base blocks per side, refined up to ``max_level`` levels (PARAMESH-style
blocks, as on the FLASH grid the paper's octree is built over, Sec. 4.1).
Cell arrays are block-major in the order of ``blocks``; inside a block the cell
with local coordinates (ci, cj, ck) sits at offset ``ci + 8*cj + 64*ck``.

Only random numbers and their layout live here: Gaussian random fields,
lognormal densities, uniform/log-uniform draws and AMR block flags.  The
physics (opacity law, emission, tree, rays) lives on the two sides that are
compared, never here.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

# physical constants (cgs)
PC = 3.0856775814913673e18
MSUN = 1.98847e33
LSUN = 3.828e33
SIGMA_SB = 5.670374419e-5
C_LIGHT = 2.99792458e10
M_H = 1.6735575e-24

CODE_UNITS = (np.pi, 1.0)          # sigma = pi, c = 1  ->  sigma T^4 / pi = T^4
CGS_UNITS = (SIGMA_SB, C_LIGHT)

__all__ = [
    "Workload", "grf", "lognormal", "dense_to_blocks", "blocks_to_dense",
    "uniform_blocks", "c1_sphere16", "c2_turb64", "c3_core128", "c4_batch64",
    "c5_amr256", "small_uniform", "point_source_box", "isothermal_box",
    "thick_blob", "dust_samples", "PC", "MSUN", "LSUN", "SIGMA_SB", "C_LIGHT",
    "M_H", "CODE_UNITS", "CGS_UNITS", "CONFIGS",
]


@dataclasses.dataclass
class Workload:
    name: str
    nb: int                      # base blocks per side
    max_level: int               # refinement levels above the base grid
    blocks: np.ndarray           # int32 [n_blk, 4] = (level, bi, bj, bk), leaf blocks
    x0: tuple                    # domain origin
    box_len: float               # domain edge length
    rho: np.ndarray              # float32 [n_blk*512]
    t_dust: np.ndarray           # float32 [n_blk*512]
    kappa: Optional[np.ndarray]  # float32 [n_blk*512] or None (opacity from T_dust)
    stars: np.ndarray            # float64 [n_star, 4] = (x, y, z, L_IR)
    units: tuple                 # (sigma, c)
    n_side: int
    theta: tuple                 # opening angle as (num, den)
    t_gas: Optional[np.ndarray] = None   # float32 [n_blk*512] for the dust step
    j_bg: float = 0.0
    cgs: bool = False

    @property
    def n_cells(self) -> int:
        return int(self.blocks.shape[0]) * 512

    @property
    def n_pix(self) -> int:
        return 12 * self.n_side * self.n_side


# --------------------------------------------------------------------------
# random fields
# --------------------------------------------------------------------------
def grf(n: int, rng: np.random.Generator, slope: float = -4.0) -> np.ndarray:
    """Unit-variance Gaussian random field on an n^3 periodic grid with P(k) ~ k^slope.

    White noise -> FFT -> amplitude k^(slope/2) with the k=0 mode removed ->
    inverse FFT -> normalised to zero mean and unit variance.  Indexed [x, y, z].
    """
    noise = rng.standard_normal((n, n, n))
    fk = np.fft.rfftn(noise)
    kx = np.fft.fftfreq(n)[:, None, None]
    ky = np.fft.fftfreq(n)[None, :, None]
    kz = np.fft.rfftfreq(n)[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    amp = k2 ** (slope / 4.0)
    amp[0, 0, 0] = 0.0
    g = np.fft.irfftn(fk * amp, s=(n, n, n), axes=(0, 1, 2))
    g -= g.mean()
    g /= g.std()
    return g


def lognormal(g: np.ndarray, sigma: float) -> np.ndarray:
    """exp(sigma g - sigma^2/2): unit mean when g is a unit Gaussian."""
    return np.exp(sigma * g - 0.5 * sigma * sigma)


# --------------------------------------------------------------------------
# layout helpers
# --------------------------------------------------------------------------
def uniform_blocks(nb: int) -> np.ndarray:
    """All level-0 blocks of an nb^3 base grid, bi fastest."""
    bk, bj, bi = np.meshgrid(np.arange(nb), np.arange(nb), np.arange(nb), indexing="ij")
    out = np.zeros((nb ** 3, 4), np.int32)
    out[:, 1] = bi.ravel()
    out[:, 2] = bj.ravel()
    out[:, 3] = bk.ravel()
    return out


def dense_to_blocks(arr: np.ndarray, blocks: np.ndarray) -> np.ndarray:
    """Dense [x, y, z] level-0 array -> block-major cell array (uniform grids)."""
    out = np.empty(blocks.shape[0] * 512, dtype=arr.dtype)
    for b, (lev, bi, bj, bk) in enumerate(blocks):
        assert lev == 0
        sub = arr[bi * 8:(bi + 1) * 8, bj * 8:(bj + 1) * 8, bk * 8:(bk + 1) * 8]
        # local index ci + 8 cj + 64 ck  ->  transpose to [ck, cj, ci] then ravel
        out[b * 512:(b + 1) * 512] = np.transpose(sub, (2, 1, 0)).ravel()
    return out


def blocks_to_dense(cells: np.ndarray, blocks: np.ndarray, nb: int) -> np.ndarray:
    """Inverse of dense_to_blocks for uniform grids; trailing dims are kept."""
    tail = cells.shape[1:]
    n = nb * 8
    out = np.zeros((n, n, n) + tail, dtype=cells.dtype)
    for b, (lev, bi, bj, bk) in enumerate(blocks):
        sub = cells[b * 512:(b + 1) * 512].reshape((8, 8, 8) + tail)   # [ck, cj, ci]
        out[bi * 8:(bi + 1) * 8, bj * 8:(bj + 1) * 8, bk * 8:(bk + 1) * 8] = \
            np.transpose(sub, (2, 1, 0) + tuple(range(3, 3 + len(tail))))
    return out


def cell_centres(w: Workload) -> np.ndarray:
    """Cell centres [n_cells, 3] in the units of box_len (block-major order)."""
    dx0 = w.box_len / (w.nb * 8)
    ci = np.arange(512) % 8
    cj = (np.arange(512) // 8) % 8
    ck = np.arange(512) // 64
    out = np.empty((w.n_cells, 3))
    for b, (lev, bi, bj, bk) in enumerate(w.blocks):
        dx = dx0 / (1 << int(lev))
        out[b * 512:(b + 1) * 512, 0] = w.x0[0] + (bi * 8 + ci + 0.5) * dx
        out[b * 512:(b + 1) * 512, 1] = w.x0[1] + (bj * 8 + cj + 0.5) * dx
        out[b * 512:(b + 1) * 512, 2] = w.x0[2] + (bk * 8 + ck + 0.5) * dx
    return out


def cell_sizes(w: Workload) -> np.ndarray:
    dx0 = w.box_len / (w.nb * 8)
    return np.repeat(dx0 / (1 << w.blocks[:, 0].astype(np.int64)), 512)


def _uniform_workload(name, rho3, t3, kap3, nb, box_len, units, n_side, stars,
                      t_gas3=None, cgs=False, x0=(0.0, 0.0, 0.0)):
    blocks = uniform_blocks(nb)
    return Workload(
        name=name, nb=nb, max_level=0, blocks=blocks, x0=tuple(x0), box_len=float(box_len),
        rho=dense_to_blocks(rho3.astype(np.float32), blocks),
        t_dust=dense_to_blocks(t3.astype(np.float32), blocks),
        kappa=None if kap3 is None else dense_to_blocks(kap3.astype(np.float32), blocks),
        stars=np.asarray(stars, np.float64).reshape(-1, 4),
        units=units, n_side=n_side, theta=(1, 2 * n_side),
        t_gas=None if t_gas3 is None else dense_to_blocks(t_gas3.astype(np.float32), blocks),
        cgs=cgs)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def _centres_1d(n, box_len):
    return (np.arange(n) + 0.5) * (box_len / n)


def c1_sphere16(n: int = 16) -> Workload:
    """Uniform-density sphere (radius 0.4 of a unit box, rho 1 inside, 1e-3 outside),
    kappa = 1, T = 1 in code units (sigma = pi), no stars, 12 rays."""
    x = _centres_1d(n, 1.0)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    r = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2)
    rho = np.where(r < 0.4, 1.0, 1e-3)
    return _uniform_workload(f"sphere{n}", rho, np.ones_like(rho), np.ones_like(rho),
                             n // 8, 1.0, CODE_UNITS, 1, np.zeros((0, 4)))


def c2_turb64(n: int = 64, seed: int = 0, n_side: int = 2) -> Workload:
    """Lognormal turbulent density (sigma_ln = 1.5, k^-4 field), kappa log-uniform in
    [0.1, 10], T^4 uniform in [0.05, 0.2] (code units), one L = 1 star at the centre."""
    ss = np.random.SeedSequence(seed).spawn(4)
    g = grf(n, np.random.default_rng(ss[0]))
    rho = lognormal(g, 1.5)
    kap = 10.0 ** np.random.default_rng(ss[1]).uniform(-1.0, 1.0, rho.shape)
    t = np.random.default_rng(ss[2]).uniform(0.05, 0.2, rho.shape) ** 0.25
    stars = [[0.5, 0.5, 0.5, 1.0]]
    return _uniform_workload(f"turb{n}", rho, t, kap, n // 8, 1.0, CODE_UNITS, n_side, stars)


def c3_core128(n: int = 128, seed: int = 0, n_side: int = 4) -> Workload:
    """Collapsing core: rho ~ (max(r, 0.01 L)/L)^-2 times a sigma = 1 lognormal field,
    150 Msun in a (0.4 pc)^3 box, T_gas log-uniform in [10, 300] K, T_dust = T_gas,
    kappa from T_dust (cgs)."""
    ss = np.random.SeedSequence(seed).spawn(4)
    L = 0.4 * PC
    x = _centres_1d(n, L)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    r = np.sqrt((X - L / 2) ** 2 + (Y - L / 2) ** 2 + (Z - L / 2) ** 2)
    g = grf(n, np.random.default_rng(ss[0]))
    shape = (np.maximum(r, 0.01 * L) / L) ** -2.0 * lognormal(g, 1.0)
    dv = (L / n) ** 3
    rho = shape * (150.0 * MSUN / (shape.sum() * dv))
    t_gas = 10.0 ** np.random.default_rng(ss[1]).uniform(1.0, np.log10(300.0), rho.shape)
    w = _uniform_workload(f"core{n}", rho, t_gas, None, n // 8, L, CGS_UNITS, n_side,
                          np.zeros((0, 4)), t_gas3=t_gas, cgs=True)
    return w


def c4_batch64(n_inst: int = 64, seed: int = 0) -> List[Workload]:
    """64 uneven instances: edge uniform over {32, 40, ..., 96}, lognormal sigma = 1.5,
    kappa and T as in the turbulent box, 0-4 stars of L = 1, N_side 2 or 4."""
    root = np.random.SeedSequence(seed)
    kids = root.spawn(n_inst + 1)
    meta = np.random.default_rng(kids[0])
    edges = meta.choice(np.arange(32, 97, 8), size=n_inst)
    nsides = meta.choice([2, 4], size=n_inst)
    nstars = meta.integers(0, 5, size=n_inst)
    out = []
    for k in range(n_inst):
        ss = kids[k + 1].spawn(4)
        n = int(edges[k])
        g = grf(n, np.random.default_rng(ss[0]))
        rho = lognormal(g, 1.5)
        kap = 10.0 ** np.random.default_rng(ss[1]).uniform(-1.0, 1.0, rho.shape)
        t = np.random.default_rng(ss[2]).uniform(0.05, 0.2, rho.shape) ** 0.25
        pos = np.random.default_rng(ss[3]).uniform(0.0, 1.0, (int(nstars[k]), 3))
        stars = np.concatenate([pos, np.ones((pos.shape[0], 1))], axis=1)
        out.append(_uniform_workload(f"batch{k}_{n}", rho, t, kap, n // 8, 1.0, CODE_UNITS,
                                     int(nsides[k]), stars))
    return out


def _block_max(field: np.ndarray, lev: int, nb: int, fine: int) -> np.ndarray:
    """Max over each level-`lev` block of the field averaged to level-`lev` cells."""
    ncell = nb * 8 << lev
    f = fine // ncell
    avg = field.reshape(ncell, f, ncell, f, ncell, f).mean(axis=(1, 3, 5))
    nbl = nb << lev
    return avg.reshape(nbl, 8, nbl, 8, nbl, 8).max(axis=(1, 3, 5))


def _balance(flags: List[np.ndarray]) -> None:
    """2:1 balance: a block next to a block refined twice must itself be refined."""
    changed = True
    while changed:
        changed = False
        for lev in range(len(flags) - 1):
            # parent of every refined level-(lev+1) block, dilated by one block
            child = flags[lev + 1]
            n1 = child.shape[0]
            par = child.reshape(n1 // 2, 2, n1 // 2, 2, n1 // 2, 2).any(axis=(1, 3, 5))
            dil = par.copy()
            for ax in range(3):
                for s in (-1, 1):
                    sh = np.roll(par, s, axis=ax)
                    idx = [slice(None)] * 3
                    idx[ax] = 0 if s == 1 else -1
                    sh[tuple(idx)] = False
                    dil |= sh
            # those level-lev blocks must be refined, and only exist if their parent is
            need = dil & ~flags[lev]
            if lev > 0:
                n0 = flags[lev].shape[0]
                exists = np.repeat(np.repeat(np.repeat(flags[lev - 1], 2, 0), 2, 1), 2, 2)
                assert exists.shape[0] == n0
                need &= exists
            if need.any():
                flags[lev] |= need
                changed = True
            # propagate upwards: a refined block's parent must be refined
            for l2 in range(lev, 0, -1):
                n2 = flags[l2].shape[0]
                par2 = flags[l2].reshape(n2 // 2, 2, n2 // 2, 2, n2 // 2, 2).any(axis=(1, 3, 5))
                if (par2 & ~flags[l2 - 1]).any():
                    flags[l2 - 1] |= par2
                    changed = True


def _amr_blocks(field: np.ndarray, nb: int, levels: int, thr: List[float]):
    """Leaf blocks of a block-refined grid; thr[l] = refinement threshold at level l."""
    fine = field.shape[0]
    flags = []
    for lev in range(levels - 1):
        fl = _block_max(field, lev, nb, fine) > thr[lev]
        if lev > 0:
            fl &= np.repeat(np.repeat(np.repeat(flags[lev - 1], 2, 0), 2, 1), 2, 2)
        flags.append(fl)
    _balance(flags)
    leaves = []
    for lev in range(levels):
        nbl = nb << lev
        if lev == 0:
            exists = np.ones((nbl,) * 3, bool)
        else:
            exists = np.repeat(np.repeat(np.repeat(flags[lev - 1], 2, 0), 2, 1), 2, 2)
        leaf = exists & (~flags[lev] if lev < levels - 1 else True)
        bi, bj, bk = np.nonzero(leaf)
        for a, b, c in zip(bi, bj, bk):
            leaves.append((lev, a, b, c))
    return np.asarray(leaves, np.int32).reshape(-1, 4)


def _amr_cells(field: np.ndarray, blocks: np.ndarray, nb: int) -> np.ndarray:
    fine = field.shape[0]
    out = np.empty(blocks.shape[0] * 512)
    cache = {}
    for b, (lev, bi, bj, bk) in enumerate(blocks):
        if lev not in cache:
            ncell = nb * 8 << lev
            f = fine // ncell
            cache[lev] = field.reshape(ncell, f, ncell, f, ncell, f).mean(axis=(1, 3, 5))
        avg = cache[lev]
        sub = avg[bi * 8:(bi + 1) * 8, bj * 8:(bj + 1) * 8, bk * 8:(bk + 1) * 8]
        out[b * 512:(b + 1) * 512] = np.transpose(sub, (2, 1, 0)).ravel()
    return out


def c5_amr256(seed: int = 0, target_leaves: int = 2_500_000, fine: int = 256,
              nb: int = 8, n_star: int = 10, n_side: int = 4) -> Workload:
    """AMR cloud, 256^3-equivalent: 64^3 base grid of 8^3 blocks, refined twice where a
    block's maximum density exceeds 10x and 100x the mean (both thresholds scaled by one
    factor so that the leaf count is close to ``target_leaves``), 2:1 balanced.  Density
    from one lognormal (sigma_ln = 1.5, k^-4) field averaged to each level, box 1 pc,
    <rho> = 1e-20 g/cm^3, 10 stars with L log-uniform in [1, 1e4] Lsun, T_gas
    log-uniform in [10, 300] K, T_dust = T_gas, kappa from T_dust."""
    ss = np.random.SeedSequence(seed).spawn(4)
    levels = 3
    g = grf(fine, np.random.default_rng(ss[0]))
    field = lognormal(g, 1.5)            # unit mean
    lo, hi = 0.05, 50.0                  # bisect the threshold scale in log space
    best = None
    for _ in range(30):
        mid = np.sqrt(lo * hi)
        blocks = _amr_blocks(field, nb, levels, [10.0 * mid, 100.0 * mid])
        nleaf = blocks.shape[0] * 512
        if best is None or abs(nleaf - target_leaves) < abs(best[1] - target_leaves):
            best = (blocks, nleaf)
        if nleaf > target_leaves:
            lo = mid
        else:
            hi = mid
        if abs(nleaf - target_leaves) < 0.02 * target_leaves:
            break
    blocks = best[0]
    L = 1.0 * PC
    rho = (_amr_cells(field, blocks, nb) * 1e-20).astype(np.float32)
    n = blocks.shape[0] * 512
    t_gas = (10.0 ** np.random.default_rng(ss[1]).uniform(1.0, np.log10(300.0), n)).astype(np.float32)
    pos = np.random.default_rng(ss[2]).uniform(0.0, L, (n_star, 3))
    lum = 10.0 ** np.random.default_rng(ss[3]).uniform(0.0, 4.0, n_star) * LSUN
    stars = np.concatenate([pos, lum[:, None]], axis=1)
    return Workload(name="amr256", nb=nb, max_level=levels - 1, blocks=blocks,
                    x0=(0.0, 0.0, 0.0), box_len=L, rho=rho, t_dust=t_gas.copy(), kappa=None,
                    stars=stars, units=CGS_UNITS, n_side=n_side, theta=(1, 2 * n_side),
                    t_gas=t_gas, cgs=True)


# --------------------------------------------------------------------------
# small fixtures for the closed-form pins
# --------------------------------------------------------------------------
def small_uniform(n: int, rho: float, kappa: float, t: float, n_side: int = 1,
                  stars=None, box_len: float = 1.0, units=CODE_UNITS) -> Workload:
    shape = (n, n, n)
    return _uniform_workload(f"uniform{n}", np.full(shape, rho), np.full(shape, t),
                             np.full(shape, kappa), n // 8, box_len, units, n_side,
                             np.zeros((0, 4)) if stars is None else stars)


def point_source_box(n: int, kappa: float, n_side: int = 2, L: float = 1.0,
                     pos=None) -> Workload:
    """Dark (T = 0) homogeneous medium with one star: the Beer-Lambert x inverse-square
    set-up of the point-source test (Sec. 5.1), in code units."""
    pos = (0.5 + 0.25 / n, 0.5 + 0.25 / n, 0.5 + 0.25 / n) if pos is None else pos
    w = small_uniform(n, 1.0, kappa, 0.0, n_side, stars=[[pos[0], pos[1], pos[2], L]])
    return w


def isothermal_box(n: int, rho: float, kappa: float, t: float, n_side: int = 1) -> Workload:
    return small_uniform(n, rho, kappa, t, n_side)


def thick_blob(n: int, n_side: int, t_blob: float = 1.0, rho_blob: float = 1e3,
               kappa: float = 1.0, centre_cell=None) -> Workload:
    """A single optically thick 2x2x2-cell blob in an empty (rho = 0) box."""
    rho = np.zeros((n, n, n))
    t = np.zeros((n, n, n))
    c = (n // 2,) * 3 if centre_cell is None else centre_cell
    sl = tuple(slice(ci - 1, ci + 1) for ci in c)
    rho[sl] = rho_blob
    t[sl] = t_blob
    return _uniform_workload(f"blob{n}", rho, t, np.full(rho.shape, kappa), n // 8, 1.0,
                             CODE_UNITS, n_side, np.zeros((0, 4)))


def dust_samples(n: int, seed: int = 1, rho_range=(1e-24, 1e-14), u_range=(1e-16, 1e-6),
                 t_range=(5.0, 2000.0)) -> np.ndarray:
    """Log-uniform (rho, u_rad, T_gas) triples [n, 3] for the equilibrium solve and the
    MLP training set (cgs)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    out = np.empty((n, 3))
    for k, (a, b) in enumerate((rho_range, u_range, t_range)):
        out[:, k] = 10.0 ** rng.uniform(np.log10(a), np.log10(b), n)
    return out


CONFIGS = {
    "sphere16": c1_sphere16,
    "turb64": c2_turb64,
    "core128": c3_core128,
    "amr256": c5_amr256,
}
