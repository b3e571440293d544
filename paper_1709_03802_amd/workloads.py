"""Seeded synthetic inputs for the DART-Ray ray-march hot path.

This module builds the *inputs* of a radiative-transfer run: the adaptive
Cartesian grid (root cubes plus octree leaves), the per-cell dust density and
stellar emissivity, the per-wavelength dust law and the ray policy.  It holds
none of the method's arithmetic (no ray tracing, no phase function, no
Eq. 5 resolution rule): both the FP64 oracle and the GPU library consume what
it produces, and neither depends on the other.

Units are code units with c = 1 (the paper fixes none).  Every generator is
deterministic for a given seed.

Workloads (the paper's grid and dust description is Sect. 2; the wavelength
range and the disk geometry stand in for its TRUST slab and Milky Way models,
which are not reproduced here):

* ``plain16``   uniform 16^3 unit cube, one wavelength, kappa*rho = 2,
                albedo 0.6, g 0.5, j = exp(-r/0.2), Nside 8 rays, Nside 2 for
                the scattered source function, direct + 2 scattering passes.
* ``disk``      30x30x6 kpc double-exponential galaxy disk on an octree of
                ~2e5 leaves, 8 wavelengths 0.15-2.2 um, adaptive ray density,
                cutoff f_U = 1e-3, step 1 + direct + 3 scattering passes.
* ``plain16_l32`` the plain16 geometry carrying 32 wavelengths.
* ``plain16_l4``  the plain16 geometry at 4 wavelengths (gradient workload).
* ``clumpy128`` uniform 128^3 lognormal medium, 16 wavelengths, 5000 star
                cells, direct + 4 scattering passes.
* ``disk_small`` a small disk octree used for parity tests of the adaptive
                path.
* ``selfheat``  a dusty 16^3 cube (tau_V = 30 centre to edge) lit by embedded
                stars in 4 bands, re-emitting in 8 infrared bands through a toy
                equilibrium grain (dust emission with self-heating).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

C_LIGHT = 1.0

# ---------------------------------------------------------------------------
# Data containers
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Grid:
    """An adaptive Cartesian grid: a block of root cubes, each an octree.

    A leaf is identified by ``level`` and integer coordinates ``ijk`` counted in
    cells of that level over the whole root block, so a leaf spans
    ``lo + ijk * root_size / 2**level`` to ``... + root_size / 2**level``.
    """

    nroot: tuple            # root cubes along x, y, z
    lo: tuple               # lower corner of the root block
    root_size: float        # edge of one root cube
    level: np.ndarray       # int32 [n]
    ijk: np.ndarray         # int64 [n, 3]
    rho: np.ndarray         # float64 [n]   dust density (times kappa_V)
    emis: np.ndarray        # float64 [nl, n] stellar volume emissivity j
    kappa: np.ndarray       # float64 [nl]  extinction per unit rho
    albedo: np.ndarray      # float64 [nl]
    g: np.ndarray           # float64 [nl]  Henyey-Greenstein anisotropy
    nside_sca: np.ndarray   # int32 [nl]   0 selects the Eq. 5 rule
    lambdas_um: np.ndarray  # float64 [nl]  informational
    n_fwhm: float = 5.0
    k_max: int = 2
    c_light: float = C_LIGHT
    # point sources (paper Sect. 3.6): positions [n_point, 3] inside the root
    # block and luminosities [nl, n_point]
    point_pos: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 3)))
    point_lum: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 0)))

    @property
    def n_point(self) -> int:
        return int(self.point_pos.shape[0])

    @property
    def n(self) -> int:
        return int(self.level.shape[0])

    @property
    def n_lambda(self) -> int:
        return int(self.kappa.shape[0])

    @property
    def max_level(self) -> int:
        return int(self.level.max()) if self.n else 0

    def side(self) -> np.ndarray:
        return self.root_size / (2.0 ** self.level.astype(np.float64))

    def centres(self) -> np.ndarray:
        s = self.side()
        return np.asarray(self.lo)[None, :] + (self.ijk.astype(np.float64) + 0.5) * s[:, None]

    def volume(self) -> np.ndarray:
        return self.side() ** 3

    def box(self):
        lo = np.asarray(self.lo, dtype=np.float64)
        return lo, lo + np.asarray(self.nroot, dtype=np.float64) * self.root_size

    def copy(self) -> "Grid":
        return dataclasses.replace(
            self, level=self.level.copy(), ijk=self.ijk.copy(), rho=self.rho.copy(),
            emis=self.emis.copy(), kappa=self.kappa.copy(), albedo=self.albedo.copy(),
            g=self.g.copy(), nside_sca=self.nside_sca.copy(), lambdas_um=self.lambdas_um.copy(),
            point_pos=self.point_pos.copy(), point_lum=self.point_lum.copy())


@dataclasses.dataclass
class RayPolicy:
    """How rays are cast (Sect. 3.1.1) and which passes run (Sect. 2)."""

    adaptive: bool = False
    nside: int = 8              # fixed mode: ray Nside; adaptive: initial Nside
    nside_max: int = 8          # adaptive: highest ray Nside
    n_rays_min: float = 4.0     # adaptive: N_rays of Eq. 2
    n_rays_max: float = 0.0     # adaptive: N_rays^max of Eq. 3 (ray merging, >= 4 n_rays_min); 0: no merging
    f_U: float = 0.0            # adaptive: blocking threshold of Eq. 1; < 0 selects Eq. 11
    a_RT: float = 0.0           # adaptive: accuracy parameter of Eq. 11 (f_U = 4 a_RT / N_s)
    r_pre: float = 0.0          # adaptive: step-1 extent
    step1: bool = False         # run step 1 (lower-limit RFED) first
    n_scatter: int = 2          # scattering iterations after the direct pass (the most run)
    f_L: float = 0.0            # stop once the pending scattered luminosity is below f_L
                                # times the total scattered in the direct pass (Sect. 2);
                                # 0 runs all n_scatter iterations
    mode_2d: bool = False       # 2D mode (Sect. 3.6): trace the first-octant sources of a
                                # mirror-symmetric grid, mirror their deposits


@dataclasses.dataclass
class Workload:
    name: str
    grid: Grid
    policy: RayPolicy
    description: str = ""


# ---------------------------------------------------------------------------
# Dust law and wavelength grids (stand-ins; the paper gives only ranges)
# ---------------------------------------------------------------------------


def dust_law(lambdas_um: np.ndarray):
    """kappa relative to V band, albedo and g on the 0.15-2.2 um range.

    kappa ~ lambda^-1.2; albedo rises 0.4 -> 0.6 and g falls 0.7 -> 0.4
    linearly in log(lambda) between 0.15 and 2.2 um.
    """
    lam = np.asarray(lambdas_um, dtype=np.float64)
    kappa = (lam / 0.55) ** (-1.2)
    t = np.log(lam / 0.15) / math.log(2.2 / 0.15)
    albedo = 0.4 + 0.2 * t
    g = 0.7 - 0.3 * t
    return kappa, albedo, g


def log_lambdas(n: int) -> np.ndarray:
    return np.exp(np.linspace(math.log(0.15), math.log(2.2), n))


DISK_LAMBDAS = np.array([0.150, 0.220, 0.300, 0.443, 0.550, 0.800, 1.250, 2.200])


# ---------------------------------------------------------------------------
# Grid builders
# ---------------------------------------------------------------------------


def uniform_leaves(n: tuple):
    """All level-0 cells of an nx*ny*nz block, x fastest."""
    nx, ny, nz = n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ijk = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.int64)
    level = np.zeros(ijk.shape[0], dtype=np.int32)
    return level, ijk


def _part1by2(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.uint64) & np.uint64(0x1FFFFF)
    x = (x | (x << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    x = (x | (x << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    x = (x | (x << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    x = (x | (x << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    x = (x | (x << np.uint64(2))) & np.uint64(0x1249249249249249)
    return x


def morton_order(level: np.ndarray, ijk: np.ndarray) -> np.ndarray:
    """Permutation that sorts leaves in Morton (octree depth-first) order."""
    if level.size == 0:
        return np.zeros(0, dtype=np.int64)
    lmax = int(level.max())
    shift = (lmax - level).astype(np.uint64)
    f = ijk.astype(np.uint64) << shift[:, None]
    key = _part1by2(f[:, 0]) | (_part1by2(f[:, 1]) << np.uint64(1)) | (_part1by2(f[:, 2]) << np.uint64(2))
    return np.argsort(key, kind="stable")


def refine_octree(nroot, lo, root_size, max_level, want_split, min_level=0):
    """Top-down refinement.  ``want_split(centre[n,3], side[n]) -> bool[n]``;
    cells above ``min_level`` are always split.

    Returns (level, ijk) of the leaves in Morton order.
    """
    lvl0, ijk0 = uniform_leaves(nroot)
    levels = []
    ijks = []
    cur_ijk = ijk0
    lo = np.asarray(lo, dtype=np.float64)
    for level in range(max_level + 1):
        side = root_size / 2.0 ** level
        centre = lo[None, :] + (cur_ijk.astype(np.float64) + 0.5) * side
        if level == max_level:
            split = np.zeros(cur_ijk.shape[0], dtype=bool)
        else:
            split = np.asarray(want_split(centre, np.full(cur_ijk.shape[0], side)), dtype=bool)
            if level < min_level:
                split[:] = True
        keep = ~split
        levels.append(np.full(int(keep.sum()), level, dtype=np.int32))
        ijks.append(cur_ijk[keep])
        parents = cur_ijk[split]
        if parents.shape[0] == 0:
            break
        off = np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], dtype=np.int64)
        cur_ijk = (2 * parents[:, None, :] + off[None, :, :]).reshape(-1, 3)
    level = np.concatenate(levels)
    ijk = np.concatenate(ijks, axis=0)
    order = morton_order(level, ijk)
    return level[order], ijk[order]


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------


def plain16(n_lambda: int = 1, n: int = 16, nside: int = 8, n_scatter: int = 2,
            lambdas: Optional[np.ndarray] = None) -> Workload:
    """Uniform n^3 unit cube, centre-to-edge tau = 1, j = exp(-r/0.2)."""
    level, ijk = uniform_leaves((n, n, n))
    size = 1.0 / n
    centre = (ijk + 0.5) * size
    r = np.linalg.norm(centre - 0.5, axis=1)
    rho = np.full(level.shape[0], 2.0)
    j = np.exp(-r / 0.2)
    if n_lambda == 1 and lambdas is None:
        kappa = np.array([1.0])
        albedo = np.array([0.6])
        g = np.array([0.5])
        lam = np.array([0.55])
    else:
        lam = log_lambdas(n_lambda) if lambdas is None else np.asarray(lambdas, dtype=np.float64)
        kappa, albedo, g = dust_law(lam)
    nl = kappa.shape[0]
    grid = Grid(nroot=(n, n, n), lo=(0.0, 0.0, 0.0), root_size=size, level=level, ijk=ijk,
                rho=rho, emis=np.repeat(j[None, :], nl, axis=0), kappa=kappa, albedo=albedo,
                g=g, nside_sca=np.full(nl, 2, dtype=np.int32), lambdas_um=lam)
    pol = RayPolicy(adaptive=False, nside=nside, nside_max=nside, n_scatter=n_scatter)
    return Workload(f"plain{n}_l{nl}", grid, pol,
                    f"uniform {n}^3 unit cube, kappa_V rho = 2, {nl} wavelength(s), Nside {nside} rays")


def disk_model(h_r=3.0, h_z=0.3, hd_r=4.5, hd_z=0.15, tau_v_faceon=1.0,
               nroot=(5, 5, 1), root_size=6.0, max_level=7, target_leaves=200_000,
               eps_lum=2e-5, lambdas=DISK_LAMBDAS, tol=0.05, tau_max=None, keep_best=False, peak=False,
               min_level=0):
    """Double-exponential stars + dust disk on an octree.

    A cell is split when its V-band optical depth across it exceeds tau_max or
    when its stellar luminosity exceeds eps_lum of the total; tau_max is
    bisected so that the leaf count lands within ``tol`` of ``target_leaves``
    (if it never does: the last build, or with ``keep_best`` the build whose
    count was closest to the target in ratio).  The split test takes the
    densities at the cell centre, or with ``peak`` at the cell's point nearest
    to the mid-plane and the axis (so that thin disks between two cell
    centres are still resolved).  ``min_level`` = 1 splits every root cube,
    so that no leaf lies across a plane through the block centre (the grid
    is then mirror symmetric leaf by leaf, as the 2D mode needs).
    """
    lo = tuple(-0.5 * np.asarray(nroot, dtype=np.float64) * root_size)
    kr0 = tau_v_faceon / (2.0 * hd_z)          # face-on central tau through the plane

    def stars(c):
        rr = np.hypot(c[:, 0], c[:, 1])
        return np.exp(-rr / h_r - np.abs(c[:, 2]) / h_z)

    def dust(c):
        rr = np.hypot(c[:, 0], c[:, 1])
        return kr0 * np.exp(-rr / hd_r - np.abs(c[:, 2]) / hd_z)

    l_tot = 4.0 * math.pi * 2.0 * math.pi * h_r ** 2 * 2.0 * h_z   # j0 = 1, infinite disk

    def nearest(c, s):
        if not peak:
            return c
        rr = np.hypot(c[:, 0], c[:, 1])
        shrink = np.maximum(rr - s / math.sqrt(2.0), 0.0) / np.maximum(rr, 1e-300)
        return np.stack([c[:, 0] * shrink, c[:, 1] * shrink,
                         np.sign(c[:, 2]) * np.maximum(np.abs(c[:, 2]) - 0.5 * s, 0.0)], axis=1)

    def build(tmax):
        def want(c, s):
            p = nearest(c, s)
            return (dust(p) * s > tmax) | (4.0 * math.pi * stars(p) * s ** 3 > eps_lum * l_tot)
        return refine_octree(nroot, lo, root_size, max_level, want, min_level=min_level)

    if tau_max is None:
        a, b = 1e-3, 10.0
        level, ijk = build(math.sqrt(a * b))
        best = None
        for _ in range(60):
            mid = math.sqrt(a * b)
            level, ijk = build(mid)
            n = level.shape[0]
            miss = abs(math.log(n / target_leaves))
            if best is None or miss < best[0]:
                best = (miss, mid, level, ijk)
            if abs(n - target_leaves) <= tol * target_leaves:
                tau_max = mid
                break
            if n > target_leaves:
                a = mid
            else:
                b = mid
        else:
            tau_max = math.sqrt(a * b)
            if keep_best:
                _, tau_max, level, ijk = best
    else:
        level, ijk = build(tau_max)

    side = root_size / 2.0 ** level
    centre = np.asarray(lo)[None, :] + (ijk + 0.5) * side[:, None]
    lam = np.asarray(lambdas, dtype=np.float64)
    kappa, albedo, g = dust_law(lam)
    nl = lam.shape[0]
    grid = Grid(nroot=tuple(nroot), lo=lo, root_size=root_size, level=level.astype(np.int32),
                ijk=ijk.astype(np.int64), rho=dust(centre), emis=np.repeat(stars(centre)[None, :], nl, axis=0),
                kappa=kappa, albedo=albedo, g=g, nside_sca=np.zeros(nl, dtype=np.int32),
                lambdas_um=lam, n_fwhm=5.0, k_max=2)
    return grid, tau_max


def disk(target_leaves=200_000, max_level=7, f_U=1e-3, n_scatter=3, nside0=4, nside_max=1024,
         tau_max=None, mode_2d=False) -> Workload:
    """The galaxy disk; ``mode_2d`` splits every root cube (no leaf across a
    plane through the centre) and runs the 2D mode."""
    grid, tmax = disk_model(target_leaves=target_leaves, max_level=max_level, tau_max=tau_max,
                            min_level=1 if mode_2d else 0)
    lo, hi = grid.box()
    r_pre = 0.15 * float(np.max(hi - lo))
    pol = RayPolicy(adaptive=True, nside=nside0, nside_max=nside_max, n_rays_min=4.0, f_U=f_U,
                    r_pre=r_pre, step1=True, n_scatter=n_scatter, mode_2d=mode_2d)
    return Workload("disk_2d" if mode_2d else "disk", grid, pol,
                    f"30x30x6 kpc double-exponential disk, {grid.n} octree leaves (tau_max={tmax:.4g}), "
                    f"{grid.n_lambda} wavelengths, adaptive rays Nside {nside0}..{nside_max}, f_U={f_U}")


def disk_small(target_leaves=3000, max_level=4, f_U=1e-3, nside_max=64, n_scatter=2) -> Workload:
    """A coarse disk octree for parity tests of the adaptive path."""
    grid, tmax = disk_model(target_leaves=target_leaves, max_level=max_level, eps_lum=1e-3, tol=0.25)
    lo, hi = grid.box()
    pol = RayPolicy(adaptive=True, nside=4, nside_max=nside_max, n_rays_min=4.0, f_U=f_U,
                    r_pre=0.15 * float(np.max(hi - lo)), step1=True, n_scatter=n_scatter)
    return Workload("disk_small", grid, pol, f"coarse disk octree, {grid.n} leaves")


def disk_tiny(target_leaves=600, max_level=3, f_U=1e-3, nside_max=32, n_scatter=2, mode_2d=False) -> Workload:
    """A very coarse disk octree (about 1000 leaves) for adaptive-path parity."""
    grid, tmax = disk_model(target_leaves=target_leaves, max_level=max_level, eps_lum=1e-3, tol=0.3,
                            min_level=1 if mode_2d else 0)
    lo, hi = grid.box()
    pol = RayPolicy(adaptive=True, nside=4, nside_max=nside_max, n_rays_min=4.0, f_U=f_U,
                    r_pre=0.15 * float(np.max(hi - lo)), step1=True, n_scatter=n_scatter, mode_2d=mode_2d)
    return Workload("disk_tiny", grid, pol, f"very coarse disk octree, {grid.n} leaves")


def gaussian_field(n: int, slope: float, seed: int) -> np.ndarray:
    """Periodic Gaussian random field with P(k) ~ k^slope, zero mean, unit variance."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    fk = np.fft.rfftn(white)
    kx = np.fft.fftfreq(n)[:, None, None]
    ky = np.fft.fftfreq(n)[None, :, None]
    kz = np.fft.rfftfreq(n)[None, None, :]
    k = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    amp = np.zeros_like(k)
    nz = k > 0
    amp[nz] = k[nz] ** (slope / 2.0)
    field = np.fft.irfftn(fk * amp, s=(n, n, n), axes=(0, 1, 2))
    field -= field.mean()
    field /= field.std()
    return field


def clumpy(n: int = 128, n_lambda: int = 16, n_stars: int = 5000, sigma_ln: float = 1.0,
           slope: float = -11.0 / 3.0, mean_tau: float = 2.0, field_seed: int = 5, star_seed: int = 6,
           nside: int = 8, n_scatter: int = 4) -> Workload:
    """Uniform n^3 unit cube with a lognormal density and point-like star cells."""
    level, ijk = uniform_leaves((n, n, n))
    gfield = gaussian_field(n, slope, field_seed)        # indexed [x, y, z]
    lnrho = sigma_ln * gfield - 0.5 * sigma_ln ** 2
    rho3 = np.exp(lnrho)
    rho3 *= 1.0 / rho3.mean()
    rho = rho3[ijk[:, 0], ijk[:, 1], ijk[:, 2]] * mean_tau      # kappa_V rho, mean tau across box
    rng = np.random.default_rng(star_seed)
    stars = rng.choice(n ** 3, size=min(n_stars, n ** 3), replace=False)
    vol = (1.0 / n) ** 3
    j = np.zeros(n ** 3)
    j[stars] = 1.0 / (4.0 * math.pi * vol * stars.shape[0])   # total luminosity 1 per wavelength
    lam = log_lambdas(n_lambda)
    kappa, albedo, g = dust_law(lam)
    grid = Grid(nroot=(n, n, n), lo=(0.0, 0.0, 0.0), root_size=1.0 / n, level=level, ijk=ijk,
                rho=rho, emis=np.repeat(j[None, :], n_lambda, axis=0), kappa=kappa, albedo=albedo,
                g=g, nside_sca=np.full(n_lambda, 2, dtype=np.int32), lambdas_um=lam)
    pol = RayPolicy(adaptive=False, nside=nside, nside_max=nside, n_scatter=n_scatter)
    return Workload(f"clumpy{n}", grid, pol,
                    f"uniform {n}^3 lognormal medium (sigma_ln {sigma_ln}, slope {slope:.3f}), "
                    f"{n_lambda} wavelengths, {stars.shape[0]} star cells")


def perturbed_rho(rho: np.ndarray, sigma: float = 0.3, seed: int = 3802) -> np.ndarray:
    """Target density for the gradient workload: rho * exp(sigma * N(0,1))."""
    rng = np.random.default_rng(seed)
    return rho * np.exp(sigma * rng.standard_normal(rho.shape[0]))


def random_octree(nroot=(2, 2, 2), root_size=0.5, max_level=3, p_split=0.4, seed=0,
                  n_lambda=1, lo=(0.0, 0.0, 0.0)) -> Grid:
    """A random octree with random density and emissivity (traversal tests)."""
    rng = np.random.default_rng(seed)

    def want(c, s):
        return rng.random(c.shape[0]) < p_split

    level, ijk = refine_octree(nroot, lo, root_size, max_level, want)
    n = level.shape[0]
    lam = log_lambdas(n_lambda) if n_lambda > 1 else np.array([0.55])
    if n_lambda > 1:
        kappa, albedo, g = dust_law(lam)
    else:
        kappa, albedo, g = np.array([1.0]), np.array([0.5]), np.array([0.4])
    return Grid(nroot=tuple(nroot), lo=tuple(lo), root_size=root_size, level=level, ijk=ijk,
                rho=rng.uniform(0.5, 3.0, n), emis=np.repeat(rng.uniform(0.1, 1.0, n)[None, :], n_lambda, axis=0),
                kappa=kappa, albedo=albedo, g=g, nside_sca=np.full(n_lambda, 2, dtype=np.int32),
                lambdas_um=lam)


def rotation(seed: int) -> np.ndarray:
    """A seeded proper rotation matrix (row-major 3x3), used to rotate ray frames."""
    rng = np.random.default_rng(seed)
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def disk_batch(n_models=16, leaves=(1e3, 1e5), seed=1709, nside=8, n_scatter=2, tol=0.25):
    """Independent disk models of uneven size for batched runs.

    Model m has seeded scale lengths, scale heights and face-on optical depth
    (stars h_R in [2, 4], h_z in [0.2, 0.4]; dust 1.5 h_R and h_z / 2 each
    scaled by [0.8, 1.2]; tau_V in [0.5, 2]) and a leaf-count target drawn
    log-uniformly in ``leaves``.  Returns a list of Workloads sharing one
    fixed-ray policy (Nside ``nside``, no cutoff, direct + n_scatter)."""
    rng = np.random.default_rng(seed)
    pol = RayPolicy(adaptive=False, nside=nside, nside_max=nside, n_scatter=n_scatter)
    out = []
    for m in range(n_models):
        target = float(np.exp(rng.uniform(np.log(leaves[0]), np.log(leaves[1]))))
        h_r = rng.uniform(2.0, 4.0)
        h_z = rng.uniform(0.2, 0.4)
        hd_r = 1.5 * h_r * rng.uniform(0.8, 1.2)
        hd_z = 0.5 * h_z * rng.uniform(0.8, 1.2)
        tau = rng.uniform(0.5, 2.0)
        max_level = int(np.clip(np.ceil(np.log(target / 25.0) / np.log(8.0)) + 2, 3, 7))
        grid, tmax = disk_model(h_r=h_r, h_z=h_z, hd_r=hd_r, hd_z=hd_z, tau_v_faceon=tau, max_level=max_level,
                                target_leaves=int(target), eps_lum=40.0 / target, tol=tol, keep_best=True,
                                peak=True)
        out.append(Workload(f"disk_batch{m}", grid, pol,
                            f"disk model {m}: {grid.n} leaves, h_R {h_r:.2f}, h_z {h_z:.2f}, tau_V {tau:.2f}"))
    return out


# ---------------------------------------------------------------------------
# Dust emission with self-heating (paper Sect. 3.3)
# ---------------------------------------------------------------------------

PLANCK_X0 = 14387.77            # h c / k in um K


@dataclasses.dataclass
class DustModel:
    """A toy equilibrium grain (the paper leaves the grain model to the user).

    Every wavelength of a grid stands for a band (U, j and luminosities are
    band-integrated).  A cell absorbs (1 - albedo) kappa rho V c U per band and
    re-emits the sum in the emission bands as 4 pi rho V kappa_i (1 - albedo_i)
    B(lambda_i, T) dlambda_i with B(lambda, T) = b0 lambda^-5 /
    (exp(x0 / (lambda T)) - 1), T set by that balance.
    """

    b0: float
    x0: float
    t_max: float
    lambdas_um: np.ndarray      # band centres of the emitting grid
    dlambda_um: np.ndarray      # band widths
    conv: float = 0.01          # stop once max dj / j_prev < conv (Sect. 3.3: 1%)
    max_iter: int = 20          # at most this many dust RT calculations


@dataclasses.dataclass
class DustWorkload:
    name: str
    stellar: Workload
    dust_grid: Grid             # same cells, emission bands, emission set by the loop
    dust_policy: RayPolicy
    dust: DustModel
    description: str = ""


IR_LAMBDAS = np.array([8.0, 12.0, 24.0, 35.0, 70.0, 100.0, 160.0, 350.0])


def ir_dust_law(lambdas_um: np.ndarray):
    """kappa relative to V, albedo and g in the infrared (toy): kappa ~
    (lambda / 0.55)^-1.4, albedo 0.05 falling as lambda^-1, g = 0.1."""
    lam = np.asarray(lambdas_um, dtype=np.float64)
    return (lam / 0.55) ** (-1.4), 0.05 * (8.0 / lam), np.full(lam.shape, 0.1)


def band_widths(lam: np.ndarray) -> np.ndarray:
    """Widths of log-centred bands: edges at geometric midpoints, the outer
    edges mirrored."""
    lam = np.asarray(lam, dtype=np.float64)
    if lam.size == 1:
        return 0.5 * lam                 # one band: half a decade-ish around its centre
    mid = np.sqrt(lam[1:] * lam[:-1])
    edges = np.concatenate([[lam[0] ** 2 / mid[0]], mid, [lam[-1] ** 2 / mid[-1]]])
    return np.diff(edges)


def selfheat(n: int = 16, tau_v: float = 30.0, b0: float = 5.8e10, nside: int = 4, n_scatter: int = 2,
             adaptive: bool = False, ir_lambdas=IR_LAMBDAS) -> DustWorkload:
    """A dusty cube lit by an embedded star cluster: uniform dust with
    centre-to-edge tau_V = tau_v, stars j ~ exp(-r / 0.15) in 4 bands
    (0.15-1 um), and the same cells emitting in 8 infrared bands (8-350 um)
    that the dust re-absorbs (tau ~ 1 at 8 um).  The default b0 puts a cell
    that absorbs the mean stellar luminosity per unit dust mass of the default
    cube near 25 K.
    """
    level, ijk = uniform_leaves((n, n, n))
    size = 1.0 / n
    centre = (ijk + 0.5) * size
    r = np.linalg.norm(centre - 0.5, axis=1)
    rho = np.full(level.shape[0], 2.0 * tau_v)
    lam_s = np.array([0.15, 0.3, 0.55, 1.0])
    k_s, a_s, g_s = dust_law(lam_s)
    emis = np.exp(-r / 0.15)[None, :] * np.array([1.0, 0.8, 0.6, 0.4])[:, None]
    star = Grid(nroot=(n, n, n), lo=(0.0, 0.0, 0.0), root_size=size, level=level, ijk=ijk, rho=rho,
                emis=emis, kappa=k_s, albedo=a_s, g=g_s, nside_sca=np.full(4, 2, dtype=np.int32), lambdas_um=lam_s)
    k_d, a_d, g_d = ir_dust_law(ir_lambdas)
    nl = len(ir_lambdas)
    dust_grid = Grid(nroot=(n, n, n), lo=(0.0, 0.0, 0.0), root_size=size, level=level.copy(), ijk=ijk.copy(),
                     rho=rho.copy(), emis=np.zeros((nl, level.shape[0])), kappa=k_d, albedo=a_d, g=g_d,
                     nside_sca=np.full(nl, 1, dtype=np.int32), lambdas_um=np.asarray(ir_lambdas, np.float64))
    dl = band_widths(ir_lambdas)
    lam = np.asarray(ir_lambdas, np.float64)
    dm = DustModel(b0=b0, x0=PLANCK_X0, t_max=1.0e4, lambdas_um=lam, dlambda_um=dl)
    if adaptive:
        pol_s = RayPolicy(adaptive=True, nside=2, nside_max=32, n_rays_min=4.0, f_U=1e-3, r_pre=0.25, step1=True,
                          n_scatter=n_scatter)
        pol_d = RayPolicy(adaptive=True, nside=2, nside_max=32, n_rays_min=4.0, f_U=1e-3, r_pre=0.25, step1=True,
                          n_scatter=n_scatter)
    else:
        pol_s = RayPolicy(adaptive=False, nside=nside, nside_max=nside, n_scatter=n_scatter)
        pol_d = RayPolicy(adaptive=False, nside=nside, nside_max=nside, n_scatter=n_scatter)
    return DustWorkload(f"selfheat{n}", Workload(f"selfheat{n}_stars", star, pol_s), dust_grid, pol_d, dm,
                        f"uniform {n}^3 cube, tau_V = {tau_v} centre to edge, embedded stars, 8 IR bands")


def by_name(name: str) -> Workload:
    if name == "plain16":
        return plain16()
    if name == "plain16_l32":
        return plain16(n_lambda=32)
    if name == "plain16_l4":
        return plain16(lambdas=np.array([0.15, 0.30, 0.55, 2.2]))
    if name == "disk":
        return disk()
    if name == "disk_small":
        return disk_small()
    if name == "disk_tiny":
        return disk_tiny()
    if name == "clumpy128":
        return clumpy()
    if name == "clumpy64_l4":
        return clumpy(n=64, n_lambda=4, n_stars=625, n_scatter=2)
    raise KeyError(name)
