"""Seeded synthetic inputs for the hierarchical-grid Monte Carlo radiative-transfer path.

This module builds *inputs only*: oct-tree descriptions (root grid + refined-cell lists +
child densities), dust tables (wavelength, extinction opacity, albedo, Henyey-Greenstein g)
and source descriptions (kind, position, spectrum, packet count).  It holds none of the
transport arithmetic; both the FP64 oracle and the GPU library consume exactly these arrays.

Tree description convention (shared input format, the paper's Sect. 2.1 hierarchy restated
for a refinement ratio of one half):

* level-0 cell index = ix + nx*(iy + ny*iz)
* the octs at level l+1 are ordered by the ascending level-l index of their parent cell;
  cell b = bx + 2*by + 4*bz of oct o has level index 8*o + b
* ``refined[l]`` lists, strictly ascending, the level-l indices of refined cells and
  ``child_rho[l]`` holds the 8*len(refined[l]) densities of the level-(l+1) cells in that order.

Workload shapes follow the paper's two tests (Sect. 4.1 molecular cloud, Sect. 4.2
circumstellar disc) with seeded stand-ins for the data the paper used but that are not
available (MHD snapshot, interstellar radiation field, dust model).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# cgs constants used to build input spectra (SI-exact definitions)
H_CGS = 6.62607015e-27
C_CGS = 2.99792458e10
K_CGS = 1.380649e-16
PC_CM = 3.0856775814913673e18
AU_CM = 1.495978707e13
RSUN_CM = 6.957e10

SRC_BACKGROUND = 0
SRC_POINT = 1
SRC_DUST = 2
SRC_BEAM = 3

BASE_SEED = 1206371000


@dataclass
class TreeDesc:
    nx: int
    ny: int
    nz: int
    root_cell_cm: float
    root_rho: np.ndarray                      # float64 [nx*ny*nz], x fastest
    refined: List[np.ndarray] = field(default_factory=list)    # per level: int64 ascending
    child_rho: List[np.ndarray] = field(default_factory=list)  # per level: float64 [8*n_ref]

    @property
    def n_levels(self) -> int:
        return len(self.refined)

    def level_counts(self) -> List[int]:
        c = [self.nx * self.ny * self.nz]
        for r in self.refined:
            c.append(8 * len(r))
        return c

    @property
    def n_nodes(self) -> int:
        return int(sum(self.level_counts()))

    @property
    def n_leaves(self) -> int:
        return self.n_nodes - int(sum(len(r) for r in self.refined))


@dataclass
class Dust:
    lambda_um: np.ndarray
    kappa_ext: np.ndarray    # cm^2 g^-1
    albedo: np.ndarray
    hg_g: np.ndarray

    @property
    def n_lambda(self) -> int:
        return int(len(self.lambda_um))


@dataclass
class Source:
    kind: int
    model: int = 0
    pos: tuple = (0.0, 0.0, 0.0)
    dir: tuple = (0.0, 0.0, 1.0)
    power: Optional[np.ndarray] = None   # [n_lambda]; None for dust emission
    packets: int = 0


@dataclass
class Workload:
    name: str
    trees: List[TreeDesc]
    dusts: List[Dust]
    sources: List[Source]
    seed: int
    rr_threshold: float = 0.0
    rr_prob: float = 0.0
    map_dirs: List[tuple] = field(default_factory=list)
    map_npix: int = 0
    meta: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------------------
# tree assembly helpers (input construction only)
# ----------------------------------------------------------------------------------------

def _root_index(ix, iy, iz, nx, ny):
    return ix + nx * (iy + ny * iz)


def top_fraction(values: np.ndarray, count: int) -> np.ndarray:
    """Indices of the ``count`` largest values, ties broken by lower index, returned ascending."""
    count = int(min(max(count, 0), len(values)))
    if count == 0:
        return np.zeros(0, dtype=np.int64)
    idx = np.arange(len(values), dtype=np.int64)
    order = np.lexsort((idx, -values))
    return np.sort(order[:count]).astype(np.int64)


def cascade_children(rng, parent_rho: np.ndarray, sigma: float) -> np.ndarray:
    """Mass-conserving multiplicative cascade: 8 children per parent, rho_c = rho_p e^{s eps}/<e^{s eps}>_8."""
    eps = rng.standard_normal((len(parent_rho), 8))
    f = np.exp(sigma * eps)
    f /= f.mean(axis=1, keepdims=True)
    return (parent_rho[:, None] * f).reshape(-1)


def gaussian_smoothed_field(rng, n: int, sigma_cells: float) -> np.ndarray:
    """Standardised periodic Gaussian-smoothed white noise on n^3, array order [z, y, x]."""
    noise = rng.standard_normal((n, n, n))
    k = 2.0 * np.pi * np.fft.fftfreq(n)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    filt = np.exp(-0.5 * (kx * kx + ky * ky + kz * kz) * sigma_cells * sigma_cells)
    g = np.fft.ifftn(np.fft.fftn(noise) * filt).real
    g -= g.mean()
    g /= g.std()
    return g


def power_law_field(rng, n: int, index: float):
    """Standardised Gaussian random field with P(k) ~ k^index on n^3 ([z, y, x]); also returns
    the fraction of its variance in the top octave (n/4 <= |k| < n/2 cycles per box)."""
    noise = rng.standard_normal((n, n, n))
    f = np.fft.fftfreq(n) * n
    kz, ky, kx = np.meshgrid(f, f, f, indexing="ij")
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    amp2 = np.zeros_like(kk)
    nz = kk > 0
    amp2[nz] = kk[nz] ** index
    g = np.fft.ifftn(np.fft.fftn(noise) * np.sqrt(amp2)).real
    g -= g.mean()
    g /= g.std()
    top = (kk >= n / 4.0) & (kk < n / 2.0)
    frac = float(amp2[top].sum() / amp2.sum())
    return g, frac


def shared_dust(n_lambda: int, kappa_v: float = 200.0) -> Dust:
    """Power-law dust: kappa ~ lambda^-1.8, albedo and g falling linearly in log lambda 0.6 -> 0."""
    lam = np.logspace(-1.0, 3.0, n_lambda)
    kap = kappa_v * (lam / 0.55) ** -1.8
    shape = np.clip(0.6 * (1.0 - np.log10(lam / 0.1) / 4.0), 0.0, 0.6)
    return Dust(lam, kap, shape.copy(), shape.copy())


def planck_nu_input(lam_um: np.ndarray, t: float) -> np.ndarray:
    """Blackbody B_nu(T) used only to build input spectra (background field, stellar luminosity)."""
    nu = C_CGS / (lam_um * 1e-4)
    x = H_CGS * nu / (K_CGS * t)
    with np.errstate(over="ignore"):
        return (2.0 * H_CGS * nu ** 3 / C_CGS ** 2) / np.expm1(x)


# Diluted-blackbody stand-in for an interstellar radiation field (W, T) pairs.
ISRF_COMPONENTS = ((1.0e-14, 7500.0), (1.0e-13, 4000.0), (4.0e-13, 3000.0))


def background_spectrum(lam_um: np.ndarray) -> np.ndarray:
    return sum(w * planck_nu_input(lam_um, t) for (w, t) in ISRF_COMPONENTS)


# ----------------------------------------------------------------------------------------
# C1: tiny two-level tree
# ----------------------------------------------------------------------------------------

def c1(variant: str = "A", seed: int = BASE_SEED + 1, n_root: int = 16, n_refine: int = 410,
       packets: int = 100_000) -> Workload:
    """Tiny two-level oct-tree (root 16^3 of side 1): log-normal density (sigma_ln 1) from
    periodic Gaussian-smoothed noise (3 root cells); the 410 densest root cells split once.

    variant 'A': children carry the fine-resolution values;
    variant 'B': the same cells split into 8 children of their parent's density;
    variant 'U': no refinement (root grid only, same root densities).
    Densities are scaled so the largest axis-aligned column optical depth through the cube,
    over level-1 column centres, is 10."""
    rng = np.random.default_rng(seed)
    nf = 2 * n_root
    g = gaussian_smoothed_field(rng, nf, 6.0)
    rho_f = np.exp(g - 0.5)                                    # [z, y, x] fine
    root = rho_f.reshape(n_root, 2, n_root, 2, n_root, 2).mean(axis=(1, 3, 5))
    root_flat = root.reshape(-1)
    refined = top_fraction(root_flat, n_refine)
    iz, iy, ix = np.unravel_index(refined, (n_root, n_root, n_root))
    ch = np.empty((len(refined), 8))
    for b in range(8):
        bx, by, bz = b & 1, (b >> 1) & 1, (b >> 2) & 1
        ch[:, b] = rho_f[2 * iz + bz, 2 * iy + by, 2 * ix + bx]
    # effective fine-resolution density of variant A for the tau normalisation
    is_ref = np.zeros(root_flat.shape, bool)
    is_ref[refined] = True
    ref3 = is_ref.reshape(root.shape).repeat(2, 0).repeat(2, 1).repeat(2, 2)
    eff = np.where(ref3, rho_f, root.repeat(2, 0).repeat(2, 1).repeat(2, 2))
    cell_cm = 1.0 / n_root
    kappa = 1.0
    h1 = cell_cm / 2.0
    tau_max = max(float((eff.sum(axis=a) * kappa * h1).max()) for a in range(3))
    s = 10.0 / tau_max
    root_flat = root_flat * s
    ch = ch * s
    if variant == "A":
        levels, kids = [refined], [ch.reshape(-1)]
    elif variant == "B":
        levels, kids = [refined], [np.repeat(root_flat[refined], 8)]
    elif variant == "U":
        levels, kids = [], []
    else:
        raise ValueError(variant)
    tree = TreeDesc(n_root, n_root, n_root, cell_cm, root_flat.copy(), levels, kids)
    dust = Dust(np.array([0.55]), np.array([kappa]), np.array([0.5]), np.array([0.6]))
    src = [Source(SRC_BACKGROUND, 0, power=np.array([1.0]), packets=packets)]
    return Workload(f"c1{variant}", [tree], [dust], src, seed,
                    meta={"tau_scale": s, "variant": variant})


# ----------------------------------------------------------------------------------------
# C2: molecular cloud
# ----------------------------------------------------------------------------------------

def c2(seed: int = BASE_SEED + 2, n_root: int = 64, max_level: int = 3, n_lambda: int = 32,
       packets: int = 10_000_000, sigma_ln: float = 1.5, spectral_index: float = -3.6,
       tau_split: float = 0.1, mean_tau_v: float = 1.0, size_pc: float = 2.0,
       kappa_v: float = 200.0, map_npix: int = 256) -> Workload:
    """Molecular-cloud stand-in (Sect. 4.1 shape): fBm (P(k) ~ k^-3.6) log-normal root field,
    refined top-down while the V-band cell optical depth exceeds 0.1 (at most 3 levels),
    children from a mass-conserving multiplicative cascade continuing the spectrum."""
    rng = np.random.default_rng(seed)
    g, top_frac = power_law_field(rng, n_root, spectral_index)
    rho = np.exp(sigma_ln * g - 0.5 * sigma_ln * sigma_ln).reshape(-1)
    cell_cm = size_pc * PC_CM / n_root
    rho *= mean_tau_v / (kappa_v * rho.mean() * n_root * cell_cm)
    var_top = sigma_ln * sigma_ln * top_frac
    tree = _refine_top_down(rng, n_root, n_root, n_root, cell_cm, rho, max_level,
                            lambda lvl, r: kappa_v * r * cell_cm * 2.0 ** -lvl > tau_split,
                            lambda lvl: np.sqrt(var_top * 2.0 ** (-0.6 * (lvl + 1))))
    dust = shared_dust(n_lambda, kappa_v)
    bg = background_spectrum(dust.lambda_um)
    src = [Source(SRC_BACKGROUND, 0, power=bg, packets=packets)]
    dirs = [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)]
    return Workload("c2", [tree], [dust], src, seed, rr_threshold=1e-3, rr_prob=0.9,
                    map_dirs=dirs, map_npix=map_npix,
                    meta={"top_octave_var": var_top, "size_pc": size_pc})


def _refine_top_down(rng, nx, ny, nz, cell_cm, root_rho, max_level, split_rule, sigma_of_level,
                     child_fn=None):
    refined, kids = [], []
    cur = root_rho
    for lvl in range(max_level):
        sel = np.nonzero(split_rule(lvl, cur))[0].astype(np.int64)
        if len(sel) == 0:
            break
        if child_fn is None:
            ch = cascade_children(rng, cur[sel], sigma_of_level(lvl))
        else:
            ch = child_fn(lvl, sel)
        refined.append(sel)
        kids.append(ch)
        cur = ch
    return TreeDesc(nx, ny, nz, cell_cm, root_rho.copy(), refined, kids)


# ----------------------------------------------------------------------------------------
# C3: circumstellar disc
# ----------------------------------------------------------------------------------------

def c3(seed: int = BASE_SEED + 3, root=(96, 96, 32), cell_au: float = 6.25, max_level: int = 6,
       tau_split: float = 2.5, n_lambda: int = 50, packets: int = 30_000_000,
       star_t: float = 4000.0, star_r_rsun: float = 2.0, kappa_v: float = 200.0,
       tau_mid_1um: float = 1.0e3, r_in_au: float = 0.1, r_out_au: float = 300.0,
       near_star_cells: float = 4.0) -> Workload:
    """Circumstellar-disc stand-in (Sect. 4.2 shape): rho = rho0 (r/r0)^-1 exp(-z^2/2h^2),
    h = h0 (r/r0)^1.125, r0 = 100 AU, h0 = 10 AU, point-sampled at cell centres, central star
    of 4000 K and 2 solar radii; refinement where the 1 um cell optical depth exceeds
    ``tau_split`` or near the star, up to ``max_level`` levels."""
    nx, ny, nz = root
    cell_cm = cell_au * AU_CM
    star = (nx / 2.0, ny / 2.0, nz / 2.0)
    dust = shared_dust(n_lambda, kappa_v)
    kappa_1 = kappa_v * (1.0 / 0.55) ** -1.8
    r0_cm = 100.0 * AU_CM
    rho0 = tau_mid_1um / (kappa_1 * r0_cm * np.log(r_out_au / r_in_au))

    def density(x, y, z):
        dx = (x - star[0]) * cell_au
        dy = (y - star[1]) * cell_au
        dz = (z - star[2]) * cell_au
        r = np.sqrt(dx * dx + dy * dy)
        rr = np.maximum(r, 1e-30)
        h = 10.0 * (rr / 100.0) ** 1.125
        val = rho0 * (rr / 100.0) ** -1.0 * np.exp(-0.5 * (dz / h) ** 2)
        return np.where((r >= r_in_au) & (r <= r_out_au), val, 0.0)

    # root cell centres
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cx = (ix.reshape(-1) + 0.5)
    cy = (iy.reshape(-1) + 0.5)
    cz = (iz.reshape(-1) + 0.5)
    rho = density(cx, cy, cz)
    root_rho = rho.copy()
    refined, kids = [], []
    for lvl in range(max_level):
        h = 2.0 ** -lvl
        dist = np.sqrt((cx - star[0]) ** 2 + (cy - star[1]) ** 2 + (cz - star[2]) ** 2)
        split = (kappa_1 * rho * h * cell_cm > tau_split) | (dist < near_star_cells * h)
        sel = np.nonzero(split)[0].astype(np.int64)
        if len(sel) == 0:
            break
        hc = h / 2.0
        b = np.arange(8)
        bx, by, bz = b & 1, (b >> 1) & 1, (b >> 2) & 1
        ncx = ((cx[sel] - 0.5 * h)[:, None] + (bx[None, :] + 0.5) * hc).reshape(-1)
        ncy = ((cy[sel] - 0.5 * h)[:, None] + (by[None, :] + 0.5) * hc).reshape(-1)
        ncz = ((cz[sel] - 0.5 * h)[:, None] + (bz[None, :] + 0.5) * hc).reshape(-1)
        crho = density(ncx, ncy, ncz)
        refined.append(sel)
        kids.append(crho)
        cx, cy, cz, rho = ncx, ncy, ncz, crho
    tree = TreeDesc(nx, ny, nz, cell_cm, root_rho, refined, kids)
    lstar = 4.0 * np.pi ** 2 * (star_r_rsun * RSUN_CM) ** 2 * planck_nu_input(dust.lambda_um, star_t)
    src = [Source(SRC_POINT, 0, pos=star, power=lstar, packets=packets)]
    return Workload("c3", [tree], [dust], src, seed, rr_threshold=1e-3, rr_prob=0.9,
                    meta={"rho0": rho0, "tau_split": tau_split, "star": star})


# ----------------------------------------------------------------------------------------
# C4: batched uneven clouds
# ----------------------------------------------------------------------------------------

def c4(seed: int = BASE_SEED + 4, n_models: int = 64, n_lambda: int = 16,
       packets: int = 1_000_000, sides=(16, 24, 32, 40, 48), levels=(1, 2, 3, 4),
       split_fraction: float = 0.1, tau_max: float = 10.0, size_pc: float = 1.0,
       kappa_v: float = 200.0, max_models: Optional[int] = None) -> Workload:
    """64 independent log-normal clouds (sigma_ln 1, Gaussian-smoothed over 3 root cells) with
    root side and level count drawn from each model's seed; the densest 10 % of each level's
    cells split (cascade children); max axis-aligned root-grid column tau = 10."""
    seqs = np.random.SeedSequence(seed).spawn(n_models)
    if max_models is not None:
        seqs = seqs[:max_models]
    trees, dusts, srcs = [], [], []
    dust = shared_dust(n_lambda, kappa_v)
    bg = background_spectrum(dust.lambda_um)
    for m, ss in enumerate(seqs):
        rng = np.random.default_rng(ss)
        n = int(rng.choice(sides))
        L = int(rng.choice(levels))
        g = gaussian_smoothed_field(rng, n, 3.0)
        rho3 = np.exp(g - 0.5)
        cell_cm = size_pc * PC_CM / n
        col = max(float((rho3.sum(axis=a)).max()) for a in range(3)) * kappa_v * cell_cm
        rho = (rho3 * (tau_max / col)).reshape(-1)
        sig = np.sqrt(0.25)

        tree = _refine_top_down(
            rng, n, n, n, cell_cm, rho, L,
            lambda lvl, r: np.isin(np.arange(len(r)), top_fraction(r, int(round(split_fraction * len(r))))),
            lambda lvl: sig * 2.0 ** (-0.3 * lvl))
        trees.append(tree)
        dusts.append(dust)
        srcs.append(Source(SRC_BACKGROUND, m, power=bg, packets=packets))
    return Workload("c4", trees, dusts, srcs, seed, rr_threshold=1e-3, rr_prob=0.9)


# ----------------------------------------------------------------------------------------
# C5: large deep-hierarchy cloud
# ----------------------------------------------------------------------------------------

def c5(seed: int = BASE_SEED + 5, n_root: int = 256, max_level: int = 5, n_lambda: int = 100,
       packets: int = 10_000_000, sigma_ln: float = 2.0, spectral_index: float = -3.6,
       mean_tau_v: float = 1.0, size_pc: float = 8.0, kappa_v: float = 200.0,
       n_cores: int = 64, core_rc=(1.0, 4.0), core_tau: float = 1.0e3,
       tau_split: float = 6.0, map_npix: int = 512) -> Workload:
    """Large deep-hierarchy cloud: root 256^3 fBm log-normal field (P(k) ~ k^-3.6,
    sigma_ln 2, mean V-band tau across the cube 1) plus 64 Plummer-like cores
    rho_c / (1 + r^2/r_c^2)^2 (r_c uniform in 1-4 root cells, seeded centres) whose central
    column tau_V = pi/2 kappa_V rho_c r_c is 1e3, point-sampled at root-cell centres; refined
    top-down while the V-band cell optical depth exceeds ``tau_split`` (at most 5 levels),
    children from the mass-conserving cascade.  The default ``tau_split`` gives 1.009e8 leaves
    (1.129e8 nodes) for the default seed (found with ``c5_tau_split_for``).  100 wavelengths, isotropic field,
    1e7 packets per wavelength, maps 512^2 toward the 8 body diagonals."""
    rng = np.random.default_rng(seed)
    g, top_frac = power_law_field(rng, n_root, spectral_index)
    rho = np.exp(sigma_ln * g - 0.5 * sigma_ln * sigma_ln)          # [z, y, x]
    cell_cm = size_pc * PC_CM / n_root
    rho *= mean_tau_v / (kappa_v * rho.mean() * n_root * cell_cm)
    cores = []
    ax = np.arange(n_root) + 0.5
    for _ in range(n_cores):
        c = rng.uniform(0.0, n_root, 3)
        rc = rng.uniform(core_rc[0], core_rc[1])
        rho_c = core_tau / (kappa_v * 0.5 * np.pi * rc * cell_cm)
        cores.append((c, rc, rho_c))
        h = int(np.ceil(12 * rc))
        lo = np.maximum(np.floor(c - h).astype(int), 0)
        hi = np.minimum(np.ceil(c + h).astype(int), n_root)
        dz = ax[lo[2]:hi[2], None, None] - c[2]
        dy = ax[None, lo[1]:hi[1], None] - c[1]
        dx = ax[None, None, lo[0]:hi[0]] - c[0]
        r2 = (dx * dx + dy * dy + dz * dz) / (rc * rc)
        rho[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += rho_c / (1.0 + r2) ** 2
    rho = rho.reshape(-1)
    var_top = sigma_ln * sigma_ln * top_frac
    tree = _refine_top_down(rng, n_root, n_root, n_root, cell_cm, rho, max_level,
                            lambda lvl, r: kappa_v * r * cell_cm * 2.0 ** -lvl > tau_split,
                            lambda lvl: np.sqrt(var_top * 2.0 ** (-0.6 * (lvl + 1))))
    dust = shared_dust(n_lambda, kappa_v)
    bg = background_spectrum(dust.lambda_um)
    src = [Source(SRC_BACKGROUND, 0, power=bg, packets=packets)]
    s3 = 1.0 / np.sqrt(3.0)
    dirs = [(sx * s3, sy * s3, sz * s3) for sx in (1, -1) for sy in (1, -1) for sz in (1, -1)]
    return Workload("c5", [tree], [dust], src, seed, rr_threshold=1e-3, rr_prob=0.9,
                    map_dirs=dirs, map_npix=map_npix,
                    meta={"cores": [(tuple(c), rc, rho_c) for c, rc, rho_c in cores],
                          "tau_split": tau_split, "size_pc": size_pc})


def c5_tau_split_for(leaves: float = 1.0e8, seed: int = BASE_SEED + 5, tol: float = 0.1,
                     **kw) -> float:
    """Bisection (in log tau_split) for the split threshold that gives ``leaves`` leaf cells
    within ``tol``; each probe builds the whole tree."""
    lo, hi = 0.1, 100.0
    for _ in range(40):
        mid = float(np.sqrt(lo * hi))
        n = c5(seed=seed, tau_split=mid, packets=1, **kw).trees[0].n_leaves
        if abs(n / leaves - 1.0) <= tol:
            return mid
        if n > leaves:
            lo = mid
        else:
            hi = mid
    return float(np.sqrt(lo * hi))


def random_tree(rng, root=(2, 2, 2), max_level=3, p_refine=0.35, cell_cm=1.0,
                rho_range=(0.0, 2.0), uniform_rho=None) -> TreeDesc:
    """Small random tree for brute-force checks: each cell refined with probability p_refine
    up to max_level levels; densities uniform in rho_range (or all equal to uniform_rho)."""
    nx, ny, nz = root
    n0 = nx * ny * nz

    def dens(k):
        if uniform_rho is not None:
            return np.full(k, float(uniform_rho))
        return rng.uniform(rho_range[0], rho_range[1], k)

    root_rho = dens(n0)
    refined, kids = [], []
    ncur = n0
    for lvl in range(max_level):
        sel = np.nonzero(rng.random(ncur) < p_refine)[0].astype(np.int64)
        if len(sel) == 0:
            break
        refined.append(sel)
        kids.append(dens(8 * len(sel)))
        ncur = 8 * len(sel)
    return TreeDesc(nx, ny, nz, cell_cm, root_rho, refined, kids)


def uniform_refined_tree(root=(2, 2, 2), level=2, rho=1.0, cell_cm=1.0) -> TreeDesc:
    """Every cell refined down to ``level``: all leaves are level-``level`` cells."""
    nx, ny, nz = root
    n = nx * ny * nz
    refined, kids = [], []
    for lvl in range(level):
        refined.append(np.arange(n, dtype=np.int64))
        n *= 8
        kids.append(np.full(n, float(rho)))
    return TreeDesc(nx, ny, nz, cell_cm, np.full(nx * ny * nz, float(rho)), refined, kids)


def refined_block(levels: int, n: int = 4, rho: float = 1.0) -> TreeDesc:
    """n^3 root cells of side 1, uniform density; the central 2^3 root cells (n = 4) or the
    root cells of index 1..n-2 on every axis are refined ``levels`` deep, the rest stay root
    leaves.  Packets crossing into the block enter a deeper leaf and leave it into a shallower
    one (the subgrid entries and exits of package splitting)."""
    inner = [i for i in range(1, n - 1)]
    centre = np.array([ix + n * (iy + n * iz) for iz in inner for iy in inner for ix in inner])
    refined, kids = [np.sort(centre).astype(np.int64)], []
    m = 8 * len(centre)
    for _ in range(1, levels):
        kids.append(np.full(m, float(rho)))
        refined.append(np.arange(m, dtype=np.int64))
        m *= 8
    kids.append(np.full(m, float(rho)))
    return TreeDesc(n, n, n, 1.0, np.full(n ** 3, float(rho)), refined, kids)


def thick_cube(n_root: int = 16, seed: int = BASE_SEED + 6, packets: int = 1_000_000) -> Workload:
    """Optically thick dust cube around a star, for the convergence of the Lambda iteration:
    root n_root^3 cells of 1 cm refined once everywhere, density 1 g cm^-3, 12 wavelengths
    1-1000 um with kappa = 30 (lambda / um)^-1.5 cm^2 g^-1 (a leaf is optically thick below
    about 10 um), albedo 0.1, isotropic scattering, and a 3000 K blackbody star of unit
    surface at the centre."""
    lam = np.logspace(0.0, 3.0, 12)
    dust = Dust(lam, 30.0 * lam ** -1.5, np.full(12, 0.1), np.zeros(12))
    tree = uniform_refined_tree((n_root, n_root, n_root), 1, rho=1.0, cell_cm=1.0)
    c = 0.5 * n_root
    star = [Source(SRC_POINT, 0, pos=(c + 0.05, c - 0.05, c + 0.02),
                   power=planck_nu_input(lam, 3000.0), packets=packets)]
    return Workload("thick_cube", [tree], [dust], star, seed, meta={"n_root": n_root})


def core_cloud(n_root: int = 15, levels: int = 3, seed: int = BASE_SEED + 7,
               packets: int = 100_000) -> Workload:
    """A thin cloud with one dense core, for subiterations: n_root^3 root cells of 1 cm (n_root
    odd) of density 0.02 g cm^-3; the central root cell is refined ``levels`` deep everywhere and
    its leaves take rho = 0.02 + 60 / (1 + r^2 / 0.12^2)^2 at their centres (r in cm from the
    cube centre); a 5000 K star of unit surface at the centre; 10 wavelengths 0.1-1000 um,
    kappa = 3 (lambda / 0.55 um)^-1.6, albedo and g falling from 0.5 as for the shared dust."""
    c = n_root // 2
    core = c + n_root * (c + n_root * c)
    refined, kids = [np.array([core], dtype=np.int64)], []
    centres = np.array([[c + 0.5, c + 0.5, c + 0.5]])
    for lvl in range(1, levels + 1):
        h = 2.0 ** -lvl
        b = np.arange(8)
        off = np.stack([b & 1, (b >> 1) & 1, (b >> 2) & 1], axis=1) - 0.5
        centres = (centres[:, None, :] + 0.5 * h * off[None, :, :] * 2.0).reshape(-1, 3)
        r2 = ((centres - (c + 0.5)) ** 2).sum(axis=1)
        rho = 0.02 + 60.0 / (1.0 + r2 / 0.12 ** 2) ** 2
        kids.append(rho)
        if lvl < levels:
            refined.append(np.arange(len(rho), dtype=np.int64))
    tree = TreeDesc(n_root, n_root, n_root, 1.0, np.full(n_root ** 3, 0.02), refined, kids)
    lam = np.logspace(-1.0, 3.0, 10)
    kap = 3.0 * (lam / 0.55) ** -1.6
    alb = np.clip(0.5 * (1.0 - np.log10(lam / 0.1) / 4.0), 0.0, 0.5)
    dust = Dust(lam, kap, alb, alb.copy())
    star = [Source(SRC_POINT, 0, pos=(c + 0.51, c + 0.49, c + 0.505),
                   power=planck_nu_input(lam, 5000.0), packets=packets)]
    return Workload("core_cloud", [tree], [dust], star, seed, rr_threshold=1e-3, rr_prob=0.9,
                    meta={"core_root_cell": int(core)})


def describe(w: Workload) -> dict:
    out = {"name": w.name, "models": len(w.trees)}
    out["nodes"] = int(sum(t.n_nodes for t in w.trees))
    out["leaves"] = int(sum(t.n_leaves for t in w.trees))
    out["levels"] = [t.n_levels for t in w.trees][:8]
    out["n_lambda"] = [d.n_lambda for d in w.dusts][:1]
    out["packets"] = int(sum(s.packets * w.dusts[s.model].n_lambda for s in w.sources))
    return out
