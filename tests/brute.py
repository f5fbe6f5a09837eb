"""Independent brute-force helpers for the pins: written from geometry and textbook formulas,
sharing nothing with the oracle's C code or the GPU library."""
from __future__ import annotations

import numpy as np

H = 6.62607015e-27
CL = 2.99792458e10
KB = 1.380649e-16
SIGMA_SB = 2.0 * np.pi ** 5 * KB ** 4 / (15.0 * H ** 3 * CL ** 2)


def leaves(tree):
    """All leaves of a tree description: (canonical node id, level, lo[3], hi[3]) in root units.
    Canonical numbering recomputed from the description's convention."""
    counts = tree.level_counts()
    off = np.concatenate([[0], np.cumsum(counts)])
    nx, ny, nz = tree.nx, tree.ny, tree.nz
    ref_maps = [dict((int(v), o) for o, v in enumerate(r)) for r in tree.refined]
    out = []
    stack = []
    for iz in range(nz):
        for iy in range(ny):
            for ix in range(nx):
                stack.append((0, ix + nx * (iy + ny * iz), (ix, iy, iz)))
    while stack:
        lvl, li, I = stack.pop()
        h = 2.0 ** -lvl
        if lvl < len(tree.refined) and li in ref_maps[lvl]:
            o = ref_maps[lvl][li]
            for b in range(8):
                bits = (b & 1, (b >> 1) & 1, (b >> 2) & 1)
                stack.append((lvl + 1, 8 * o + b, tuple(2 * I[a] + bits[a] for a in range(3))))
        else:
            lo = np.array([I[a] * h for a in range(3)])
            out.append((int(off[lvl] + li), lvl, lo, lo + h))
    out.sort(key=lambda t: t[0])
    return out


def node_rho(tree):
    parts = [tree.root_rho] + list(tree.child_rho)
    return np.concatenate(parts)


def contains(lo, hi, p):
    return bool(np.all(p >= lo) and np.all(p < hi))


def clip_length(s, d, t_end, lo, hi):
    """Length of the part of segment s + t d, t in [0, t_end], inside the box [lo, hi]."""
    t0, t1 = 0.0, t_end
    for a in range(3):
        if d[a] == 0.0:
            if s[a] < lo[a] or s[a] > hi[a]:
                return 0.0, 0.0
            continue
        ta = (lo[a] - s[a]) / d[a]
        tb = (hi[a] - s[a]) / d[a]
        if ta > tb:
            ta, tb = tb, ta
        t0 = max(t0, ta)
        t1 = min(t1, tb)
    if t1 <= t0:
        return 0.0, 0.0
    return t1 - t0, t0


def box_exit(s, d, n):
    """Parameter t where the ray s + t d leaves the box [0, n)."""
    t = np.inf
    for a in range(3):
        if d[a] > 0:
            t = min(t, (n[a] - s[a]) / d[a])
        elif d[a] < 0:
            t = min(t, (0.0 - s[a]) / d[a])
    return t


def planck_nu(nu, t):
    x = H * nu / (KB * t)
    with np.errstate(over="ignore"):
        return (2.0 * H * nu ** 3 / CL ** 2) / np.expm1(x)


def trapezoid_dnu(lam_um):
    nu = CL / (np.asarray(lam_um) * 1e-4)
    if len(nu) == 1:
        return np.ones(1)
    d = np.empty_like(nu)
    d[0] = abs(nu[1] - nu[0]) / 2
    d[-1] = abs(nu[-1] - nu[-2]) / 2
    d[1:-1] = np.abs(nu[2:] - nu[:-2]) / 2
    return d


def hg_cdf(mu, g):
    """Closed-form cumulative distribution of the Henyey-Greenstein phase function in mu."""
    return (1.0 - g * g) / (2.0 * g) * ((1.0 + g * g - 2.0 * g * mu) ** -0.5 - 1.0 / (1.0 + g))


def philox_key(seed, iteration):
    return seed & 0xFFFFFFFF, ((seed >> 32) + iteration) & 0xFFFFFFFF


def stream_id(model, source, lam):
    return (model << 20) | (source << 12) | lam
