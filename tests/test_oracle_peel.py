"""Pins of the oracle's peel-off (paper Sect. 2.4): the phase function, the column to the model
border against brute-force segment-box clipping, the extinction tables against the marched
column, the single-scattering closed form with its angular dependence, the integral over all
observer directions against the escaping scattered energy, and the projection onto pixels."""
import math

import numpy as np
import pytest
from scipy import integrate

import gen
import oracle
from tests import brute


@pytest.mark.parametrize("g", [-0.5, 0.0, 0.3, 0.6, 0.9])
def test_hg_phase_normalised(g):
    """Per steradian: integral 1 over the sphere, mean cosine g."""
    f0 = integrate.quad(lambda mu: 2 * math.pi * oracle.hg_phase(g, mu), -1, 1, limit=200)[0]
    f1 = integrate.quad(lambda mu: 2 * math.pi * mu * oracle.hg_phase(g, mu), -1, 1, limit=200)[0]
    assert abs(f0 - 1.0) < 1e-9 and abs(f1 - g) < 1e-9


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def test_column_exact_against_brute_force():
    """Random refined tree, random points and directions (oblique and axis-aligned): the marched
    column equals the sum over leaves of density x clipped length of the ray to the border."""
    rng = np.random.default_rng(21)
    tree = gen.random_tree(rng, (3, 2, 4), 3, 0.4, rho_range=(0.1, 2.0))
    o = oracle.Model(tree)
    lv = brute.leaves(tree)
    rho = brute.node_rho(tree)
    dims = np.array([3.0, 2.0, 4.0])
    dirs = [_unit(rng.normal(size=3)) for _ in range(6)] + [np.array(v, float) for v in
                                                             ((1, 0, 0), (0, -1, 0), (0, 0, 1))]
    pts = rng.uniform(0.0, 1.0, (40, 3)) * dims
    for n in dirs:
        col = o.peel_column(n, pts)
        for p, c in zip(pts, col):
            t_end = brute.box_exit(p, n, dims)
            ref = sum(rho[nid] * brute.clip_length(p, n, t_end, lo, hi)[0] for nid, _, lo, hi in lv)
            assert abs(c - ref) <= 1e-12 * max(ref, 1.0), (n, p, c, ref)


def test_tables_exact_for_uniform_density_and_axis_directions():
    """Uniform density: along an axis every point of a face is the same distance from the
    border, so the table value of any tile is exact; the column is density x distance."""
    tree = gen.refined_block(2, rho=1.5)
    o = oracle.Model(tree)
    rng = np.random.default_rng(5)
    pts = rng.uniform(0.0, 4.0, (200, 3))
    dims = np.array([4.0, 4.0, 4.0])
    for n in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        n = np.array(n, dtype=np.float64)
        exact = o.peel_column(n, pts)
        ref = np.array([1.5 * brute.box_exit(p, n, dims) for p in pts])
        assert np.allclose(exact, ref, rtol=1e-13, atol=1e-13)
        for tiles in (1, 3):
            assert np.allclose(o.peel_column(n, pts, tiles=tiles), ref, rtol=1e-13, atol=1e-13)


def test_table_values_at_tile_centres():
    """A ray that leaves its refined root cell exactly through a tile centre gets the marched
    column from the tables too (uniform density, tiles 1, 2 and 5).  The direction leaves the
    model through a side face, so the column depends on where on the face the ray starts."""
    tree = gen.refined_block(2, rho=0.7)
    o = oracle.Model(tree)
    dims = np.array([4.0, 4.0, 4.0])
    n = _unit([0.8, 0.3, 0.52])
    for tiles in (1, 2, 5):
        pts = []
        for r in ((1, 1, 1), (2, 1, 2), (1, 2, 1)):
            for tx in range(tiles):
                for ty in range(tiles):
                    # exit through the +z face of root cell r at the centre of tile (tx, ty)
                    q = np.array([r[0] + (tx + 0.5) / tiles, r[1] + (ty + 0.5) / tiles, r[2] + 1.0])
                    pts.append(q - 0.05 * n)
        pts = np.array(pts)
        ref = np.array([0.7 * brute.box_exit(p, n, dims) for p in pts])
        assert np.allclose(o.peel_column(n, pts, tiles=tiles), ref, rtol=1e-12, atol=1e-12)


def test_table_error_shrinks_with_tile_count():
    """Oblique direction through a non-uniform refined tree: the tabled column approaches the
    marched one as the tiles get smaller."""
    rng = np.random.default_rng(9)
    tree = gen.random_tree(rng, (4, 4, 4), 3, 0.5, rho_range=(0.2, 2.0))
    o = oracle.Model(tree)
    pts = rng.uniform(0.0, 4.0, (400, 3))
    n = _unit([0.5, -0.3, 0.8])
    exact = o.peel_column(n, pts)
    err = [np.mean(np.abs(o.peel_column(n, pts, tiles=t) - exact)) for t in (1, 4, 16)]
    assert err[0] > 0 and err[1] < err[0] and err[2] < 0.25 * err[0], err


def _pure_scatterer_cube(kappa, n_lambda=1):
    """Two wavelengths with the same dust when n_lambda = 2 (their bandwidths differ)."""
    tree = gen.refined_block(2)
    lam = np.array([1.0, 2.0])[:n_lambda]
    dust = gen.Dust(lam, np.full(n_lambda, kappa), np.ones(n_lambda), np.full(n_lambda, 0.6))
    return tree, dust


@pytest.mark.parametrize("tiles", [0, 4])
def test_single_scattering_closed_form(tiles):
    """Optically thin pure scatterer (tau 0.02 along a beam through a 4^3 cube, g = 0.6): the
    peel-off energy per steradian toward n is, to first order in tau, N w0 times the integral
    along the beam of sigma exp(-sigma z) Phi(d.n) exp(-sigma l(z, n)).  Forward, backward and
    side views; a sign error in the phase-function cosine moves the forward/backward ratio by a
    factor of about 30."""
    kappa = 0.005
    tree, dust = _pure_scatterer_cube(kappa, n_lambda=2)
    o = oracle.Model(tree, dust)
    npk = 1_000_000
    x0, y0 = 2.35, 1.65
    src = [gen.Source(gen.SRC_BEAM, 0, pos=(x0, y0, 0.0), dir=(0.0, 0.0, 1.0),
                      power=np.array([1.0, 1.0]), packets=npk)]
    dirs = [_unit([0.6, 0.0, 0.8]), _unit([0.6, 0.0, -0.8]), np.array([1.0, 0.0, 0.0])]
    npix = 16
    _, _, st, _ = o.trace(src, seed=3, peel=dict(n_obs=dirs, npix=npix, width=8.0, tiles=tiles))
    img = st["peel_image"]
    dnu = brute.trapezoid_dnu(dust.lambda_um)
    pix_cm2 = (8.0 / npix) ** 2
    dims = np.array([4.0, 4.0, 4.0])
    for i in range(2):
        w0 = 1.0 * dnu[i] / npk  # beam power per Hz times the bandwidth, per packet
        for q, n in enumerate(dirs):
            got = img[q, i].sum() * pix_cm2 * dnu[i]
            phase = oracle.hg_phase(0.6, n[2])

            def f(z):
                p = np.array([x0, y0, z])
                return (kappa * math.exp(-kappa * z) * phase
                        * math.exp(-kappa * brute.box_exit(p, n, dims)))
            ref = npk * w0 * integrate.quad(f, 0.0, 4.0)[0]
            assert abs(got / ref - 1.0) < 0.05, (i, q, got, ref)


def test_peel_over_all_directions_equals_escaping_scattered_energy():
    """Scattering cube (tau ~ 1, albedo 0.7, g 0.5) in the isotropic field: the peel-off energy
    per steradian summed over 64 near-uniform directions times 4 pi / 64 estimates the energy
    that escapes after at least one scattering, which the records count directly."""
    tree = gen.refined_block(2)
    dust = gen.Dust(np.array([1.0]), np.array([0.25]), np.array([0.7]), np.array([0.5]))
    o = oracle.Model(tree, dust)
    npk = 60000
    src = [gen.Source(gen.SRC_BACKGROUND, 0, power=np.array([1.0]), packets=npk)]
    k = np.arange(64) + 0.5
    z = 1.0 - 2.0 * k / 64.0
    phi = math.pi * (1.0 + 5.0 ** 0.5) * k
    r = np.sqrt(1.0 - z * z)
    dirs = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    npix = 8
    pix_cm2 = (8.0 / npix) ** 2
    total = 0.0
    rec = None
    for q0 in range(0, 64, 16):
        _, _, st, rec = o.trace(src, seed=12, rec_stride=1,
                                peel=dict(n_obs=dirs[q0:q0 + 16], npix=npix, width=8.0))
        total += st["peel_image"].sum() * pix_cm2
    peeled = total * 4.0 * math.pi / 64.0
    escaped = rec["w"][(rec["status"] == 0) & (rec["events"] > 0)].sum()
    assert abs(peeled / escaped - 1.0) < 0.02, (peeled, escaped)


def test_pixel_projection():
    """A beam along z at (x0, y0) seen along +x lies in the image column of y0 (e1 = +y) and,
    seen along +y, in the column of -x0 (e1 = -x); every row along z is reached."""
    tree, dust = _pure_scatterer_cube(0.05)
    o = oracle.Model(tree, dust)
    x0, y0 = 2.35, 1.65
    src = [gen.Source(gen.SRC_BEAM, 0, pos=(x0, y0, 0.0), dir=(0.0, 0.0, 1.0),
                      power=np.array([1.0]), packets=50000)]
    npix = 40
    _, _, st, _ = o.trace(src, seed=4, max_events=1,
                          peel=dict(n_obs=[[1, 0, 0], [0, 1, 0]], npix=npix, width=4.0))
    img = st["peel_image"][:, 0]
    i_x = int(math.floor(((y0 - 2.0) / 4.0 + 0.5) * npix))
    i_y = int(math.floor((-(x0 - 2.0) / 4.0 + 0.5) * npix))
    for q, col in ((0, i_x), (1, i_y)):
        nz_cols = np.nonzero(img[q].sum(axis=0))[0]
        assert list(nz_cols) == [col], (q, nz_cols)
        assert np.count_nonzero(img[q][:, col]) == npix
