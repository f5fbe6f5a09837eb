"""Pins of the FP64 oracle against closed forms, invariants, special cases and brute force.

Each test names the part it pins.  The oracle follows the paper's Sects. 2.1, 2.3, 3.1, 4 and
4.1 and the tracking readings listed in its header; none of these tests re-implements the
oracle's arithmetic: they use geometry, closed forms and statistics."""
import math
import os

import numpy as np
import pytest

import gen
import oracle
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def model(tree, dust=None):
    if dust is None:
        dust = gen.Dust(np.array([1.0]), np.array([1.0]), np.array([0.0]), np.array([0.0]))
    return oracle.Model(tree, dust)


# ---------------------------------------------------------------------------------------
# random numbers
# ---------------------------------------------------------------------------------------

def test_philox_known_answers():
    """Philox4x32-10 against the published known-answer vectors (Salmon et al. SC'11)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = oracle.philox(v[4], v[5], v[0:4])[0]
        assert [int(x) for x in out] == v[6:10]


def test_uniform_mapping_exact_and_uniform():
    """U = (2 (x>>9) + 1) 2^-24: open interval, exactly representable in float32, uniform."""
    xs = np.array([0, 1, 511, 512, 0xFFFFFFFF, 0x80000000], dtype=np.uint64)
    u = np.array([oracle.lib().om_uniform(int(x)) for x in xs])
    assert u.min() > 0 and u.max() < 1
    assert np.all(u.astype(np.float32).astype(np.float64) == u)
    assert u[0] == 2.0 ** -24 and u[4] == 1.0 - 2.0 ** -24
    ctr = np.zeros((200000, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(200000)
    ctr[:, 1] = 7
    blocks = oracle.philox(123, 456, ctr)
    uu = oracle.uniform(blocks.reshape(-1))
    hist, _ = np.histogram(uu, bins=64, range=(0, 1))
    exp = len(uu) / 64
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < 120  # 63 dof, p ~ 1e-5
    assert abs(np.mean(-np.log(uu)) - 1.0) < 5.0 / math.sqrt(len(uu))


# ---------------------------------------------------------------------------------------
# tree and point location (Sect. 2.1)
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed,root,levels", [(1, (1, 1, 1), 3), (2, (2, 3, 1), 3),
                                              (3, (3, 2, 2), 2), (4, (2, 2, 2), 4)])
def test_locate_brute_force(seed, root, levels):
    """Canonical numbering and half-open location match a brute-force leaf enumeration."""
    rng = np.random.default_rng(seed)
    tree = gen.random_tree(rng, root, levels, 0.4)
    m = model(tree)
    lv = brute.leaves(tree)
    assert m.n_nodes == tree.n_nodes
    assert int((m.child < 0).sum()) == len(lv) == tree.n_leaves
    n = np.array(root, dtype=float)
    pts = [rng.uniform(0, 1, (3000, 3)) * n]
    # lattice points of the finest level: faces, edges and corners of leaves
    hmin = 2.0 ** -(tree.n_levels)
    lat = rng.integers(0, (n / hmin).astype(int) + 1, (3000, 3)) * hmin
    pts.append(lat)
    pts.append(np.array([[0, 0, 0], n, n - 1e-12, [n[0], 0, 0], [0.5, 0.5, -1e-300],
                         [np.nan, 0.1, 0.1], [np.nextafter(n[0], 0), 0, 0]], dtype=float))
    P = np.vstack(pts)
    lev, node = m.locate(P)
    for p, l, nd in zip(P, lev, node):
        inside = np.all(p >= 0) and np.all(p < n) and not np.any(np.isnan(p))
        if not inside:
            assert nd == -1 and l == -1
            continue
        hits = [(i, lvl) for (i, lvl, lo, hi) in lv if brute.contains(lo, hi, p)]
        assert len(hits) == 1
        assert (nd, l) == hits[0]


# ---------------------------------------------------------------------------------------
# traversal geometry
# ---------------------------------------------------------------------------------------

def beams(rng, n, count, absorber_dirs=None):
    srcs = []
    for _ in range(count):
        s = rng.uniform(0.05, 0.95, 3) * np.array(n)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        srcs.append(gen.Source(gen.SRC_BEAM, 0, pos=tuple(s), dir=tuple(d), power=np.array([1.0]),
                               packets=1))
    return srcs


def test_crossing_count_closed_form():
    """Straight rays through a uniformly refined level-l tree: leaf entries = 1 + the number of
    level-l faces crossed on each axis (generic directions)."""
    rng = np.random.default_rng(11)
    root, lvl = (2, 3, 2), 2
    tree = gen.uniform_refined_tree(root, lvl, rho=0.3)
    m = model(tree)
    srcs = beams(rng, root, 60)
    _, _, st, rec = m.trace(srcs, seed=5, rec_stride=1)
    for s, r in zip(srcs, rec):
        p0 = np.array(s.pos)
        d = np.array(s.dir) / np.linalg.norm(s.dir)
        t = brute.box_exit(p0, d, root)
        e = p0 + (t - 1e-9) * d
        expect = 1 + sum(abs(math.floor(e[a] * 2 ** lvl) - math.floor(p0[a] * 2 ** lvl))
                         for a in range(3))
        assert r["crossings"] == expect
        assert r["status"] == 0 and r["events"] == 0


def test_edge_exit_tie_goes_to_lowest_axis():
    """A ray hitting a cell edge where the x-neighbour is outside the root and the
    y-neighbour inside: ties go to the lowest axis, so the packet escapes at once."""
    tree = gen.TreeDesc(2, 3, 1, 1.0, np.full(6, 0.1), [], [])
    m = model(tree)
    d = np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0)
    src = [gen.Source(gen.SRC_BEAM, 0, pos=(1.5, 1.5, 0.5), dir=tuple(d), power=np.array([1.0]),
                      packets=1)]
    _, _, _, rec = m.trace(src, seed=1, rec_stride=1)
    assert rec[0]["crossings"] == 1 and rec[0]["status"] == 0


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_axis_rays_on_internal_faces(seed):
    """Axis-aligned rays lying exactly on internal faces and edges of a random tree: each cell
    is half-open, so the ray belongs to the cells above the face; escaped weight and per-cell
    deposits match brute-force clipping with half-open boxes."""
    rng = np.random.default_rng(seed)
    root = (2, 2, 2)
    tree = gen.random_tree(rng, root, 3, 0.5, cell_cm=1.0, rho_range=(0.0, 1.0))
    m = model(tree)
    lv = brute.leaves(tree)
    rho = brute.node_rho(tree)
    hmin = 2.0 ** -max(tree.n_levels, 1)
    for k in range(30):
        a = int(rng.integers(0, 3))
        sgn = 1.0 if rng.random() < 0.5 else -1.0
        p0 = rng.integers(1, int(2 / hmin), 3) * hmin
        p0[a] = 0.0 if sgn > 0 else 2.0 - 1e-9
        d = np.zeros(3)
        d[a] = sgn
        src = [gen.Source(gen.SRC_BEAM, 0, pos=tuple(p0), dir=tuple(d), power=np.array([1.0]),
                          packets=1)]
        e_abs, _, _, rec = m.trace(src, seed=3, rec_stride=1)
        tend = brute.box_exit(p0, d, root)
        segs = []
        for (nid, l, lo, hi) in lv:
            if any(not (lo[b] <= p0[b] < hi[b]) for b in range(3) if b != a):
                continue
            L, t0 = brute.clip_length(p0, d, tend, lo, hi)
            if L > 0:
                segs.append((t0, nid, L))
        segs.sort()
        w = 1.0
        dep = np.zeros(m.n_nodes)
        for (_, nid, L) in segs:
            tau = rho[nid] * L
            dep[nid] += w * (-math.expm1(-tau))
            w *= math.exp(-tau)
        assert rec[0]["w"] == pytest.approx(w, rel=1e-13, abs=1e-300)
        np.testing.assert_allclose(e_abs, dep, rtol=1e-12, atol=1e-300)


def test_path_lengths_brute_force():
    """Pure absorber on a random tree: escaped weight w0 exp(-sum sigma_c l_c) and per-cell
    deposits w_in (1 - exp(-sigma_c l_c)), with l_c from segment-box clipping of every leaf."""
    rng = np.random.default_rng(12)
    root = (3, 2, 2)
    tree = gen.random_tree(rng, root, 3, 0.4, cell_cm=0.7, rho_range=(0.0, 1.5))
    kappa = 1.3
    dust = gen.Dust(np.array([1.0]), np.array([kappa]), np.array([0.0]), np.array([0.0]))
    m = oracle.Model(tree, dust)
    lv = brute.leaves(tree)
    rho = brute.node_rho(tree)
    for k in range(25):
        src = beams(rng, root, 1)
        e_abs, _, st, rec = m.trace(src, seed=9, rec_stride=1)
        p0 = np.array(src[0].pos)
        d = np.array(src[0].dir) / np.linalg.norm(src[0].dir)
        tend = brute.box_exit(p0, d, root)
        segs = []
        for (nid, l, lo, hi) in lv:
            L, t0 = brute.clip_length(p0, d, tend, lo, hi)
            if L > 0:
                segs.append((t0, nid, L))
        segs.sort()
        w = 1.0
        dep = np.zeros(m.n_nodes)
        for (_, nid, L) in segs:
            tau = kappa * rho[nid] * tree.root_cell_cm * L
            dep[nid] += w * (-math.expm1(-tau))
            w *= math.exp(-tau)
        assert rec[0]["w"] == pytest.approx(w, rel=1e-12, abs=1e-300)
        np.testing.assert_allclose(e_abs, dep, rtol=1e-11, atol=1e-15)


def test_slab_attenuation_closed_form():
    """Beam through a uniform slab (density only in an x-range of cells, wide in y and z):
    w_out = w0 exp(-kappa rho L / |d_x|)."""
    rng = np.random.default_rng(13)
    root = (4, 64, 64)
    rho_root = np.zeros(root[0] * root[1] * root[2])
    ix = np.arange(len(rho_root)) % root[0]
    rho_root[(ix >= 1) & (ix < 3)] = 0.8
    tree = gen.TreeDesc(*root, 0.5, rho_root, [], [])
    kappa = 0.9
    m = oracle.Model(tree, gen.Dust(np.array([1.0]), np.array([kappa]), np.array([0.0]),
                                    np.array([0.0])))
    srcs = []
    for _ in range(40):
        d = np.array([1.0, rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3)])
        d /= np.linalg.norm(d)
        srcs.append(gen.Source(gen.SRC_BEAM, 0, pos=(0.5, 32.1, 31.7), dir=tuple(d),
                               power=np.array([1.0]), packets=1))
    _, _, _, rec = m.trace(srcs, seed=3, rec_stride=1)
    for s, r in zip(srcs, rec):
        d = np.array(s.dir)
        expect = math.exp(-kappa * 0.8 * 2.0 * 0.5 / d[0])
        assert r["w"] == pytest.approx(expect, rel=1e-14)


def test_point_in_uniform_cube_closed_form():
    """Isotropic point source at the centre of a uniform absorbing cube (refined once):
    w_out = w0 exp(-sigma min_a((N_a/2)/|d_a|)), directions recomputed from the Philox stream."""
    root = (4, 4, 4)
    tree = gen.uniform_refined_tree(root, 1, rho=0.6, cell_cm=0.25)
    kappa = 2.0
    m = oracle.Model(tree, gen.Dust(np.array([1.0]), np.array([kappa]), np.array([0.0]),
                                    np.array([0.0])))
    N = 500
    seed = 0x1234567890
    src = [gen.Source(gen.SRC_POINT, 0, pos=(2.0, 2.0, 2.0), power=np.array([1.0]), packets=N)]
    _, _, st, rec = m.trace(src, seed=seed, rec_stride=1)
    k0, k1 = brute.philox_key(seed, 0)
    ctr = np.zeros((N, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(N)
    ctr[:, 1] = brute.stream_id(0, 0, 0)
    b = oracle.philox(k0, k1, ctr)
    u0 = oracle.uniform(b[:, 0])
    u1 = oracle.uniform(b[:, 1])
    mu = 2 * u0 - 1
    st_ = np.sqrt(1 - mu * mu)
    d = np.stack([st_ * np.cos(2 * np.pi * u1), st_ * np.sin(2 * np.pi * u1), mu], axis=1)
    r = np.min(2.0 / np.abs(d), axis=1)
    expect = (1.0 / N) * np.exp(-kappa * 0.6 * 0.25 * r)
    np.testing.assert_allclose(rec["w"], expect, rtol=1e-12)


def test_background_injection_quadrature():
    """Uniform pure-absorber box (non-cubic) in an isotropic field: the mean absorbed fraction
    per packet equals a deterministic quadrature over the faces (weighted by area), entry points
    and Lambertian inward directions of 1 - exp(-sigma chord), within 3 sigma of the Monte
    Carlo estimate."""
    root = (5, 3, 2)
    sig = 0.25   # per root-cell unit
    tree = gen.TreeDesc(*root, 1.0, np.full(30, sig), [], [])
    m = oracle.Model(tree, gen.Dust(np.array([1.0]), np.array([1.0]), np.array([0.0]),
                                    np.array([0.0])))
    N = 200000
    _, _, st, rec = m.trace([gen.Source(gen.SRC_BACKGROUND, 0, power=np.array([1.0]),
                                        packets=N)], seed=77, rec_stride=1)
    w0 = st["e_emit"] / N
    f = 1.0 - rec["w"] / w0
    fmc, sd = f.mean(), f.std() / math.sqrt(N)
    n = 36
    g = (np.arange(n) + 0.5) / n
    tot, area = 0.0, 0.0
    dims = np.array(root, dtype=float)
    for a in range(3):
        t1, t2 = [b for b in range(3) if b != a]
        A = dims[t1] * dims[t2]
        x, y, u, ph = np.meshgrid(g * dims[t1], g * dims[t2], g, g * 2 * np.pi, indexing="ij")
        mu = np.sqrt(u)
        s_ = np.sqrt(1 - u)
        d1, d2 = s_ * np.cos(ph), s_ * np.sin(ph)

        def ex(pos, dd, L):
            with np.errstate(divide="ignore"):
                return np.where(dd > 0, (L - pos) / dd, np.where(dd < 0, -pos / dd, np.inf))
        chord = np.minimum(np.minimum(ex(x, d1, dims[t1]), ex(y, d2, dims[t2])), dims[a] / mu)
        tot += 2 * A * np.mean(1 - np.exp(-sig * chord))
        area += 2 * A
    fq = tot / area
    assert abs(fmc - fq) < 3 * sd + 2e-4, (fmc, fq, sd)
    # entry points uniform over the surface: a root cell is born into with probability
    # (number of box faces it lies on) / (total surface in cell units)
    idx = np.arange(30)
    I = np.stack([idx % 5, (idx // 5) % 3, idx // 15], axis=1)
    nf = sum(((I[:, a] == 0).astype(int) + (I[:, a] == root[a] - 1)) for a in range(3))
    p = nf / area
    cnt = np.bincount(rec["birth"], minlength=30)
    sel = p > 0
    chi2 = (((cnt[sel] - N * p[sel]) ** 2) / (N * p[sel])).sum()
    dof = sel.sum() - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof), chi2
    assert np.all(cnt[~sel] == 0)


# ---------------------------------------------------------------------------------------
# energy bookkeeping and free paths
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("rr", [(0.0, 0.0), (0.2, 0.5)])
def test_energy_conservation(rr):
    """Emitted = absorbed + escaped + killed + truncated - roulette gain."""
    w = gen.c1("A", packets=20000)
    m = oracle.Model(w.trees[0], w.dusts[0])
    _, _, st, _ = m.trace(w.sources, seed=w.seed, rr_threshold=rr[0], rr_prob=rr[1],
                          max_events=40)
    rhs = st["e_abs"] + st["e_esc"] + st["e_killed"] + st["e_trunc"] - st["e_rr_gain"]
    assert rhs == pytest.approx(st["e_emit"], rel=1e-11)
    if rr[1] > 0:
        assert st["kills"] > 0 and st["e_rr_gain"] > 0


def test_pure_scatterer_and_free_path_in_scattering_depth():
    """Albedo 1: nothing absorbed, everything escapes.  Albedo 0.5: the fraction of beam packets
    leaving a slab unscattered is exp(-a tau_ext) (free paths drawn in scattering optical depth)
    and their weight is w0 exp(-(1-a) tau_ext)."""
    w = gen.c1("A", packets=20000)
    d1 = gen.Dust(np.array([0.55]), np.array([1.0]), np.array([1.0]), np.array([0.3]))
    m = oracle.Model(w.trees[0], d1)
    e_abs, e_esc, st, _ = m.trace(w.sources, seed=w.seed)
    assert st["e_abs"] == 0.0 and np.all(e_abs == 0.0)
    assert st["e_esc"] == pytest.approx(st["e_emit"], rel=1e-13)
    root = (2, 64, 64)
    tree = gen.TreeDesc(*root, 1.0, np.full(2 * 64 * 64, 0.5), [], [])
    a = 0.5
    m2 = oracle.Model(tree, gen.Dust(np.array([1.0]), np.array([2.0]), np.array([a]),
                                     np.array([0.0])))
    N = 40000
    _, _, st2, rec = m2.trace([gen.Source(gen.SRC_BEAM, 0, pos=(1.0, 32.0, 32.0),
                                          dir=(1.0, 0.0, 0.0), power=np.array([1.0]), packets=N)],
                              seed=21, rec_stride=1)
    tau_ext = 2.0 * 0.5 * 1.0
    p = math.exp(-a * tau_ext)
    frac = float(np.mean(rec["events"] == 0))
    assert abs(frac - p) < 4 * math.sqrt(p * (1 - p) / N)
    un = rec[rec["events"] == 0]
    np.testing.assert_allclose(un["w"], math.exp(-(1 - a) * tau_ext) / N, rtol=1e-14)


def test_henyey_greenstein_sampling():
    """Inverse-CDF sampling against the closed-form HG distribution: F(mu(u)) = u and the
    Legendre moments <mu> = g, <P2(mu)> = g^2."""
    for g in (0.6, -0.3, 0.05, 0.9):
        us = (np.arange(20000) + 0.5) / 20000
        mus = np.array([oracle.hg_mu(g, u) for u in us])
        np.testing.assert_allclose(brute.hg_cdf(mus, g), us, atol=1e-11)
        assert mus.mean() == pytest.approx(g, abs=2e-4)
        assert (1.5 * mus ** 2 - 0.5).mean() == pytest.approx(g * g, abs=5e-4)
    mus = np.array([oracle.hg_mu(0.0, u) for u in us])
    np.testing.assert_allclose(mus, 2 * us - 1, atol=1e-15)


def test_rotation_geometry():
    """The turned direction makes angle acos(mu) with the old one, is a unit vector, and for
    d = z equals (sin t cos p, sin t sin p, mu)."""
    rng = np.random.default_rng(5)
    for _ in range(300):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        mu, phi = rng.uniform(-1, 1), rng.uniform(0, 2 * np.pi)
        dn = oracle.rotate(d, mu, phi)
        assert np.linalg.norm(dn) == pytest.approx(1.0, abs=1e-14)
        assert float(dn @ d) == pytest.approx(mu, abs=1e-12)
    dn = oracle.rotate([0, 0, 1.0], 0.3, 1.1)
    st = math.sqrt(1 - 0.09)
    np.testing.assert_allclose(dn, [st * math.cos(1.1), st * math.sin(1.1), 0.3], atol=1e-14)


# ---------------------------------------------------------------------------------------
# invariants of the hierarchy
# ---------------------------------------------------------------------------------------

def test_split_invariance():
    """Splitting cells into 8 equal-density children leaves every packet's history unchanged
    (weight, events, fate) and the children's absorbed energy sums to the parent's."""
    wu = gen.c1("U", packets=20000)
    wb = gen.c1("B", packets=20000)
    mu_ = oracle.Model(wu.trees[0], wu.dusts[0])
    mb = oracle.Model(wb.trees[0], wb.dusts[0])
    eu, escu, su, ru = mu_.trace(wu.sources, seed=wu.seed, rec_stride=1)
    eb, escb, sb, rb = mb.trace(wb.sources, seed=wb.seed, rec_stride=1)
    assert np.array_equal(ru["events"], rb["events"])
    assert np.array_equal(ru["status"], rb["status"])
    np.testing.assert_allclose(rb["w"], ru["w"], rtol=1e-11)
    assert sb["crossings"] > su["crossings"]
    ref = wb.trees[0].refined[0]
    child_sum = eb[4096:].reshape(-1, 8).sum(axis=1)
    np.testing.assert_allclose(child_sum, eu[ref], rtol=1e-10)
    unref = np.setdiff1d(np.arange(4096), ref)
    np.testing.assert_allclose(eb[unref], eu[unref], rtol=1e-10, atol=1e-300)


def test_linearity_and_packet_ranges():
    """Doubling the source power doubles every deposit exactly; the packet-id range [0, N)
    equals the sum of [0, N/2) and [N/2, N)."""
    w = gen.c1("A", packets=10000)
    m = oracle.Model(w.trees[0], w.dusts[0])
    e1, s1, _, _ = m.trace(w.sources, seed=w.seed, rr_threshold=0.05, rr_prob=0.5)
    w2 = [gen.Source(gen.SRC_BACKGROUND, 0, power=np.array([2.0]), packets=10000)]
    e2, s2, _, _ = m.trace(w2, seed=w.seed, rr_threshold=0.05, rr_prob=0.5)
    assert np.array_equal(e2, 2 * e1)
    assert np.array_equal(s2, 2 * s1)
    ea, _, _, _ = m.trace(w.sources, seed=w.seed, pid_begin=0, pid_end=5000)
    eb, _, _, _ = m.trace(w.sources, seed=w.seed, pid_begin=5000, pid_end=10000)
    ef, _, _, _ = m.trace(w.sources, seed=w.seed)
    np.testing.assert_allclose(ea + eb, ef, rtol=1e-12, atol=1e-300)


# ---------------------------------------------------------------------------------------
# temperatures (Sect. 4: one dust component at equilibrium)
# ---------------------------------------------------------------------------------------

def test_temperature_grey_closed_form():
    """Constant kappa_abs on a fine frequency grid: T = (A / (4 m kappa sigma_SB))^(1/4)."""
    lam = np.logspace(np.log10(0.02), np.log10(3e5), 6000)
    kap = np.full(len(lam), 3.0)
    tree = gen.TreeDesc(1, 1, 1, 2.0, np.array([0.7]), [], [])
    m = oracle.Model(tree, gen.Dust(lam, kap, np.zeros(len(lam)), np.zeros(len(lam))))
    mass = 0.7 * 8.0
    for T in (8.0, 20.0, 90.0, 400.0, 1800.0):
        A = 4.0 * mass * 3.0 * brute.SIGMA_SB * T ** 4
        t = m.solve_temperature(np.array([A]), 2.0, 3000.0)[0]
        assert t == pytest.approx(T, rel=2e-6)


def test_temperature_inverts_emission_and_clamps():
    """For any kappa(nu), A = 4 pi m sum kappa_abs B(T_rad) dnu gives back T_rad; A outside the
    bracket clamps to its ends; refined cells carry no temperature."""
    rng = np.random.default_rng(3)
    dust = gen.shared_dust(24)
    tree = gen.random_tree(rng, (2, 2, 1), 2, 0.5, cell_cm=1e15, rho_range=(1e-22, 1e-20))
    m = oracle.Model(tree, dust)
    lv = m.level_of_nodes()
    rho = brute.node_rho(tree)
    mass = rho * (tree.root_cell_cm * 2.0 ** -lv) ** 3
    nu = brute.CL / (dust.lambda_um * 1e-4)
    dnu = brute.trapezoid_dnu(dust.lambda_um)
    kabs = (1 - dust.albedo) * dust.kappa_ext
    trad = rng.uniform(5, 2000, m.n_nodes)
    A = np.array([4 * np.pi * mass[i] * np.sum(kabs * brute.planck_nu(nu, trad[i]) * dnu)
                  for i in range(m.n_nodes)])
    A[0] = 0.0
    A[1] = 1e300
    t = m.solve_temperature(A, 2.0, 3000.0)
    leaf = m.leaf_mask
    idx = np.nonzero(leaf)[0]
    idx = idx[idx > 1]
    np.testing.assert_allclose(t[idx], trad[idx], rtol=1e-10)
    if leaf[0]:
        assert t[0] == 2.0
    if leaf[1]:
        assert t[1] == 3000.0
    assert np.all(t[~leaf] == 0.0)


def test_thin_cloud_reaches_background_temperature():
    """Optically thin cube in an isotropic blackbody field B(T_bg): every cell absorbs
    4 pi m sum kappa B(T_bg) dnu (mean-chord theorem), so its temperature is T_bg."""
    tbg = 25.0
    lam = np.logspace(np.log10(5.0), np.log10(3000.0), 40)
    kap = 50.0 * (lam / 100.0) ** -1.5
    dust = gen.Dust(lam, kap, np.zeros(40), np.zeros(40))
    tree = gen.TreeDesc(2, 2, 2, 1.0, np.full(8, 2e-6), [], [])
    m = oracle.Model(tree, dust)
    nu = brute.CL / (lam * 1e-4)
    src = [gen.Source(gen.SRC_BACKGROUND, 0, power=brute.planck_nu(nu, tbg), packets=20000)]
    e, _, _, _ = m.trace(src, seed=8)
    t = m.solve_temperature(e, 2.0, 3000.0)
    np.testing.assert_allclose(t, tbg, rtol=5e-3)


# ---------------------------------------------------------------------------------------
# dust-emission sampling
# ---------------------------------------------------------------------------------------

def test_cdf_pick_brute_force():
    """The 64-bit cell pick equals a linear scan of exact prefix sums (Python integers),
    including zero-luminosity cells and targets on every boundary."""
    rng = np.random.default_rng(4)
    for trial in range(40):
        n = int(rng.integers(1, 9))
        q = rng.integers(0, 2 ** 32 + 1, n).astype(np.uint64)
        q[rng.random(n) < 0.3] = 0
        if q.sum() == 0:
            q[0] = 1
        Q = [0]
        for v in q:
            Q.append(Q[-1] + int(v))
        tot = Q[-1]
        rs = [int(x) for x in rng.integers(0, 2 ** 63, 20, dtype=np.int64)] + [0, 2 ** 64 - 1]
        for c in range(n):   # smallest r whose target reaches Q[c]
            rs.append(min(2 ** 64 - 1, -(-(Q[c] << 64) // tot)))
        for r in rs:
            target = (r * tot) >> 64
            expect = max(c for c in range(n) if Q[c] <= target and q[c] > 0 or
                         (Q[c] <= target and c == 0 and q[0] > 0))
            k = oracle.cdf_pick(q, r)
            assert Q[k] <= target < Q[k + 1]
            assert k == expect


def test_dust_emission_cell_frequencies():
    """Dust-emission packets start in leaves with frequency proportional to each leaf's
    luminosity 4 pi m kappa_abs B(T) dnu (chi-square over the birth leaves)."""
    rng = np.random.default_rng(6)
    tree = gen.random_tree(rng, (2, 2, 1), 2, 0.4, cell_cm=1.0, rho_range=(0.2, 2.0))
    dust = gen.Dust(np.array([100.0]), np.array([1e-3]), np.array([0.0]), np.array([0.0]))
    m = oracle.Model(tree, dust)
    leaf = m.leaf_mask
    tn = np.where(leaf, rng.uniform(10, 60, m.n_nodes), 0.0)
    N = 200000
    _, _, st, rec = m.trace([gen.Source(gen.SRC_DUST, 0, packets=N)], seed=2, t_node=tn,
                            rec_stride=1)
    lv = m.level_of_nodes()
    mass = brute.node_rho(tree) * (2.0 ** -lv) ** 3
    nu = brute.CL / (100.0 * 1e-4)
    L = np.where(leaf, 4 * np.pi * mass * 1e-3 * brute.planck_nu(nu, np.maximum(tn, 1)), 0.0)
    p = L / L.sum()
    counts = np.bincount(rec["birth"], minlength=m.n_nodes)
    sel = p > 0
    chi2 = (((counts[sel] - N * p[sel]) ** 2) / (N * p[sel])).sum()
    dof = sel.sum() - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)
    # equal-energy packets: every weight is L_tot / N up to the 2^-32 quantisation
    assert st["e_emit"] == pytest.approx(L.sum(), rel=1e-6, abs=0.0)


# ---------------------------------------------------------------------------------------
# surface-brightness maps (Sect. 4.1)
# ---------------------------------------------------------------------------------------

def test_render_uniform_cube_closed_form_and_refinement_invariance():
    """Uniform cube at constant T: I = (1 - a) B(T) (1 - exp(-kappa rho chord)) for axis and
    oblique views; a uniformly refined copy gives the same map."""
    lam = np.array([60.0, 250.0])
    dust = gen.Dust(lam, np.array([5.0, 0.7]), np.array([0.2, 0.0]), np.array([0.0, 0.0]))
    root = (4, 4, 4)
    T = 30.0
    for tree in (gen.TreeDesc(*root, 3.0, np.full(64, 0.4), [], []),
                 gen.uniform_refined_tree(root, 2, rho=0.4, cell_cm=3.0)):
        m = oracle.Model(tree, dust)
        tn = np.where(m.leaf_mask, T, 0.0)
        nu = brute.CL / (lam * 1e-4)
        S = (1 - dust.albedo) * brute.planck_nu(nu, T)
        img, cr = m.render([0, 0, 1.0], 8, tn, [0, 1])
        for q in range(2):
            expect = S[q] * -math.expm1(-dust.kappa_ext[q] * 0.4 * 3.0 * 4.0)
            np.testing.assert_allclose(img[q], expect, rtol=1e-13)
        n = np.array([0.3, -0.5, 0.81])
        n /= np.linalg.norm(n)
        img2, _ = m.render(n, 16, tn, [0, 1], width=7.0)
        e1 = np.array([-n[1], n[0], 0.0]) / math.hypot(n[0], n[1])
        e2 = np.cross(n, e1)
        for j in range(16):
            for i in range(16):
                Q = np.array([2.0, 2.0, 2.0]) + ((i + 0.5) / 16 - 0.5) * 7 * e1 + ((j + 0.5) / 16 - 0.5) * 7 * e2
                t0, t1 = -np.inf, np.inf
                for a in range(3):
                    ta, tb = (0 - Q[a]) / n[a], (4 - Q[a]) / n[a]
                    t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
                chord = max(t1 - t0, 0.0)
                for q in range(2):
                    expect = S[q] * -math.expm1(-dust.kappa_ext[q] * 0.4 * 3.0 * chord)
                    assert img2[q, j, i] == pytest.approx(expect, rel=1e-11, abs=1e-300)


# ---------------------------------------------------------------------------------------
# Lambda iteration (Sect. 3.1 Eq. 2)
# ---------------------------------------------------------------------------------------

def test_lambda_iteration_energy_balance():
    """At the fixed point of J_{n+1} = Lambda S_n + J_0, S = f(J), every leaf re-emits what it
    absorbs, so the dust emission leaving the model equals the absorbed stellar power."""
    lam = np.logspace(-1, 3, 12)
    kap = 0.3 * (lam / 0.55) ** -1.6
    alb = np.clip(0.5 * (1 - np.log10(lam / 0.1) / 4), 0, 0.5)
    dust = gen.Dust(lam, kap, alb, alb.copy())
    root = (4, 4, 4)
    tree = gen.uniform_refined_tree(root, 1, rho=1.0, cell_cm=1.0)
    tree.child_rho[0] = tree.child_rho[0] * np.linspace(0.5, 1.5, len(tree.child_rho[0]))
    m = oracle.Model(tree, dust)
    nu = brute.CL / (lam * 1e-4)
    lstar = 1e-2 * brute.planck_nu(nu, 5000.0)
    src = [gen.Source(gen.SRC_POINT, 0, pos=(2.0, 2.0, 2.0), power=lstar, packets=20000)]
    hist, a_stars, stats = oracle.lambda_iterate(m, src, seed=31, n_max=30, tol=1e-3,
                                                 dust_packets=20000)
    assert 2 < len(hist) < 31
    leaf = m.leaf_mask
    assert 20.0 < hist[-1][leaf].min() and hist[-1][leaf].max() < 3000.0
    last = stats[-1]
    assert last["e_esc"] == pytest.approx(a_stars.sum(), rel=0.03)
    # re-emission conserves energy within the trace as well
    assert last["e_abs"] + last["e_esc"] == pytest.approx(last["e_emit"], rel=1e-10)
