"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same seeded inputs.

Bars: bit-exact for Philox blocks, point location and integer counts (plain FP64 form);
per node |E_gpu - E_ora| <= 1e-6 E_ora + 1e-12 max(E_ora) in the FP64 form; relative RMS
error (paper Eq. 6 form) <= 1e-3 and below the Monte Carlo noise in the FP32-local form;
temperatures within 1e-6 relative; FP64 maps within 1e-6 relative per pixel."""
import math

import numpy as np
import pytest

import gen
import oracle
from tests import brute

pytestmark = pytest.mark.gpu

rt = pytest.importorskip("paper_1206_3710_amd")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def new_ctx(torch):
    return rt.Context(0)


def fp64_close(e_gpu, e_ora):
    tol = 1e-6 * np.abs(e_ora) + 1e-12 * np.abs(e_ora).max()
    bad = np.abs(e_gpu - e_ora) > tol
    return int(bad.sum()), float(np.max(np.abs(e_gpu - e_ora) / np.maximum(np.abs(e_ora), 1e-300)))


def rel_rms(a, ref):
    return float(np.sqrt(((a - ref) ** 2).sum() / (ref ** 2).sum()))


# ---------------------------------------------------------------------------------------

def test_philox_bit_exact(torch):
    ctx = new_ctx(torch)
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2 ** 32, (5000, 4), dtype=np.uint64).astype(np.uint32)
    for k0, k1 in [(0, 0), (0xA4093822, 0x299F31D0), (123456789, 987654321)]:
        g = ctx.philox(k0, k1, ctr)
        o = oracle.philox(k0, k1, ctr)
        assert np.array_equal(g, o)


@pytest.mark.parametrize("seed,root,levels", [(1, (1, 1, 1), 3), (2, (2, 3, 1), 4), (3, (5, 3, 2), 2)])
def test_locate_bit_exact(torch, seed, root, levels):
    rng = np.random.default_rng(seed)
    tree = gen.random_tree(rng, root, levels, 0.4)
    ora = oracle.Model(tree)
    ctx = new_ctx(torch)
    m = ctx.build_tree(tree)
    n = np.array(root, float)
    hmin = 2.0 ** -max(tree.n_levels, 1)
    P = np.vstack([rng.uniform(0, 1, (20000, 3)) * n,
                   rng.integers(0, (n / hmin).astype(int) + 1, (20000, 3)) * hmin,
                   np.array([[0, 0, 0], n, [np.nan, 0, 0], [-1e-300, 0, 0], n - 1e-12])])
    lg, ng = ctx.locate(m, P)
    lo, no = ora.locate(P)
    assert np.array_equal(lg.cpu().numpy(), lo)
    assert np.array_equal(ng.cpu().numpy(), no)


GPU_ONLY = ("block_size", "blocks_per_cu", "refill_threshold", "schedule")


def _trace_pair(torch, w, precision, **kw):
    srcs = w.sources
    ora = oracle.Model(w.trees[0], w.dusts[0])
    eo, esco, sto, reco = ora.trace(srcs, seed=w.seed,
                                    **{k: v for k, v in kw.items() if k not in GPU_ONLY})
    ctx = new_ctx(torch)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, w.dusts[0])
    r = ctx.trace_packets(srcs, seed=w.seed, precision=precision, **kw)
    return ora, eo, esco, sto, reco, r


@pytest.mark.parametrize("variant", ["A", "B"])
def test_trace_fp64_c1(torch, variant):
    """Tiny two-level tree, 1e5 background packets: per-node parity and identical counts."""
    w = gen.c1(variant)
    ora, eo, esco, sto, reco, r = _trace_pair(torch, w, rt.FP64, rec_stride=97)
    eg = r["e_abs_node"].cpu().numpy()
    nbad, worst = fp64_close(eg, eo)
    assert nbad == 0, worst
    st = r["stats"]
    assert st["crossings"] == sto["crossings"]
    assert st["scatterings"] == sto["scatterings"]
    assert st["packets"] == sto["packets"]
    # the oracle sums the 1e5 weights one by one: its rounding error is up to ~N eps
    assert st["e_emit"] == pytest.approx(sto["e_emit"], rel=1e-10)
    np.testing.assert_allclose(r["e_esc"].cpu().numpy(), esco, rtol=1e-9)
    rg = r["records"]
    for f in ("status", "crossings", "events", "node", "birth"):
        assert np.array_equal(rg[f], reco[f]), f
    np.testing.assert_allclose(rg["w"], reco["w"], rtol=1e-9)


def test_trace_fp64_roulette(torch):
    """Russian roulette on: kills, gains and every packet's fate match."""
    w = gen.c1("A", packets=30000)
    ora, eo, esco, sto, reco, r = _trace_pair(torch, w, rt.FP64, rr_threshold=0.3, rr_prob=0.5,
                                              rec_stride=1)
    nbad, worst = fp64_close(r["e_abs_node"].cpu().numpy(), eo)
    assert nbad == 0, worst
    st = r["stats"]
    assert st["kills"] == sto["kills"] and st["kills"] > 0
    assert st["e_rr_gain"] == pytest.approx(sto["e_rr_gain"], rel=1e-9)
    assert np.array_equal(r["records"]["status"], reco["status"])


def _mc_noise(w, seed_b):
    ora = oracle.Model(w.trees[0], w.dusts[0])
    ea, _, _, _ = ora.trace(w.sources, seed=w.seed)
    eb, _, _, _ = ora.trace(w.sources, seed=seed_b)
    return ea, rel_rms(eb, ea) / math.sqrt(2.0)


@pytest.mark.parametrize("sched,block,thr,per_cu", [
    (rt.SCHED_GLOBAL, 256, 0.0, 0), (rt.SCHED_GLOBAL, 64, 0.25, 0), (rt.SCHED_GLOBAL, 512, 0.75, 0),
    (rt.SCHED_REGIONS, 256, 0.0, 0), (rt.SCHED_REGIONS, 512, 0.5, 0), (rt.SCHED_REGIONS, 256, 0.5, 16)])
def test_trace_fp32_local_c1(torch, sched, block, thr, per_cu):
    """FP32-local forms (one global queue; region by region, including small regions that
    force many sweeps): relative RMS error <= 1e-3 and below the MC noise."""
    w = gen.c1("A")
    ora, eo, esco, sto, reco, r = _trace_pair(torch, w, rt.FP32_LOCAL, block_size=block,
                                              refill_threshold=thr, schedule=sched,
                                              blocks_per_cu=per_cu)
    eg = r["e_abs_node"].cpu().numpy()
    _, noise = _mc_noise(w, w.seed + 1000)
    err = rel_rms(eg, eo)
    assert err <= 1e-3 and err < noise, (err, noise)
    st = r["stats"]
    assert st["packets"] == sto["packets"]
    assert abs(st["crossings"] - sto["crossings"]) <= 1e-4 * sto["crossings"]
    cons = st["e_abs"] + st["e_esc"] + st["e_killed"] + st["e_trunc"] - st["e_rr_gain"]
    assert cons == pytest.approx(st["e_emit"], rel=1e-5)


@pytest.mark.parametrize("n", [1, 63, 65, 1000])
def test_ragged_packet_counts(torch, n):
    w = gen.c1("A", packets=n)
    for prec in (rt.FP64, rt.FP32_LOCAL):
        ora, eo, esco, sto, reco, r = _trace_pair(torch, w, prec, rec_stride=1)
        assert r["stats"]["packets"] == n
        if prec == rt.FP64:
            nbad, worst = fp64_close(r["e_abs_node"].cpu().numpy(), eo)
            assert nbad == 0
            assert np.array_equal(r["records"]["crossings"], reco["crossings"])


def test_beams_and_points_random_trees(torch):
    """Beam and point sources (several per call) through random multi-level trees."""
    rng = np.random.default_rng(9)
    tree = gen.random_tree(rng, (3, 2, 2), 4, 0.45, cell_cm=0.5, rho_range=(0.0, 3.0))
    dust = gen.Dust(np.array([0.4, 1.0, 3.0]), np.array([2.0, 1.0, 0.4]), np.array([0.6, 0.3, 0.0]),
                    np.array([0.7, -0.2, 0.0]))
    srcs = []
    for k in range(6):
        d = rng.normal(size=3)
        srcs.append(gen.Source(gen.SRC_BEAM, 0, pos=tuple(rng.uniform(0, 1, 3) * [3, 2, 2]),
                               dir=tuple(d), power=np.array([1.0, 2.0, 3.0]), packets=777))
        srcs.append(gen.Source(gen.SRC_POINT, 0, pos=tuple(rng.uniform(0, 1, 3) * [3, 2, 2]),
                               power=np.array([3.0, 1.0, 0.5]), packets=1500))
    ora = oracle.Model(tree, dust)
    eo, esco, sto, reco = ora.trace(srcs, seed=77, per_lambda=True, rec_stride=1,
                                    rr_threshold=0.1, rr_prob=0.3)
    ctx = new_ctx(torch)
    m = ctx.build_tree(tree)
    ctx.set_dust(m, dust)
    r = ctx.trace_packets(srcs, seed=77, precision=rt.FP64, per_lambda=True, rec_stride=1,
                          rr_threshold=0.1, rr_prob=0.3)
    el = r["e_abs_lambda_node"].cpu().numpy().reshape(3, -1)
    nbad, worst = fp64_close(el.ravel(), eo.ravel())
    assert nbad == 0, worst
    assert r["stats"]["crossings"] == sto["crossings"]
    # records: oracle layout (source-major, then wavelength) with equal packet counts per source
    # differs only in the stride per job; compare per source
    gi = 0
    oi = 0
    for s in srcs:
        nrec = 1500  # oracle nrec uses the largest packet count
        for lam in range(3):
            g = r["records"][gi:gi + s.packets]
            o = reco[oi:oi + s.packets]
            assert np.array_equal(g["crossings"], o["crossings"])
            assert np.array_equal(g["node"], o["node"])
            gi += s.packets
            oi += nrec


def test_multi_model_batch(torch):
    """Several uneven models traced together in one call (both forms)."""
    w = gen.c4(max_models=3, packets=3000, n_lambda=4)
    ctx = new_ctx(torch)
    ids = []
    for t, d in zip(w.trees, w.dusts):
        ids.append(ctx.build_tree(t))
        ctx.set_dust(ids[-1], d)
    srcs = [gen.Source(s.kind, ids[i], power=s.power, packets=s.packets) for i, s in enumerate(w.sources)]
    r64 = ctx.trace_packets(srcs, seed=w.seed, precision=rt.FP64, rr_threshold=w.rr_threshold,
                            rr_prob=w.rr_prob)
    r32 = ctx.trace_packets(srcs, seed=w.seed, precision=rt.FP32_LOCAL, rr_threshold=w.rr_threshold,
                            rr_prob=w.rr_prob)
    e64 = r64["e_abs_node"].cpu().numpy()
    e32 = r32["e_abs_node"].cpu().numpy()
    # exact per-model comparison needs identical stream ids: run the oracle with the same
    # source index by padding with empty-power sources
    base = 0
    for i, (t, d) in enumerate(zip(w.trees, w.dusts)):
        ora = oracle.Model(t, d)
        pads = [gen.Source(gen.SRC_BACKGROUND, 0, power=np.zeros(4), packets=1) for _ in range(i)]
        eo, _, _, _ = ora.trace(pads + [gen.Source(srcs[i].kind, 0, power=srcs[i].power,
                                                   packets=srcs[i].packets)],
                                seed=w.seed, model_index=ids[i], rr_threshold=w.rr_threshold,
                                rr_prob=w.rr_prob)
        nn = ora.n_nodes
        nbad, worst = fp64_close(e64[base:base + nn], eo)
        assert nbad == 0, (i, worst)
        assert rel_rms(e32[base:base + nn], eo) <= 1e-3
        base += nn


def test_temperature_parity(torch):
    """FP64 temperature solve against the oracle's bisection for absorbed powers spanning the
    whole bracket (including both clamps and empty cells)."""
    w = gen.c2(n_root=16, max_level=2, n_lambda=12, packets=2000)
    ora = oracle.Model(w.trees[0], w.dusts[0])
    rng = np.random.default_rng(4)
    leaf = ora.leaf_mask
    lv = ora.level_of_nodes()
    mass = ora.node_rho() * (w.trees[0].root_cell_cm * 2.0 ** -lv) ** 3
    trad = rng.uniform(1.0, 4000.0, ora.n_nodes)
    A = np.array([ora.emission(i, t) if leaf[i] else 0.0 for i, t in enumerate(trad)])
    A *= rng.uniform(0.999, 1.001, len(A))
    A[rng.random(len(A)) < 0.01] = 0.0
    to = ora.solve_temperature(A, 2.0, 3000.0)
    ctx = new_ctx(torch)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, w.dusts[0])
    tg = ctx.solve_temperature(m, A, 2.0, 3000.0).cpu().numpy()
    np.testing.assert_allclose(tg, to, rtol=1e-6, atol=0)
    assert np.all(tg[~leaf] == 0)


@pytest.mark.parametrize("n_lambda", [12, 100])
def test_temperature_converges_to_the_root(torch, n_lambda):
    """The GPU solve (Newton started from an inverse table of the emission per unit mass) finds
    the same root as the oracle's bisection to 1e-12, to 1e-10 relative, for radiation
    temperatures spread over the whole bracket and past both ends."""
    w = gen.c2(n_root=8, max_level=2, n_lambda=n_lambda, packets=1000)
    ora = oracle.Model(w.trees[0], w.dusts[0])
    rng = np.random.default_rng(11)
    leaf = ora.leaf_mask
    trad = np.exp(rng.uniform(np.log(1.0), np.log(5000.0), ora.n_nodes))
    A = np.array([ora.emission(i, t) if leaf[i] else 0.0 for i, t in enumerate(trad)])
    to = ora.solve_temperature(A, 2.0, 3000.0)
    ctx = new_ctx(torch)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, w.dusts[0])
    tg = ctx.solve_temperature(m, A, 2.0, 3000.0).cpu().numpy()
    np.testing.assert_allclose(tg[leaf], to[leaf], rtol=1e-10, atol=0)
    inside = leaf & (trad > 2.5) & (trad < 2900.0)
    np.testing.assert_allclose(tg[inside], trad[inside], rtol=1e-9)
    assert np.all(tg[leaf & (trad <= 2.0)] == 2.0) and np.all(tg[leaf & (trad >= 3000.0)] == 3000.0)


def test_render_parity(torch):
    """FP64 maps against the oracle: axis and oblique views, several wavelengths (two passes)."""
    w = gen.c2(n_root=16, max_level=2, n_lambda=20, packets=1000)
    ora = oracle.Model(w.trees[0], w.dusts[0])
    rng = np.random.default_rng(5)
    tn = np.where(ora.leaf_mask, rng.uniform(8, 40, ora.n_nodes), 0.0)
    ctx = new_ctx(torch)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, w.dusts[0])
    ctx.set_temperature(m, tn)
    lam = list(range(0, 20, 1))
    for n_obs, npix, width in [((1.0, 0, 0), 32, 0.0), ((0, 0, -1.0), 40, 0.0),
                               ((0.3, -0.7, 0.5), 33, 20.0)]:
        io, co = ora.render(n_obs, npix, tn, lam, width=width)
        ig, cg = ctx.render_map(m, n_obs, npix, lam, width=width)
        ig = ig.cpu().numpy()
        assert cg == co
        np.testing.assert_allclose(ig, io, rtol=1e-6, atol=1e-12 * io.max())


@pytest.mark.parametrize("n_lambda", [20, 100])
def test_render_fp32_against_oracle(torch, n_lambda):
    """FP32-transfer maps against the oracle's FP64 maps directly (same cells, equal crossing
    counts): each pixel within 1e-4 relative, values below 1e-7 of the brightest map of the
    selection counted against that floor (the same FP32 error model as against the GPU's FP64
    map).  100 wavelengths take one pass of 128."""
    w = gen.c2(n_root=16, max_level=2, n_lambda=n_lambda, packets=1000)
    ora = oracle.Model(w.trees[0], w.dusts[0])
    rng = np.random.default_rng(6)
    # a tenth of the leaves without a temperature: they attenuate and emit nothing
    tn = np.where(ora.leaf_mask & (rng.random(ora.n_nodes) > 0.1), rng.uniform(8, 40, ora.n_nodes), 0.0)
    ctx = new_ctx(torch)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, w.dusts[0])
    ctx.set_temperature(m, tn)
    lam = list(range(n_lambda))
    for n_obs, npix, width in [((1.0, 0, 0), 32, 0.0), ((0.3, -0.7, 0.5), 33, 20.0)]:
        io, co = ora.render(n_obs, npix, tn, lam, width=width)
        ig, cg = ctx.render_map(m, n_obs, npix, lam, width=width, precision=rt.FP32_LOCAL)
        ig = ig.cpu().numpy()
        assert cg == co
        floor = 1e-7 * np.abs(io).max()
        err = np.abs(ig - io)
        assert np.all(err <= 1e-4 * np.abs(io) + floor), (err / np.maximum(np.abs(io), floor)).max()


def test_dust_emission_parity(torch):
    """Dust-emission source (fixed temperatures): identical cell picks and deposits."""
    w = gen.c2(n_root=12, max_level=2, n_lambda=6, packets=1000)
    ora = oracle.Model(w.trees[0], w.dusts[0])
    rng = np.random.default_rng(6)
    tn = np.where(ora.leaf_mask, rng.uniform(10, 80, ora.n_nodes), 0.0)
    src = [gen.Source(gen.SRC_DUST, 0, packets=5000)]
    eo, esco, sto, reco = ora.trace(src, seed=3, t_node=tn, rec_stride=1)
    ctx = new_ctx(torch)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, w.dusts[0])
    ctx.set_temperature(m, tn)
    r = ctx.trace_packets(src, seed=3, precision=rt.FP64, rec_stride=1)
    assert np.array_equal(r["records"]["birth"], reco["birth"])
    nbad, worst = fp64_close(r["e_abs_node"].cpu().numpy(), eo)
    assert nbad == 0, worst
    r32 = ctx.trace_packets(src, seed=3, precision=rt.FP32_LOCAL, rec_stride=1)
    assert np.array_equal(r32["records"]["birth"], reco["birth"])


def test_lambda_iteration_parity(torch):
    """Three Lambda-iteration steps (Eq. 2): temperatures after each run match the oracle."""
    lam = np.logspace(-1, 3, 10)
    kap = 0.3 * (lam / 0.55) ** -1.6
    alb = np.clip(0.5 * (1 - np.log10(lam / 0.1) / 4), 0, 0.5)
    dust = gen.Dust(lam, kap, alb, alb.copy())
    tree = gen.uniform_refined_tree((4, 4, 4), 1, rho=1.0, cell_cm=1.0)
    tree.child_rho[0] = tree.child_rho[0] * np.linspace(0.5, 1.5, len(tree.child_rho[0]))
    nu = brute.CL / (lam * 1e-4)
    star = [gen.Source(gen.SRC_POINT, 0, pos=(2.1, 1.9, 2.05), power=1e-2 * brute.planck_nu(nu, 5000.0),
                       packets=4000)]
    ora = oracle.Model(tree, dust)
    hist, _, _ = oracle.lambda_iterate(ora, star, seed=31, n_fixed=3, dust_packets=4000)
    ctx = new_ctx(torch)
    m = ctx.build_tree(tree)
    ctx.set_dust(m, dust)
    tg, nd, crit = ctx.lambda_iterate(m, star, seed=31, dust_packets=4000, n_max=3, tol=0.0)
    assert nd == 3
    np.testing.assert_allclose(tg.cpu().numpy(), hist[-1], rtol=1e-6)


def test_errors_leave_context_usable(torch):
    ctx = new_ctx(torch)
    w = gen.c1("A", packets=100)
    m = ctx.build_tree(w.trees[0])
    with pytest.raises(rt.RTError) as e:
        ctx.trace_packets(w.sources, seed=1)
    assert e.value.code == rt.RT_ESTATE
    ctx.set_dust(m, w.dusts[0])
    bad = [gen.Source(gen.SRC_BACKGROUND, 0, power=np.array([1.0]), packets=0)]
    with pytest.raises(rt.RTError) as e:
        ctx.trace_packets(bad, seed=1)
    assert e.value.code == rt.RT_EINVAL
    with pytest.raises(rt.RTError):
        ctx.trace_packets([gen.Source(gen.SRC_POINT, 0, pos=(16.0, 1, 1), power=np.array([1.0]),
                                      packets=5)], seed=1)
    with pytest.raises(rt.RTError) as e:
        ctx.trace_packets([gen.Source(gen.SRC_DUST, 0, packets=5)], seed=1)
    assert e.value.code == rt.RT_ESTATE
    with pytest.raises(rt.RTError):
        ctx.set_dust(m, gen.Dust(np.array([1.0]), np.array([1.0]), np.array([1.5]), np.array([0.0])))
    with pytest.raises(rt.RTError):
        ctx.build_tree(gen.TreeDesc(2, 2, 2, 1.0, np.full(8, -1.0), [], []))
    with pytest.raises(rt.RTError):
        ctx.build_tree(gen.TreeDesc(2, 2, 2, 1.0, np.ones(8), [np.array([3, 1])], [np.ones(16)]))
    r = ctx.trace_packets(w.sources, seed=1)
    assert r["stats"]["packets"] == 100


@pytest.mark.parametrize("levels,per_cu", [(3, 32), (4, 32), (4, 16)])
def test_split_regions_and_records(torch, levels, per_cu):
    """Region schedule with a small LDS capacity (many blocks per CU), so that single root-cell
    subtrees are larger than a region and are split into bricks of their children, one or two
    levels down: deposits, fates and crossing counts against the oracle, including packets that
    enter a split cell from a coarser neighbour (a point source in a coarse cell)."""
    # root cells 0-6 refined uniformly to `levels` levels; root cell 7 stays a leaf, so packets
    # leaving it enter split cells from a coarser level
    rng = np.random.default_rng(3)
    refined, kids = [np.arange(7, dtype=np.int64)], []
    n = 7 * 8
    for lvl in range(1, levels):
        kids.append(np.full(n, 0.5))
        refined.append(np.arange(n, dtype=np.int64))
        n *= 8
    kids.append(rng.uniform(0.1, 2.0, n))
    tree = gen.TreeDesc(2, 2, 2, 0.5, np.full(8, 0.5), refined, kids)
    dust = gen.Dust(np.array([1.0]), np.array([1.0]), np.array([0.5]), np.array([0.4]))
    src = [gen.Source(gen.SRC_BACKGROUND, 0, power=np.array([1.0]), packets=40000),
           gen.Source(gen.SRC_POINT, 0, pos=(1.51, 1.47, 1.53), power=np.array([2.0]), packets=40000)]
    ora = oracle.Model(tree, dust)
    eo, esco, sto, reco = ora.trace(src, seed=5, rec_stride=1)
    ctx = new_ctx(torch)
    m = ctx.build_tree(tree)
    ctx.set_dust(m, dust)
    r = ctx.trace_packets(src, seed=5, precision=rt.FP32_LOCAL, schedule=rt.SCHED_REGIONS,
                          blocks_per_cu=per_cu, rec_stride=1)
    eg = r["e_abs_node"].cpu().numpy()
    assert rel_rms(eg, eo) <= 1e-3
    rg = r["records"]
    assert r["stats"]["packets"] == 80000 and r["stats"]["truncated"] == 0
    same = np.mean(rg["crossings"] == reco["crossings"])
    assert same > 0.99, same
    assert np.array_equal(rg["birth"], reco["birth"])
    r64 = ctx.trace_packets(src, seed=5, precision=rt.FP64)
    assert r["stats"]["crossings"] == pytest.approx(r64["stats"]["crossings"], rel=1e-3)


def test_region_and_global_schedules_agree(torch):
    """The two FP32-local schedules follow the same arithmetic: per-node results agree far
    below the Monte Carlo noise, and the crossing counts are equal."""
    w = gen.c2(n_root=24, max_level=3, n_lambda=6, packets=20000)
    ctx = new_ctx(torch)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, w.dusts[0])
    kw = dict(seed=w.seed, precision=rt.FP32_LOCAL, rr_threshold=w.rr_threshold, rr_prob=w.rr_prob)
    a = ctx.trace_packets(w.sources, schedule=rt.SCHED_GLOBAL, **kw)
    b = ctx.trace_packets(w.sources, schedule=rt.SCHED_REGIONS, blocks_per_cu=8, **kw)
    ea, eb = a["e_abs_node"].cpu().numpy(), b["e_abs_node"].cpu().numpy()
    assert rel_rms(eb, ea) < 1e-5
    assert a["stats"]["crossings"] == b["stats"]["crossings"]
    assert a["stats"]["scatterings"] == b["stats"]["scatterings"]


@pytest.mark.parametrize("block,per_cu", [(256, 4), (512, 2), (768, 1), (1024, 1)])
def test_region_launch_shapes_follow_the_same_histories(torch, block, per_cu):
    """Every launch shape of the region pass, with small birth batches (many sweeps whose births
    the pass kernel's blocks write after their work items) and small work items, follows the
    global schedule's histories: the same per-packet fates, crossings and scatterings, the
    same emitted energy, and per-node results equal to FP32 summation order.  Each pass wave
    takes its next-queue records in chunks; the unused chunk ends must drop out of the sort."""
    w = gen.c2(n_root=24, max_level=3, n_lambda=6, packets=20000)
    ctx = new_ctx(torch)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, w.dusts[0])
    kw = dict(seed=w.seed, precision=rt.FP32_LOCAL, rr_threshold=w.rr_threshold, rr_prob=w.rr_prob,
              rec_stride=5)
    a = ctx.trace_packets(w.sources, schedule=rt.SCHED_GLOBAL, **kw)
    b = ctx.trace_packets(w.sources, schedule=rt.SCHED_REGIONS, block_size=block, blocks_per_cu=per_cu,
                          batch_packets=3000, chunk_packets=512, **kw)
    for k in ("crossings", "scatterings", "kills", "packets"):
        assert a["stats"][k] == b["stats"][k], k
    assert abs(a["stats"]["e_emit"] - b["stats"]["e_emit"]) <= 1e-12 * a["stats"]["e_emit"]
    ra, rb = a["records"], b["records"]
    for f in ("status", "crossings", "events", "node", "birth"):
        assert np.array_equal(ra[f], rb[f]), f
    assert rel_rms(b["e_abs_node"].cpu().numpy(), a["e_abs_node"].cpu().numpy()) < 1e-5


def test_region_tail_parking(torch):
    """Packets re-queued inside their cell when a work item's queue runs dry (forced after every
    crossing round here) resume without a counted crossing: same crossings, scatterings and
    per-packet fates as without re-queueing, and the same per-node result to FP32 rounding."""
    w = gen.c2(n_root=24, max_level=3, n_lambda=4, packets=20000)
    ctx = new_ctx(torch)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, w.dusts[0])
    kw = dict(seed=w.seed, precision=rt.FP32_LOCAL, rr_threshold=w.rr_threshold, rr_prob=w.rr_prob,
              schedule=rt.SCHED_REGIONS, blocks_per_cu=8, rec_stride=7)
    a = ctx.trace_packets(w.sources, tail_park=-1, **kw)
    b = ctx.trace_packets(w.sources, tail_park=1, **kw)
    for k in ("crossings", "scatterings", "kills", "packets"):
        assert a["stats"][k] == b["stats"][k], k
    ra, rb = a["records"], b["records"]
    for f in ("status", "crossings", "events", "node", "birth"):
        assert np.array_equal(ra[f], rb[f]), f
    ea, eb = a["e_abs_node"].cpu().numpy(), b["e_abs_node"].cpu().numpy()
    assert rel_rms(eb, ea) < 1e-5


def test_autotune_and_cache(torch, tmp_path):
    """The autotuner returns candidate launch parameters, a second call is answered from its
    cache file, and tracing with the tuned parameters gives the same histories as the
    defaults (launch parameters change only the processing order)."""
    w = gen.c2(n_root=24, max_level=3, n_lambda=4, packets=40000)
    ctx = new_ctx(torch)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, w.dusts[0])
    cache = str(tmp_path / "tune.txt")
    kw = dict(seed=w.seed, rr_threshold=w.rr_threshold, rr_prob=w.rr_prob)
    p1, r1 = ctx.autotune(w.sources, precision=rt.FP32_LOCAL, sample_fraction=0.5, cache=cache, **kw)
    assert r1 > 0
    assert p1["block_size"] in (512, 768, 1024) and p1["blocks_per_cu"] == 1
    assert p1["tail_park"] in (8, 16, 32, -1) and p1["chunk_packets"] % p1["block_size"] == 0
    p2, r2 = ctx.autotune(w.sources, precision=rt.FP32_LOCAL, sample_fraction=0.5, cache=cache, **kw)
    assert p2 == p1 and r2 == pytest.approx(r1, rel=1e-6)
    assert len(open(cache).read().strip().splitlines()) == 1
    a = ctx.trace_packets(w.sources, precision=rt.FP32_LOCAL, **kw)
    b = ctx.trace_packets(w.sources, precision=rt.FP32_LOCAL, **kw, **p1)
    for k in ("crossings", "scatterings", "kills", "packets"):
        assert a["stats"][k] == b["stats"][k], k
    ea, eb = a["e_abs_node"].cpu().numpy(), b["e_abs_node"].cpu().numpy()
    assert rel_rms(eb, ea) < 1e-5
    p64, _ = ctx.autotune(w.sources, precision=rt.FP64, sample_fraction=0.25, **kw)
    assert p64["block_size"] in (64, 128, 256)


def test_sweep_graph_replay_matches_direct_launches(torch):
    """The sweeps of the region schedule replayed from a captured HIP graph (16 sweeps per
    replay, twice in a row to reuse the instantiated graph) give the histories of direct
    launches: equal counts and per-packet records, per-node results to FP32 summation order.
    Tail parking is off: which packets a wave re-queues depends on the order in which the waves
    of a block take their packets, so with it the number of sweeps may differ by one between
    any two runs."""
    w = gen.c2(n_root=24, max_level=3, n_lambda=4, packets=60000)
    ctx = new_ctx(torch)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, w.dusts[0])
    kw = dict(seed=w.seed, precision=rt.FP32_LOCAL, rr_threshold=w.rr_threshold, rr_prob=w.rr_prob,
              schedule=rt.SCHED_REGIONS, blocks_per_cu=8, batch_packets=20000, rec_stride=11,
              tail_park=-1)
    a = ctx.trace_packets(w.sources, **kw)
    for _ in range(2):
        b = ctx.trace_packets(w.sources, sweep_graph=1, **kw)
        for k in ("crossings", "scatterings", "kills", "packets"):
            assert a["stats"][k] == b["stats"][k], k
        assert b["stats"]["main_launches"] == a["stats"]["main_launches"]
        for f in ("status", "crossings", "events", "node", "birth"):
            assert np.array_equal(a["records"][f], b["records"][f]), f
        ea, eb = a["e_abs_node"].cpu().numpy(), b["e_abs_node"].cpu().numpy()
        assert rel_rms(eb, ea) < 1e-5


@pytest.mark.parametrize("n_lambda", [12, 100, 140])
def test_render_fp32_transfer_against_fp64(torch, n_lambda):
    """Maps with the transfer in FP32: the same cells as the FP64 map (equal crossing counts),
    each pixel within 1e-4 relative of it (a few hundred FP32 steps of a few roundings each).
    12 wavelengths take one pass of 16, 100 one pass of 128 (the last group of 8 padded), 140 a
    pass of 128 and one of 16."""
    w = gen.c2(n_root=24, max_level=3, n_lambda=n_lambda, packets=20000)
    ctx = new_ctx(torch)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, w.dusts[0])
    r = ctx.trace_packets(w.sources, seed=w.seed, precision=rt.FP64)
    ctx.solve_temperature(m, r["e_abs_node"], 2.0, 3000.0)
    lam = list(range(n_lambda))
    for d in [(1.0, 0.0, 0.0), (0.3, -0.5, 0.81)]:
        i64, c64 = ctx.render_map(m, d, 48, lam, precision=rt.FP64)
        i32, c32 = ctx.render_map(m, d, 48, lam, precision=rt.FP32_LOCAL)
        assert c32 == c64 > 0
        a64, a32 = i64.cpu().numpy(), i32.cpu().numpy()
        # values below the FP32 range of a wavelength's map (far Wien tail at dust temperatures)
        # count against the brightest map of the selection
        floor = 1e-7 * np.abs(a64).max()
        err = np.abs(a32 - a64)
        rel = err / np.maximum(np.abs(a64), floor)
        print("max relative error per wavelength", rel.max(axis=(1, 2)))
        assert np.all(err <= 1e-4 * np.abs(a64) + floor)
