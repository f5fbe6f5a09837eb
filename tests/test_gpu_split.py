"""GPU parity of package splitting at subgrid entry with the roulette at subgrid exit (paper
Sect. 2.3) in the FP32-local region schedule, against the oracle run with the same split
factor on the same seeded inputs.

Every branch draws from the counter-based stream with its own branch identifier, so the
oracle and the GPU follow the same histories: the sampled main-line records (the package as
emitted) must reproduce the oracle's fates, the split and roulette counts must agree to the
fraction of FP32-rerouted histories, and the absorbed energy per node must agree far below the
Monte Carlo noise.  Splitting only rescales the main line's weight by powers of N, exactly, in
both precisions.  A run that exhausts the sweep's queue room skips splits: it must stay
energy-conserving and unbiased (closed forms of a beam through a pure absorber)."""
import math

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

rt = pytest.importorskip("paper_1206_3710_amd")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def rel_rms(a, ref):
    return float(np.sqrt(((a - ref) ** 2).sum() / (ref ** 2).sum()))


def energy_gap(st):
    lhs = st["e_emit"] + st["e_rr_gain"] + st["e_split_gain"]
    rhs = st["e_abs"] + st["e_esc"] + st["e_killed"] + st["e_trunc"] + st["e_split_killed"]
    return abs(lhs - rhs) / lhs


def _box_case():
    """Scattering block refined 3 levels deep in an isotropic field, plus a point source in a
    coarse root cell."""
    tree = gen.refined_block(3)
    dust = gen.Dust(np.array([1.0]), np.array([1.0]), np.array([0.9]), np.array([0.3]))
    src = [gen.Source(gen.SRC_BACKGROUND, 0, power=np.array([1.0]), packets=20000),
           gen.Source(gen.SRC_POINT, 0, pos=(0.4, 0.6, 3.5), power=np.array([3.0]), packets=20000)]
    return tree, dust, src, 17


def _rand_case():
    """Random three-level tree (level changes inside refined root cells, for the coarser reading
    of "grid"), scattering dust, isotropic field and a point source."""
    tree = gen.random_tree(np.random.default_rng(5), root=(4, 4, 4), max_level=3, p_refine=0.4)
    dust = gen.Dust(np.array([1.0]), np.array([0.5]), np.array([0.6]), np.array([0.2]))
    src = [gen.Source(gen.SRC_BACKGROUND, 0, power=np.array([1.0]), packets=20000),
           gen.Source(gen.SRC_POINT, 0, pos=(1.4, 2.6, 2.5), power=np.array([3.0]), packets=20000)]
    return tree, dust, src, 23


def _c1_case():
    w = gen.c1("A", packets=40000)
    return w.trees[0], w.dusts[0], w.sources, w.seed


def _run(torch, tree, dust, src, seed, **kw):
    ctx = rt.Context(0)
    m = ctx.build_tree(tree)
    ctx.set_dust(m, dust)
    r = ctx.trace_packets(src, seed=seed, precision=rt.FP32_LOCAL, schedule=rt.SCHED_REGIONS, **kw)
    ctx.close()
    return r


def test_split_factor_one_changes_nothing(torch):
    """split_n 1 is the unsplit path: identical records and counts."""
    tree, dust, src, seed = _c1_case()
    kw = dict(rr_threshold=1e-2, rr_prob=0.8, rec_stride=13)
    a = _run(torch, tree, dust, src, seed, **kw)
    b = _run(torch, tree, dust, src, seed, split_n=1, **kw)
    for k in ("crossings", "scatterings", "kills", "packets"):
        assert a["stats"][k] == b["stats"][k], k
    assert b["stats"]["splits"] == 0 and b["stats"]["split_kills"] == 0
    for f in ("status", "crossings", "events", "node", "birth", "w"):
        assert np.array_equal(a["records"][f], b["records"][f]), f


@pytest.mark.parametrize("case,n,per_cu,depth", [("c1", 2, 0, 0), ("c1", 4, 16, 0), ("box", 4, 0, 0),
                                                ("box", 8, 8, 0), ("rand", 4, 0, 0), ("rand", 4, 0, 1),
                                                ("rand", 2, 8, 2)])
def test_split_parity_against_oracle(torch, case, n, per_cu, depth):
    """depth > 0: the coarser readings of "grid" (levels below depth one grid with their
    ancestor at depth)."""
    tree, dust, src, seed = {"c1": _c1_case, "box": _box_case, "rand": _rand_case}[case]()
    kw = dict(rr_threshold=1e-2, rr_prob=0.8, split_depth=depth)
    ora = oracle.Model(tree, dust)
    eo, _, sto, reco = ora.trace(src, seed=seed, rec_stride=1, split_n=n, **kw)
    # a few thousand births per sweep keep the split-off packages within the sweep's room (the
    # random tree, one region, splits about 13 times per emitted packet with every oct a grid)
    r = _run(torch, tree, dust, src, seed, rec_stride=1, split_n=n, blocks_per_cu=per_cu,
             batch_packets=1024 if case == "rand" else 4096, **kw)
    st = r["stats"]
    assert st["split_skips"] == 0
    assert sto["splits"] > 0 and sto["split_kills"] > 0
    # main line: the package as emitted, one record per packet
    rg = r["records"]
    assert len(rg) == len(reco)
    assert np.array_equal(rg["birth"], reco["birth"])
    same = ((rg["status"] == reco["status"]) & (rg["crossings"] == reco["crossings"])
            & (rg["events"] == reco["events"]) & (rg["node"] == reco["node"]))
    assert same.mean() >= 0.99, same.mean()
    assert np.any(reco["status"] == 3) and np.any(rg["status"] == 3)
    # FP32 weights: the step model of the full-size test (2^-24 (8 n + n^2 / 2), n = crossings
    # + events + 1) holds for all but a few packets (a grazing exit stretches the effect of the
    # FP32 direction error); none is off by more than 1e-4, far below a factor of N
    steps = rg["crossings"].astype(np.float64) + rg["events"] + 1.0
    tol = 2.0 ** -24 * (8.0 * steps + 0.5 * steps * steps) * np.abs(reco["w"])
    dw = np.abs(rg["w"] - reco["w"])
    assert np.mean(dw[same] > tol[same]) <= 1e-3
    bad = same & (dw > 1e-4 * np.abs(reco["w"]))
    assert not bad.any(), (rg[bad][:5], reco[bad][:5])
    # all branches: counts agree to the fraction of rerouted histories
    for k in ("splits", "split_kills", "crossings", "scatterings"):
        assert abs(st[k] - sto[k]) <= 0.01 * sto[k] + 5, (k, st[k], sto[k])
    assert st["packets"] == sto["packets"] and st["truncated"] == 0
    assert energy_gap(st) < 1e-5, energy_gap(st)
    # per node: far below the Monte Carlo noise of an independent split realisation
    eg = r["e_abs_node"].cpu().numpy()
    eb, _, _, _ = ora.trace(src, seed=seed + 1000, split_n=n, **kw)
    noise = rel_rms(eb, eo) / math.sqrt(2.0)
    err = rel_rms(eg, eo)
    print(f"{case} split {n}: rel RMS {err:.3e}, noise {noise:.3e}, splits {st['splits']}")
    assert err <= 1e-3 and err < 0.25 * noise, (err, noise)


@pytest.mark.parametrize("n", [2, 4, 8])
def test_split_scales_main_line_by_powers_of_n(torch, n):
    """Without the roulette at events nothing in a history depends on the size of its weight:
    with and without splitting the package as emitted follows the same path, and its final
    weight differs by N^k exactly (a split divides it by N, a surviving exit roulette multiplies
    it by N; both exact for N a power of two), on the GPU as in the oracle.  In the small cloud
    packets born in, or escaping from, refined cells end with k = +1 or -1."""
    tree, dust, src, seed = _c1_case()
    ora = oracle.Model(tree, dust)
    _, _, _, ro1 = ora.trace(src, seed=seed, rec_stride=1)
    _, _, _, ron = ora.trace(src, seed=seed, rec_stride=1, split_n=n)
    g1 = _run(torch, tree, dust, src, seed, rec_stride=1)["records"]
    gn = _run(torch, tree, dust, src, seed, rec_stride=1, split_n=n, batch_packets=4096)["records"]
    for f in ("crossings", "events"):
        esc = gn["status"] == 0
        assert np.array_equal(gn[f][esc], g1[f][esc]), f
    both = ((gn["status"] == 0) & (ron["status"] == 0) & (ro1["status"] == 0)
            & (gn["crossings"] == ron["crossings"]) & (gn["events"] == ron["events"]))
    assert both.sum() > 10000
    rg = gn["w"][both] / g1["w"][both]
    ro = ron["w"][both] / ro1["w"][both]
    assert np.array_equal(rg, ro)
    k = np.log2(ro) / math.log2(n)
    assert np.array_equal(k, np.round(k)) and np.any(k < 0) and np.any(k > 0)


@pytest.mark.parametrize("n", [4, 16])
def test_split_room_exhausted_stays_unbiased(torch, n):
    """4096 beam packets enter the refined block in one sweep, so the N - 1 new packages of
    every split do not all fit in the sweep's queue room: the splits that do not fit are
    skipped.  The run conserves energy, and the mean escaped energy of a pure absorber stays
    w0 exp(-tau) within 4 standard deviations of the worst case (every split skipped, the exit
    roulette alone: variance (N - 1) w0^2 exp(-2 tau) per packet)."""
    tree = gen.refined_block(2)
    kappa = 0.2
    dust = gen.Dust(np.array([1.0]), np.array([kappa]), np.array([0.0]), np.array([0.0]))
    npk = 4096
    src = [gen.Source(gen.SRC_BEAM, 0, pos=(0.3, 1.7, 2.2), dir=(1.0, 0.0, 0.0),
                      power=np.array([1.0]), packets=npk)]
    r = _run(torch, tree, dust, src, 11, split_n=n)
    st = r["stats"]
    assert st["split_skips"] > 0 and st["splits"] > 0
    assert st["splits"] + st["split_skips"] == npk  # one subgrid entry per packet
    # each package as emitted enters 10 cells, each new package 8 (see the oracle's pin)
    assert st["crossings"] == 10 * npk + 8 * (n - 1) * st["splits"]
    assert energy_gap(st) < 1e-5
    w0 = st["e_emit"] / npk
    tau = kappa * (4.0 - 0.3)
    esc = float(r["e_esc"].cpu().numpy()[0]) / npk
    sd = w0 * math.exp(-tau) * math.sqrt((n - 1.0) / npk)
    assert abs(esc - w0 * math.exp(-tau)) < 4.0 * sd, (esc, w0 * math.exp(-tau), sd)


@pytest.mark.parametrize("n", [16, 64])
def test_split_fp64_queue_exhausted_stays_unbiased(torch, n):
    """The FP64 form's queue of split-off packages holds 4 per emitted packet here (16384 for
    4096 beam packets), so with N - 1 = 15 or 63 new packages per split most splits do not fit
    and are skipped, and the last reservation straddles the end of the queue (its slots inside
    the queue are marked empty).  Crossing count, energy identity and the mean escaped energy
    as for the region schedule."""
    tree = gen.refined_block(2)
    kappa = 0.2
    dust = gen.Dust(np.array([1.0]), np.array([kappa]), np.array([0.0]), np.array([0.0]))
    npk = 4096
    src = [gen.Source(gen.SRC_BEAM, 0, pos=(0.3, 1.7, 2.2), dir=(1.0, 0.0, 0.0),
                      power=np.array([1.0]), packets=npk)]
    ctx = rt.Context(0)
    m = ctx.build_tree(tree)
    ctx.set_dust(m, dust)
    r = ctx.trace_packets(src, seed=11, precision=rt.FP64, split_n=n)
    ctx.close()
    st = r["stats"]
    assert st["split_skips"] > 0 and st["splits"] > 0
    assert st["splits"] + st["split_skips"] == npk
    assert st["splits"] * (n - 1) <= 4 * npk
    assert st["crossings"] == 10 * npk + 8 * (n - 1) * st["splits"]
    assert energy_gap(st) < 1e-12
    w0 = st["e_emit"] / npk
    tau = kappa * (4.0 - 0.3)
    esc = float(r["e_esc"].cpu().numpy()[0]) / npk
    sd = w0 * math.exp(-tau) * math.sqrt((n - 1.0) / npk)
    assert abs(esc - w0 * math.exp(-tau)) < 4.0 * sd, (esc, w0 * math.exp(-tau), sd)


def test_split_rejected_in_the_one_queue_form(torch):
    """Splitting runs in the region schedule and the FP64 form; the one-queue FP32-local form
    and factors above 64 are rejected, and the context stays usable."""
    tree, dust, src, seed = _c1_case()
    ctx = rt.Context(0)
    m = ctx.build_tree(tree)
    ctx.set_dust(m, dust)
    with pytest.raises(rt.RTError):
        ctx.trace_packets(src, seed=seed, split_n=2, precision=rt.FP32_LOCAL, schedule=rt.SCHED_GLOBAL)
    for prec in (rt.FP32_LOCAL, rt.FP64):
        with pytest.raises(rt.RTError):
            ctx.trace_packets(src, seed=seed, precision=prec, split_n=65)
        r = ctx.trace_packets(src, seed=seed, precision=prec, split_n=2)
        assert r["stats"]["splits"] > 0
    ctx.close()


@pytest.mark.parametrize("case,n,depth", [("c1", 2, 0), ("c1", 4, 0), ("box", 4, 0), ("box", 8, 0),
                                          ("rand", 4, 0), ("rand", 4, 1), ("rand", 3, 2)])
def test_split_fp64_equals_oracle(torch, case, n, depth):
    """The FP64 form with splitting follows the oracle's histories exactly: every main-line
    record (fate, crossings, events, end node, birth) equal and its weight to 1e-9; the counts
    of splits, exit-roulette kills, crossings, scatterings and event kills equal over all
    branches; the absorbed energy per node and the escaped energy to 1e-9 (the order of the
    FP64 atomic sums), with the split packages followed from a queue in later launches."""
    tree, dust, src, seed = {"c1": _c1_case, "box": _box_case, "rand": _rand_case}[case]()
    kw = dict(rr_threshold=1e-2, rr_prob=0.8, split_n=n, split_depth=depth)
    ora = oracle.Model(tree, dust)
    eo, esco, sto, reco = ora.trace(src, seed=seed, rec_stride=1, **kw)
    ctx = rt.Context(0)
    m = ctx.build_tree(tree)
    ctx.set_dust(m, dust)
    r = ctx.trace_packets(src, seed=seed, precision=rt.FP64, rec_stride=1, **kw)
    ctx.close()
    st, rg = r["stats"], r["records"]
    assert st["split_skips"] == 0 and sto["splits"] > 0 and sto["split_kills"] > 0
    for f in ("status", "crossings", "events", "node", "birth"):
        assert np.array_equal(rg[f], reco[f]), f
    np.testing.assert_allclose(rg["w"], reco["w"], rtol=1e-9)
    for k in ("splits", "split_kills", "crossings", "scatterings", "kills", "packets"):
        assert st[k] == sto[k], (k, st[k], sto[k])
    for k in ("e_split_gain", "e_split_killed", "e_rr_gain", "e_killed", "e_emit"):
        assert abs(st[k] - sto[k]) <= 1e-9 * abs(sto[k]) + 1e-300, (k, st[k], sto[k])
    np.testing.assert_allclose(r["e_abs_node"].cpu().numpy(), eo, rtol=1e-9, atol=1e-12 * eo.max())
    np.testing.assert_allclose(r["e_esc"].cpu().numpy(), esco, rtol=1e-9)
    assert energy_gap(st) < 1e-12


def test_split_fp64_counts_packages_that_end_before_a_crossing(torch):
    """Split-off packages in an optically thick block (40 per root cell) with the event roulette
    on every event nearly all scatter and are killed in the cell they were split in, with no
    crossing of their own; whole waves of the queue launches end that way.  Their scatterings,
    kills and killed energy still reach the totals: the counts equal the oracle's and the
    energy identity holds."""
    tree = gen.refined_block(2)
    dust = gen.Dust(np.array([1.0]), np.array([40.0]), np.array([0.9]), np.array([0.0]))
    src = [gen.Source(gen.SRC_POINT, 0, pos=(0.99, 2.1, 2.2), power=np.array([1.0]), packets=4000)]
    kw = dict(rr_threshold=1.0, rr_prob=0.99, split_n=8, split_depth=0)
    eo, esco, sto, _ = oracle.Model(tree, dust).trace(src, seed=29, rec_stride=0, **kw)
    ctx = rt.Context(0)
    m = ctx.build_tree(tree)
    ctx.set_dust(m, dust)
    r = ctx.trace_packets(src, seed=29, precision=rt.FP64, **kw)
    ctx.close()
    st = r["stats"]
    assert sto["splits"] > 500 and sto["kills"] > 2 * sto["packets"]
    for k in ("splits", "split_kills", "crossings", "scatterings", "kills", "packets"):
        assert st[k] == sto[k], (k, st[k], sto[k])
    for k in ("e_split_gain", "e_split_killed", "e_rr_gain", "e_killed", "e_emit"):
        assert abs(st[k] - sto[k]) <= 1e-9 * abs(sto[k]) + 1e-300, (k, st[k], sto[k])
    np.testing.assert_allclose(r["e_abs_node"].cpu().numpy(), eo, rtol=1e-9, atol=1e-12 * eo.max())
    assert energy_gap(st) < 1e-12


def test_split_reduces_noise_in_refined_block(torch):
    """The oracle's noise pin on the GPU: strongly scattering block refined three levels deep in
    an isotropic field, same number of emitted packages; splitting by 4 lowers the relative RMS
    difference (Eq. 7 form) of the deepest cells between 6 independent runs and their mean."""
    tree = gen.refined_block(3)
    dust = gen.Dust(np.array([1.0]), np.array([1.0]), np.array([0.9]), np.array([0.3]))
    src = [gen.Source(gen.SRC_BACKGROUND, 0, power=np.array([1.0]), packets=3000)]
    o = oracle.Model(tree, dust)
    deep = (o.level_of_nodes() == 3) & o.leaf_mask
    ctx = rt.Context(0)
    m = ctx.build_tree(tree)
    ctx.set_dust(m, dust)

    def noise(n):
        es = np.array([ctx.trace_packets(src, seed=3 + 7 * k, precision=rt.FP32_LOCAL, split_n=n)
                       ["e_abs_node"].cpu().numpy()[deep] for k in range(6)])
        ref = es.mean(axis=0)
        return float(np.sqrt(((es - ref) ** 2).mean() / (ref ** 2).mean()))
    n1, n4 = noise(1), noise(4)
    ctx.close()
    assert n4 < 0.85 * n1, (n1, n4)
