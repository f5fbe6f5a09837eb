"""Pins of the oracle's package splitting at subgrid entry with Russian roulette at subgrid exit
(paper Sect. 2.3; the noise study of Sect. 4.1, Table 1).

Splitting and the exit roulette keep every expectation unchanged, so the pins are the exact
energy identity, closed forms in expectation, agreement in expectation with the unsplit
estimator, and the reduction of the noise in the refined cells that the paper reports for the
external field."""
import math

import numpy as np
import pytest

import gen
import oracle


def energy_gap(st):
    lhs = st["e_emit"] + st["e_rr_gain"] + st["e_split_gain"]
    rhs = st["e_abs"] + st["e_esc"] + st["e_killed"] + st["e_trunc"] + st["e_split_killed"]
    return abs(lhs - rhs) / lhs


def test_split_factor_one_changes_nothing():
    w = gen.c1("A", packets=5000)
    o = oracle.Model(w.trees[0], w.dusts[0])
    a = o.trace(w.sources, seed=w.seed, rec_stride=7)
    b = o.trace(w.sources, seed=w.seed, rec_stride=7, split_n=1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[3], b[3])
    assert b[2]["splits"] == 0 and b[2]["split_kills"] == 0


@pytest.mark.parametrize("n,rr", [(2, False), (4, True), (8, True)])
def test_split_energy_identity(n, rr):
    """Emitted + roulette gains = absorbed + escaped + killed + truncated, to rounding."""
    w = gen.c1("A", packets=8000)
    o = oracle.Model(w.trees[0], w.dusts[0])
    kw = dict(rr_threshold=1e-2, rr_prob=0.8) if rr else {}
    _, _, st, _ = o.trace(w.sources, seed=w.seed, split_n=n, **kw)
    assert st["splits"] > 0 and st["split_kills"] > 0
    assert energy_gap(st) < 1e-12


def test_branch_ids_distinct():
    """Children of one split, and splits at different crossings or on different branches, get
    different nonzero 30-bit branch identifiers."""
    ids = set()
    for b in (0, 1, 12345, 0x3FFFFFFF):
        for n in range(1, 200):
            for c in range(1, 8):
                v = oracle.branch_id(b, n, c)
                assert 0 < v < (1 << 30)
                ids.add((b, n, c, v))
    vals = [v for (_, _, _, v) in ids]
    assert len(set(vals)) == len(vals)


@pytest.mark.parametrize("n", [2, 4])
def test_split_unbiased_beam_closed_form(n):
    """Pure absorber, uniform density, beam straight through the refined block: every history
    is a straight line, the mean escaped energy is w0 exp(-tau) and the mean absorbed energy
    w0 (1 - exp(-tau)); splitting at the block's entry and the roulette at its exit leave the
    mean unchanged, with variance e^-2tau (1 - 1/n) per emitted packet."""
    tree = gen.refined_block(2)
    kappa = 0.2
    dust = gen.Dust(np.array([1.0]), np.array([kappa]), np.array([0.0]), np.array([0.0]))
    o = oracle.Model(tree, dust)
    npk = 20000
    src = [gen.Source(gen.SRC_BEAM, 0, pos=(0.3, 1.7, 2.2), dir=(1.0, 0.0, 0.0),
                      power=np.array([1.0]), packets=npk)]
    _, esc, st, _ = o.trace(src, seed=11, split_n=n)
    w0 = st["e_emit"] / npk
    tau = kappa * 1.0 * (4.0 - 0.3)
    assert st["splits"] == npk  # one level increase on the way in
    mean = esc[0] / npk
    sd = w0 * math.exp(-tau) * math.sqrt((1.0 - 1.0 / n) / npk)
    assert abs(mean - w0 * math.exp(-tau)) < 4.0 * sd
    assert abs(st["e_abs"] / npk - w0 * (1.0 - math.exp(-tau))) < 4.0 * sd + 1e-12 * w0


def test_split_crossing_count_closed_form():
    """Pure absorber, beam along x through the block refined 2 levels deep: the package as
    emitted enters its birth cell, 8 level-2 cells and the root cell behind the block (10
    cells, split at the first level-2 cell, roulette at the last crossing); each of the N - 1
    new packages starts in that first level-2 cell, already counted, and enters the other 7
    and the root cell behind (8).  No event happens, so the total is exact whatever the
    roulette decides."""
    tree = gen.refined_block(2)
    dust = gen.Dust(np.array([1.0]), np.array([0.2]), np.array([0.0]), np.array([0.0]))
    o = oracle.Model(tree, dust)
    npk = 500
    src = [gen.Source(gen.SRC_BEAM, 0, pos=(0.3, 1.7, 2.2), dir=(1.0, 0.0, 0.0),
                      power=np.array([1.0]), packets=npk)]
    for n in (1, 2, 5):
        _, _, st, rec = o.trace(src, seed=4, split_n=n, rec_stride=1)
        assert st["crossings"] == npk * (10 + 8 * (n - 1)), (n, st["crossings"])
        assert np.all(rec["crossings"] == 10)
        if n > 1:
            assert st["splits"] == npk


def _per_level(o, e):
    lv = o.level_of_nodes()
    return np.array([e[lv == l].sum() for l in range(int(lv.max()) + 1)])


def test_split_unbiased_per_level():
    """Scattering cloud in an isotropic field: the absorbed energy per hierarchy level agrees
    in expectation with and without splitting (means over 8 independent seeds, within 4 combined
    standard errors)."""
    w = gen.c1("A", packets=6000)
    o = oracle.Model(w.trees[0], w.dusts[0])
    runs = {1: [], 4: []}
    for n in runs:
        for k in range(8):
            e, _, _, _ = o.trace(w.sources, seed=w.seed + 100 * k, split_n=n)
            runs[n].append(_per_level(o, e))
    a, b = np.array(runs[1]), np.array(runs[4])
    se = np.sqrt(a.var(axis=0, ddof=1) / len(a) + b.var(axis=0, ddof=1) / len(b))
    assert np.all(np.abs(a.mean(axis=0) - b.mean(axis=0)) < 4.0 * se)


def test_split_reduces_noise_in_refined_cells():
    """The paper's finding for the external field (Table 1): with the same number of emitted
    packages, splitting lowers the cell-by-cell noise in the deepest level.  Strongly scattering
    medium (albedo 0.9), block refined three levels deep in an isotropic field; noise is the
    relative RMS difference (Eq. 7 form) of 6 independent runs from their mean."""
    tree = gen.refined_block(3)
    dust = gen.Dust(np.array([1.0]), np.array([1.0]), np.array([0.9]), np.array([0.3]))
    o = oracle.Model(tree, dust)
    src = [gen.Source(gen.SRC_BACKGROUND, 0, power=np.array([1.0]), packets=3000)]
    deep = (o.level_of_nodes() == 3) & o.leaf_mask

    def noise(n):
        es = np.array([o.trace(src, seed=3 + 7 * k, split_n=n)[0][deep] for k in range(6)])
        ref = es.mean(axis=0)
        return float(np.sqrt(((es - ref) ** 2).mean() / (ref ** 2).mean()))
    n1, n4 = noise(1), noise(4)
    assert n4 < 0.85 * n1, (n1, n4)


# ------------------------------------------------------------------------------------------
# A coarser reading of "grid": all levels below d form one grid with their level-d ancestor
# (d = 1: the root grid and one grid per refined root cell's subtree).
# ------------------------------------------------------------------------------------------

def staircase_tree():
    """Three root cells along x; the middle one is refined, and of its children the one at
    bx = 1, by = bz = 0 is refined again.  A beam along x at y = z = 0.3 passes root cell 0,
    one level-1 cell, two level-2 cells and root cell 2."""
    refined = [np.array([1], dtype=np.int64), np.array([1], dtype=np.int64)]
    kids = [np.full(8, 1.0), np.full(8, 1.0)]
    return gen.TreeDesc(3, 1, 1, 1.0, np.full(3, 1.0), refined, kids)


def _beam(packets):
    return [gen.Source(gen.SRC_BEAM, 0, pos=(0.3, 0.3, 0.3), dir=(1.0, 0.0, 0.0),
                       power=np.array([1.0]), packets=packets)]


@pytest.mark.parametrize("n", [2, 3])
def test_split_depth_crossing_counts_closed_form(n):
    """Pure absorber, no events, so every history is the straight line through the staircase:
    root 0, level 1, level 2, level 2, root 2 (5 cells per package as emitted).
    * Every oct a grid (d = 0, and d = 2 >= the deepest level): the package splits entering
      level 1 (N - 1 new packages, each entering 3 more cells), all N split again entering
      level 2 (N (N - 1) new ones, 2 more cells each), and the N^2 are rouletted once leaving
      for root 2 (one level change of the grid level, 2 -> 0).
    * d = 1: one split entering the refined root cell (N - 1 new packages, 3 cells each); the
      step from level 1 into level 2 stays inside that grid, so no second split, and one
      roulette on leaving it."""
    dust = gen.Dust(np.array([1.0]), np.array([0.3]), np.array([0.0]), np.array([0.0]))
    o = oracle.Model(staircase_tree(), dust)
    npk = 400
    every = 5 + 3 * (n - 1) + 2 * n * (n - 1)
    for depth, per, splits in ((0, every, n + 1), (2, every, n + 1), (5, every, n + 1),
                               (1, 5 + 3 * (n - 1), 1)):
        _, _, st, rec = o.trace(_beam(npk), seed=8, split_n=n, rec_stride=1, split_depth=depth)
        assert st["crossings"] == npk * per, (depth, st["crossings"])
        assert st["splits"] == npk * splits, (depth, st["splits"])
        assert np.all(rec["crossings"] == 5)
        assert energy_gap(st) < 1e-12


def test_split_depth_at_or_below_the_deepest_level_is_the_oct_reading():
    """With d at least the deepest level every level is its own grid: results identical, bit
    for bit, to d = 0 (same splits, same roulette draws).  A random three-level tree in an
    isotropic field; with d = 1 the level changes inside refined root cells no longer split."""
    tree = gen.random_tree(np.random.default_rng(5), root=(4, 4, 4), max_level=3, p_refine=0.4)
    assert tree.n_levels == 3
    dust = gen.Dust(np.array([1.0]), np.array([0.5]), np.array([0.6]), np.array([0.2]))
    o = oracle.Model(tree, dust)
    src = [gen.Source(gen.SRC_BACKGROUND, 0, power=np.array([1.0]), packets=3000)]
    a = o.trace(src, seed=21, split_n=4, rec_stride=5)
    for deepest in (3, 7):
        b = o.trace(src, seed=21, split_n=4, rec_stride=5, split_depth=deepest)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[3], b[3])
        assert a[2]["splits"] == b[2]["splits"] > 0
    c = o.trace(src, seed=21, split_n=4, rec_stride=5, split_depth=1)
    assert 0 < c[2]["splits"] < a[2]["splits"]
    assert energy_gap(c[2]) < 1e-12


@pytest.mark.parametrize("n", [2, 4])
def test_split_depth_one_unbiased_beam_closed_form(n):
    """Pure absorber, beam through the staircase: the escaped energy has mean w0 exp(-tau)
    and, with one split and one roulette per package, variance e^-2tau (1 - 1/N) w0^2."""
    kappa = 0.3
    dust = gen.Dust(np.array([1.0]), np.array([kappa]), np.array([0.0]), np.array([0.0]))
    o = oracle.Model(staircase_tree(), dust)
    npk = 20000
    _, esc, st, _ = o.trace(_beam(npk), seed=13, split_n=n, split_depth=1)
    w0 = st["e_emit"] / npk
    tau = kappa * (3.0 - 0.3)
    mean = esc[0] / npk
    sd = w0 * math.exp(-tau) * math.sqrt((1.0 - 1.0 / n) / npk)
    assert abs(mean - w0 * math.exp(-tau)) < 4.0 * sd
    assert st["split_kills"] > 0


def test_split_depth_one_unbiased_per_level():
    """Scattering random tree in an isotropic field: with the coarser reading the absorbed energy
    per level agrees in expectation with the unsplit estimator (8 seeds each, 4 standard
    errors)."""
    tree = gen.random_tree(np.random.default_rng(5), root=(4, 4, 4), max_level=3, p_refine=0.4)
    dust = gen.Dust(np.array([1.0]), np.array([0.5]), np.array([0.6]), np.array([0.2]))
    o = oracle.Model(tree, dust)
    src = [gen.Source(gen.SRC_BACKGROUND, 0, power=np.array([1.0]), packets=4000)]
    a = np.array([_per_level(o, o.trace(src, seed=50 + 100 * k)[0]) for k in range(8)])
    b = np.array([_per_level(o, o.trace(src, seed=50 + 100 * k, split_n=4, split_depth=1)[0])
                  for k in range(8)])
    se = np.sqrt(a.var(axis=0, ddof=1) / len(a) + b.var(axis=0, ddof=1) / len(b))
    assert np.all(np.abs(a.mean(axis=0) - b.mean(axis=0)) < 4.0 * se)
