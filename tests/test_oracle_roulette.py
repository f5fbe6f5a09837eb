"""Pins of the oracle's Russian roulette at scattering events (paper Sect. 2.3: packages whose
weight falls below a threshold n are killed with probability p, and the survivors carry the
killed ones' expected weight).

The roulette must leave every expectation unchanged.  The pins check that on the oracle's own
packet records, against closed forms and against runs without the roulette:
  * in a pure scatterer nothing is absorbed, so every emitted unit of energy escapes (or is
    cut off at an event cap) in expectation, roulette or not;
  * every sub-threshold event kills a fraction p of the packages, and a survivor of k such events
    carries w0 / (1 - p)^k, which is the only survivor weight that keeps the expectation of a
    binary kill at the weight before it; above the threshold nothing happens;
  * on a strongly scattering refined cloud the absorbed energy per hierarchy level and the
    escaped energy agree in expectation with the unrouletted run.
A planted survivor factor 1/p, and a kill test with the comparison inverted, each fail these
pins (the last test builds both mistakes into CPU copies of the oracle)."""
import contextlib
import ctypes as C
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import gen
import oracle

ORACLE_DIR = os.path.dirname(os.path.abspath(oracle.__file__))


def scatter_cube(rho=0.5):
    """A uniform pure scatterer, root 4^3: optical depth 2 across, 1 from the centre."""
    tree = gen.TreeDesc(4, 4, 4, 1.0, np.full(64, rho), [], [])
    dust = gen.Dust(np.array([1.0]), np.array([1.0]), np.array([1.0]), np.array([0.3]))
    return oracle.Model(tree, dust)


def centre_star(n):
    return [gen.Source(gen.SRC_POINT, 0, pos=(2.0, 2.0, 2.0), power=np.array([1.0]), packets=n)]


def check_unbiased_in_pure_scatterer(p, n=200_000, seed=5):
    """Pure scatterer, roulette at every event, histories cut at their third event (truncated,
    before that event's roulette, so that every weight stays below w0 / (1 - p)^2 and the
    estimator's variance is bounded): the escaped plus truncated energy equals the emitted
    energy in expectation.  Returns (mean per emitted, its standard error)."""
    m = scatter_cube()
    _, _, st, rec = m.trace(centre_star(n), seed=seed, rr_threshold=1e30, rr_prob=p, rec_stride=1,
                            max_events=2)
    assert st["e_abs"] == 0.0
    assert st["kills"] > 0 and st["truncated"] > 0
    x = np.where(rec["status"] != 1, rec["w"], 0.0) * n   # escaped or truncated weight / w0
    mean, se = float(x.mean()), float(x.std() / math.sqrt(n))
    assert abs(mean - 1.0) < 4.0 * se, (mean, se)
    return mean, se


def check_kill_fraction_and_survivor_weight(p, n=100_000, seed=7):
    """Roulette at every event: kills / events is p within 4 sigma, and every escaped package
    that survived k events carries w0 / (1 - p)^k.  With the threshold at 2 w0 the roulette stops
    once a survivor's weight reaches 2 w0."""
    m = scatter_cube()
    w0 = 1.0 / n
    _, _, st, rec = m.trace(centre_star(n), seed=seed, rr_threshold=1e30, rr_prob=p, rec_stride=1)
    events = int(rec["events"].sum())
    killed = rec["status"] == 1
    assert int(killed.sum()) == st["kills"]
    frac = st["kills"] / events
    assert abs(frac - p) < 4.0 * math.sqrt(p * (1 - p) / events), (frac, p)
    esc = rec["status"] == 0
    k = rec["events"][esc].astype(np.float64)
    np.testing.assert_allclose(rec["w"][esc], w0 * (1.0 - p) ** -k, rtol=1e-12)
    # a killed package ends with the weight it had before the killing event: w0 / (1-p)^(k-1)
    kk = rec["events"][killed].astype(np.float64)
    np.testing.assert_allclose(rec["w"][killed], w0 * (1.0 - p) ** -(kk - 1.0), rtol=1e-12)
    # threshold 2 w0: survivors stop being rouletted once their weight is >= 2 w0
    _, _, st2, rec2 = m.trace(centre_star(n), seed=seed, rr_threshold=2.0, rr_prob=p, rec_stride=1)
    kmax = 0
    while (1.0 - p) ** -kmax < 2.0:
        kmax += 1
    esc2 = rec2["status"] == 0
    k2 = np.minimum(rec2["events"][esc2], kmax).astype(np.float64)
    np.testing.assert_allclose(rec2["w"][esc2], w0 * (1.0 - p) ** -k2, rtol=1e-12)
    assert np.all(rec2["events"][rec2["status"] == 1] <= kmax)
    return frac


@pytest.mark.parametrize("p", [0.3, 0.5])
def test_roulette_unbiased_in_pure_scatterer(p):
    check_unbiased_in_pure_scatterer(p)


@pytest.mark.parametrize("p", [0.3, 0.9])
def test_roulette_kill_fraction_and_survivor_weight(p):
    check_kill_fraction_and_survivor_weight(p)


def test_roulette_matches_no_roulette_per_level():
    """Strongly scattering refined cloud (albedo 0.9, the tiny two-level tree), external field:
    absorbed energy per hierarchy level, total absorbed and escaped energy, roulette on
    (threshold 0.9 w0, p = 0.9: about a third of the packages are killed) against off, 8 seeds
    each: equal within 4 combined standard errors."""
    w = gen.c1("A", packets=20_000)
    dust = gen.Dust(np.array([0.55]), np.array([1.0]), np.array([0.9]), np.array([0.6]))
    m = oracle.Model(w.trees[0], dust)
    lv = m.level_of_nodes()
    n_lev = int(lv.max()) + 1

    def runs(rr_t, rr_p):
        rows = []
        for s in range(8):
            e_abs, e_esc, st, _ = m.trace(w.sources, seed=1000 + s, rr_threshold=rr_t, rr_prob=rr_p)
            per_level = np.bincount(lv, weights=e_abs, minlength=n_lev)
            rows.append(np.concatenate([per_level, [st["e_abs"], float(e_esc.sum())]]) / st["e_emit"])
            if rr_p > 0:  # the roulette acts on a large part of the energy
                assert st["kills"] > 0.2 * st["packets"] and st["e_rr_gain"] > 0.1 * st["e_emit"]
        return np.array(rows)

    on, off = runs(0.9, 0.9), runs(0.0, 0.0)
    mean_on, mean_off = on.mean(axis=0), off.mean(axis=0)
    se = np.sqrt(on.var(axis=0, ddof=1) / len(on) + off.var(axis=0, ddof=1) / len(off))
    assert np.all(np.abs(mean_on - mean_off) < 4.0 * se), (mean_on, mean_off, se)


# ---------------------------------------------------------------------------------------
# planted mistakes: each must fail the pins above
# ---------------------------------------------------------------------------------------

MUTANTS = {
    "survivor factor 1/p": ("double nw = p->w / (1.0 - c->rr_p);", "double nw = p->w / c->rr_p;"),
    "inverted kill test": ("if (unif(x[0]) < c->rr_p) {", "if (unif(x[0]) >= c->rr_p) {"),
}


@contextlib.contextmanager
def mutant_oracle(tmp_dir, old, new):
    """Load a copy of the oracle with one source line replaced (the module's library handle is
    swapped for the duration)."""
    src = open(os.path.join(ORACLE_DIR, "oracle.c")).read()
    assert src.count(old) == 1, old
    os.makedirs(tmp_dir, exist_ok=True)
    with open(os.path.join(tmp_dir, "oracle.c"), "w") as f:
        f.write(src.replace(old, new))
    shutil.copy(os.path.join(ORACLE_DIR, "oracle.h"), tmp_dir)
    so = os.path.join(tmp_dir, "liboracle_mutant.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                           "-shared", "-o", so, os.path.join(tmp_dir, "oracle.c"), "-lm"])
    saved = (oracle._lib, oracle._SO, oracle.build)
    try:
        oracle._lib, oracle._SO = None, so
        oracle.build = lambda force=False: so
        assert oracle.lib()._name == so
        yield
    finally:
        oracle._lib, oracle._SO, oracle.build = saved


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_roulette_mistakes_fail_the_pins(name, tmp_path):
    old, new = MUTANTS[name]
    with mutant_oracle(str(tmp_path / "mutant"), old, new):
        with pytest.raises(AssertionError):
            check_unbiased_in_pure_scatterer(0.3, n=50_000)
        with pytest.raises(AssertionError):
            check_kill_fraction_and_survivor_weight(0.3, n=50_000)
    # the real oracle passes the same checks at that size
    check_unbiased_in_pure_scatterer(0.3, n=50_000)
    check_kill_fraction_and_survivor_weight(0.3, n=50_000)
