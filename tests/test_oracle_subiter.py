"""Pins of the oracle's subiterations on complete subtrees (paper Sect. 3.1 and App. B): the
per-level arrays split the absorbed energy by the shallowest level a package visited, a
subiteration keeps its packages and its emission inside its subtree, and steps on the whole
model are the plain Lambda iteration."""
import numpy as np

import gen
import oracle
from tests import brute


def _dust(albedo, n=6):
    lam = np.logspace(0, 3, n)
    return gen.Dust(lam, 5.0 * lam ** -1.2, np.full(n, albedo), np.full(n, 0.2))


def _small_case():
    lam = np.logspace(-1, 3, 10)
    kap = 3.0 * (lam / 0.55) ** -1.6
    alb = np.clip(0.5 * (1 - np.log10(lam / 0.1) / 4), 0, 0.5)
    dust = gen.Dust(lam, kap, alb, alb.copy())
    tree = gen.refined_block(2)
    rng = np.random.default_rng(6)
    tree.child_rho = [rng.uniform(0.5, 2.0, len(c)) for c in tree.child_rho]
    nu = brute.CL / (lam * 1e-4)
    star = [gen.Source(gen.SRC_POINT, 0, pos=(2.1, 1.9, 2.05), power=1e-2 * brute.planck_nu(nu, 5000.0),
                       packets=3000)]
    return tree, dust, star


def test_whole_model_steps_are_the_lambda_iteration():
    """Subiterations whose subtree is the whole model give the Lambda iteration's temperatures,
    and the per-level arrays add up to the absorbed energy."""
    tree, dust, star = _small_case()
    o = oracle.Model(tree, dust)
    hs, _, stats = oracle.subiterate(o, star, seed=8, schedule=[-1, -1, -1], dust_packets=3000)
    hl, _, _ = oracle.lambda_iterate(o, star, seed=8, n_fixed=3, dust_packets=3000)
    for a, b in zip(hs, hl):
        np.testing.assert_allclose(a, b, rtol=1e-12)
    t = hl[1]
    a, _, st, _ = o.trace([gen.Source(gen.SRC_DUST, 0, packets=3000)], seed=8, iteration=2, t_node=t,
                          level_arrays=True)
    np.testing.assert_allclose(st["e_lvl"].sum(axis=0), a, rtol=1e-12, atol=1e-300)


def test_arrays_follow_the_shallowest_level():
    """A star in a level-2 cell of a block refined two levels deep (no level-1 leaves): without
    scattering its packages never return, so the level-2 array holds everything deposited in
    level-2 cells, the level-0 array everything outside, the level-1 array nothing; with strong
    scattering packages come back into the block after visiting level 0."""
    tree = gen.refined_block(2)
    src = [gen.Source(gen.SRC_POINT, 0, pos=(1.6, 1.7, 2.3), power=np.full(6, 1.0), packets=4000)]
    for albedo, returns in ((0.0, False), (0.9, True)):
        o = oracle.Model(tree, _dust(albedo))
        lv = o.level_of_nodes()
        a, _, st, _ = o.trace(src, seed=2, level_arrays=True)
        e = st["e_lvl"]
        for m in range(3):
            assert np.all(e[m][lv < m] == 0.0)        # never deeper than the cell itself
        assert np.all(e[1] == 0.0)
        np.testing.assert_allclose(e[0][lv == 0], a[lv == 0], rtol=1e-12)
        if returns:
            assert e[0][lv == 2].sum() > 0.0
        else:
            assert np.all(e[0][lv == 2] == 0.0)
            np.testing.assert_allclose(e[2][lv == 2], a[lv == 2], rtol=1e-12)
    # the external field enters through the root grid: everything is level 0, even where the
    # boundary cells are refined
    bg = [gen.Source(gen.SRC_BACKGROUND, 0, power=np.full(6, 1.0), packets=3000)]
    fine = gen.uniform_refined_tree((2, 2, 2), 1, rho=1.0, cell_cm=1.0)
    a, _, st, _ = oracle.Model(fine, _dust(0.5)).trace(bg, seed=3, level_arrays=True)
    assert a.sum() > 0.0
    np.testing.assert_allclose(st["e_lvl"][0], a, rtol=1e-12, atol=1e-300)


def test_subtree_keeps_emission_and_packages_inside():
    """Subiteration below the refined root cell (1, 1, 1): only its leaves emit, every deposit
    stays in it at levels below its own, and emitted = absorbed + left."""
    tree = gen.refined_block(2)
    o = oracle.Model(tree, _dust(0.6))
    root = 1 + 4 * (1 + 4 * 1)
    assert o.child[root] >= 0
    inside = o.subtree_mask(root)
    lv = o.level_of_nodes()
    assert inside.sum() == 8 + 64 and np.all(lv[inside] >= 1)
    t = np.where(o.leaf_mask, 60.0, 0.0)
    a, _, st, _ = o.trace([gen.Source(gen.SRC_DUST, 0, packets=5000)], seed=4, t_node=t,
                          level_arrays=True, self_absorption=True, subtree=root)
    assert np.all(a[~inside] == 0.0) and a[inside].sum() > 0.0
    assert np.all(st["e_emit_node"][~inside] == 0.0)
    assert np.all(st["e_lvl"][0] == 0.0)
    lhs = st["e_emit"]
    rhs = st["e_abs"] + st["e_esc"] + st["e_killed"] + st["e_trunc"] - st["e_rr_gain"]
    assert abs(lhs - rhs) <= 1e-12 * lhs


def test_subiteration_changes_only_its_subtree():
    """A step on a subtree leaves every temperature outside it as it was."""
    tree, dust, star = _small_case()
    o = oracle.Model(tree, dust)
    root = 2 + 4 * (1 + 4 * 2)
    hs, _, _ = oracle.subiterate(o, star, seed=8, schedule=[-1, root], dust_packets=3000)
    inside = o.subtree_mask(root)
    assert np.array_equal(hs[2][~inside], hs[1][~inside])
    assert np.any(hs[2][inside & o.leaf_mask] != hs[1][inside & o.leaf_mask])


def test_accelerated_whole_model_steps_are_the_accelerated_iteration():
    """Subiterations with the accelerated iteration (Eq. 3 inside the subtree) whose subtree is
    the whole model give the accelerated Lambda iteration's temperatures: the cell's arrays sum
    to A_dust, and its own-level array holds the self-absorption the diagonal operator removes."""
    tree, dust, star = _small_case()
    o = oracle.Model(tree, dust)
    hs, _, _ = oracle.subiterate(o, star, seed=8, schedule=[-1, -1, -1], dust_packets=3000, ali=True)
    hl, _, _ = oracle.lambda_iterate(o, star, seed=8, n_fixed=3, dust_packets=3000, ali=True)
    for a, b in zip(hs, hl):
        np.testing.assert_allclose(a, b, rtol=1e-12)


def test_accelerated_subiterations_converge_faster_in_a_thick_core():
    """A star inside a dense refined root cell (density 20 against 0.05 outside): after a
    whole-model step and two steps on the core's subtree, the accelerated form has heated the
    core more than the plain one (both start from the same first step and rise toward the same
    fixed point from below), and neither changes a temperature outside the subtree in its
    subtree steps."""
    lam = np.logspace(-1, 3, 10)
    dust = gen.Dust(lam, 3.0 * (lam / 0.55) ** -1.6, np.clip(0.5 * (1 - np.log10(lam / 0.1) / 4), 0, 0.5),
                    np.clip(0.5 * (1 - np.log10(lam / 0.1) / 4), 0, 0.5))
    core = 1 + 4 * (1 + 4 * 1)
    tree = gen.TreeDesc(4, 4, 4, 1.0, np.full(64, 0.05), [np.array([core]), np.arange(8)],
                        [np.full(8, 20.0), np.full(64, 20.0)])
    nu = brute.CL / (lam * 1e-4)
    star = [gen.Source(gen.SRC_POINT, 0, pos=(1.55, 1.45, 1.6), power=1e-2 * brute.planck_nu(nu, 5000.0),
                       packets=1000)]
    o = oracle.Model(tree, dust)
    sched = [-1, core, core]
    hp, _, _ = oracle.subiterate(o, star, seed=3, schedule=sched, dust_packets=1000)
    ha, _, _ = oracle.subiterate(o, star, seed=3, schedule=sched, dust_packets=1000, ali=True)
    inside = o.subtree_mask(core)
    leaf = o.leaf_mask
    assert ha[1][inside & leaf].mean() > hp[1][inside & leaf].mean()
    assert ha[-1][inside & leaf].mean() > 1.03 * hp[-1][inside & leaf].mean()
    for h in (hp, ha):
        for k in (2, 3):
            assert np.array_equal(h[k][~inside], h[k - 1][~inside])


def _nested_corner():
    """Root 2^3 of side 1 and density 1: root cell 0 refined once, and its level-1 child 7
    (x, y, z in [0.5, 1)) refined again; every other child of root cell 0 is a level-1 leaf."""
    return gen.TreeDesc(2, 2, 2, 1.0, np.ones(8), [np.array([0]), np.array([7])],
                        [np.ones(8), np.ones(8)])


def test_split_packages_file_under_the_level_of_the_package_they_split_from():
    """With package splitting (every level change splits or roulettes) a split-off package keeps
    the shallowest level visited of the package it split from:
      * a pure absorber lit by a star in a level-1 leaf: the packages entering the level-2 cells
        split there, and everything deposited in level-2 cells lands in the level-1 array (none
        in the level-0 or level-2 arrays: a straight path that leaves the root cell never comes
        back into it);
      * the external field, split on every entry into a deeper cell: everything is level 0."""
    tree = _nested_corner()
    absorber = gen.Dust(np.array([1.0]), np.array([1.0]), np.array([0.0]), np.array([0.0]))
    o = oracle.Model(tree, absorber)
    lv = o.level_of_nodes()
    star = [gen.Source(gen.SRC_POINT, 0, pos=(0.2, 0.3, 0.25), power=np.array([1.0]), packets=6000)]
    a, _, st, _ = o.trace(star, seed=5, level_arrays=True, split_n=4)
    e = st["e_lvl"]
    assert st["splits"] > 100 and st["split_kills"] > 0
    assert a[lv == 2].sum() > 0.0
    np.testing.assert_allclose(e[1][lv == 2], a[lv == 2], rtol=1e-12)
    assert np.all(e[2] == 0.0) and np.all(e[0][lv >= 1] == 0.0)
    np.testing.assert_allclose(e.sum(axis=0), a, rtol=1e-12, atol=1e-300)
    bg = [gen.Source(gen.SRC_BACKGROUND, 0, power=np.array([1.0]), packets=6000)]
    o2 = oracle.Model(tree, _dust(0.7, n=1))
    a2, _, st2, _ = o2.trace(bg, seed=6, level_arrays=True, split_n=4)
    assert st2["splits"] > 100 and a2[lv == 2].sum() > 0.0
    np.testing.assert_allclose(st2["e_lvl"][0], a2, rtol=1e-12, atol=1e-300)
    assert np.all(st2["e_lvl"][1:] == 0.0)


def test_split_subiterations_agree_with_unsplit_ones():
    """Subiterations with package splitting estimate the same temperatures as without: after a
    whole-model step and a subtree step the mass-weighted mean |T_split - T| / T over the leaves
    is within the spread between two unsplit runs with different keys (times 2)."""
    tree, dust, star = _small_case()
    o = oracle.Model(tree, dust)
    root = 2 + 4 * (1 + 4 * 2)
    sched = [-1, root]
    ha, _, _ = oracle.subiterate(o, star, seed=8, schedule=sched, dust_packets=3000)
    hb, _, _ = oracle.subiterate(o, star, seed=9, schedule=sched, dust_packets=3000)
    hs, _, sts = oracle.subiterate(o, star, seed=10, schedule=sched, dust_packets=3000, split_n=4)
    assert sts[0]["splits"] > 0  # (the subtree holds one level of leaves only)
    leaf = o.leaf_mask
    mass = o.node_rho() * 8.0 ** -o.level_of_nodes().astype(float)

    def diff(x, y):
        return float((mass[leaf] * np.abs(x[leaf] - y[leaf]) / y[leaf]).sum() / mass[leaf].sum())
    assert diff(hs[-1], ha[-1]) < 2.0 * diff(hb[-1], ha[-1]), (diff(hs[-1], ha[-1]), diff(hb[-1], ha[-1]))


# ---------------------------------------------------------------------------------------
# energy flow from each grid to its parent (Sect. 3.3)
# ---------------------------------------------------------------------------------------

def _beam_row():
    """Root 4 x 1 x 1 of side 1 and density 1 (pure absorber, kappa 1): root cell 1 (x in
    [1, 2)) refined once, and its child (0, 0, 0) (x in [1, 1.5), y, z in [0, 0.5)) refined
    again."""
    tree = gen.TreeDesc(4, 1, 1, 1.0, np.ones(4), [np.array([1]), np.array([0])],
                        [np.ones(8), np.ones(8)])
    dust = gen.Dust(np.array([1.0]), np.array([1.0]), np.array([0.0]), np.array([0.0]))
    return oracle.Model(tree, dust)


def test_flux_of_a_beam_closed_form():
    """A beam along +x at y = z = 0.37 from x = 0.5 leaves the subtree of the level-1 refined
    cell at x = 1.5 and that of root cell 1 at x = 2, each once per packet, with the weight it
    has there: N w0 exp(-1.0) and N w0 exp(-1.5).  Along -x from x = 1.2 it leaves both at
    x = 1 in the same crossing (N w0 exp(-0.2) each), then root cell 0 (a leaf: no subtree) and
    the model."""
    o = _beam_row()
    inner = o.offsets[1] + 0            # root cell 1's child (0, 0, 0): the refined level-1 cell
    assert o.child[1] >= 0 and o.child[inner] >= 0
    n = 500
    src = [gen.Source(gen.SRC_BEAM, 0, pos=(0.5, 0.37, 0.37), dir=(1.0, 0.0, 0.0),
                      power=np.array([1.0]), packets=n)]
    _, _, st, _ = o.trace(src, seed=1, flux=True)
    f = st["e_flux"]
    np.testing.assert_allclose(f[inner], np.exp(-1.0), rtol=1e-13)
    np.testing.assert_allclose(f[1], np.exp(-1.5), rtol=1e-13)
    others = np.ones(o.n_nodes, dtype=bool)
    others[[1, inner]] = False
    assert np.all(f[others] == 0.0)
    src = [gen.Source(gen.SRC_BEAM, 0, pos=(1.2, 0.37, 0.37), dir=(-1.0, 0.0, 0.0),
                      power=np.array([1.0]), packets=n)]
    _, _, st, _ = o.trace(src, seed=1, flux=True)
    f = st["e_flux"]
    np.testing.assert_allclose(f[[1, inner]], np.exp(-0.2), rtol=1e-13)
    assert np.all(f[others] == 0.0)


def test_flux_out_of_the_iterated_subtree_is_what_leaves_it():
    """In a subtree step every package that leaves the subtree is ended there: the flow out of
    the subtree's root equals the escaped energy, no refined cell outside it sees any flow, and
    the flows of the refined cells inside it are positive."""
    tree = gen.refined_block(2)
    o = oracle.Model(tree, _dust(0.6))
    root = 1 + 4 * (1 + 4 * 1)
    inside = o.subtree_mask(root)
    t = np.where(o.leaf_mask, 60.0, 0.0)
    _, _, st, _ = o.trace([gen.Source(gen.SRC_DUST, 0, packets=4000)], seed=4, t_node=t,
                          level_arrays=True, subtree=root, flux=True)
    f = st["e_flux"]
    assert f[root] > 0.0
    assert abs(f[root] - st["e_esc"]) <= 1e-12 * st["e_esc"]
    refined = ~o.leaf_mask
    outside = refined & ~inside
    outside[root] = False
    assert np.all(f[outside] == 0.0)
    assert np.all(f[refined & inside] > 0.0)


def test_automatic_iteration_follows_its_rules():
    """The oracle's automatic iteration on a thin cloud with a dense core around a star: the
    first step takes the whole model; a repeated subtree whose largest imbalance did not drop
    below `stall` of its previous value is replaced by the whole model; with the flow tracking
    on, a step below r whose outflow changed by more than flux_frac of what r's parent absorbs
    makes the next step include that parent; the temperatures equal those of the explicit
    schedule of the same roots."""
    w = gen.core_cloud(packets=20000)
    o = oracle.Model(w.trees[0], w.dusts[0])
    kw = dict(seed=w.seed, n_steps=6, dust_packets=20000, frac=0.5, stall=0.8,
              rr_threshold=w.rr_threshold, rr_prob=w.rr_prob)
    h0, r0 = oracle.subiterate_auto(o, w.sources, flux_frac=0.0, **kw)
    assert r0[0] == -1
    for a, b in zip(r0[:-1], r0[1:]):   # no subtree twice in a row here (the stall rule)
        assert not (a >= 0 and a == b)
    hs, _, _ = oracle.subiterate(o, w.sources, w.seed, r0, 20000, rr_threshold=w.rr_threshold,
                                 rr_prob=w.rr_prob)
    for a, b in zip(h0, hs):
        np.testing.assert_allclose(a, b, rtol=1e-13)
    h1, r1 = oracle.subiterate_auto(o, w.sources, flux_frac=0.02, **kw)
    par = oracle.canonical_parents(o)
    tagged_steps = [k for k in range(1, len(r1)) if r1[k] >= 0 and r1[k - 1] >= 0 and r1[k] == par[r1[k - 1]]]
    assert tagged_steps, r1   # a parent grid taken because its inflow from the child changed
    assert r1 != r0
