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
