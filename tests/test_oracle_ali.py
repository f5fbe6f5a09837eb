"""Pins of the oracle's accelerated Lambda iteration with a diagonal operator (paper Sect. 3.1,
Eq. 3): the self-absorption tally in one-cell and two-cell models, where it is fixed exactly,
the algebra of the update at the fixed point, and faster convergence than the plain Lambda
iteration toward the same temperatures."""
import numpy as np

import gen
import oracle
from tests import brute


def _dust(albedo):
    lam = np.logspace(0, 3, 8)
    kap = 5.0 * (lam / 1.0) ** -1.5
    return gen.Dust(lam, kap, np.full(8, albedo), np.full(8, 0.3))


def _dust_source(packets):
    return [gen.Source(gen.SRC_DUST, 0, packets=packets)]


def test_single_cell_absorbs_only_its_own_emission():
    """One root cell: every deposit of a dust packet happens in its birth cell before its first
    crossing (which is its escape), so the tally equals the whole absorbed energy; the energy
    emitted per birth cell is the emitted total."""
    tree = gen.TreeDesc(1, 1, 1, 1.0, np.array([2.0]), [], [])
    o = oracle.Model(tree, _dust(0.5))
    a, _, st, _ = o.trace(_dust_source(20000), seed=3, t_node=np.array([80.0]), self_absorption=True)
    assert a[0] > 0
    assert abs(st["e_self"][0] - a[0]) <= 1e-12 * a[0]
    assert abs(st["e_emit_node"][0] - st["e_emit"]) <= 1e-12 * st["e_emit"]


def test_two_cells_returns_are_not_self_absorption():
    """Two root cells, only cell 0 warm (cell 1 at 0 K emits nothing).  Without scattering a
    packet that has left cell 0 never comes back, so cell 0's absorption is all its own first
    visit; with strong scattering some packets return after their first crossing."""
    tree = gen.TreeDesc(2, 1, 1, 1.0, np.array([2.0, 2.0]), [], [])
    t = np.array([80.0, 0.0])
    for albedo, returns in ((0.0, False), (0.9, True)):
        o = oracle.Model(tree, _dust(albedo))
        a, _, st, _ = o.trace(_dust_source(20000), seed=4, t_node=t, self_absorption=True)
        assert st["e_emit_node"][1] == 0.0 and st["e_self"][1] == 0.0
        if returns:
            assert st["e_self"][0] < (1.0 - 1e-3) * a[0]
        else:
            assert abs(st["e_self"][0] - a[0]) <= 1e-12 * a[0]


def test_update_keeps_the_fixed_point():
    """If the absorbed power already balances the emission at T (A_stars + A_dust = E(T)) and
    the cells emitted E(T), the accelerated update returns E(T) whatever part of it was
    self-absorbed, so the temperature is unchanged."""
    rng = np.random.default_rng(2)
    tree = gen.uniform_refined_tree((2, 2, 2), 1, rho=1.0, cell_cm=1.0)
    o = oracle.Model(tree, _dust(0.2))
    leaf = o.leaf_mask
    t = np.where(leaf, rng.uniform(20.0, 300.0, o.n_nodes), 0.0)
    e = o.emission_all(t)
    a_stars = e * rng.uniform(0.0, 0.6, o.n_nodes)
    a_dust = e - a_stars
    e_self = a_dust * rng.uniform(0.0, 0.99, o.n_nodes)
    a_new = oracle.ali_step_absorbed(a_stars, a_dust, e_self, e)
    np.testing.assert_allclose(a_new[leaf], e[leaf], rtol=1e-12)
    t_new = o.solve_temperature(a_new)
    np.testing.assert_allclose(t_new[leaf], t[leaf], rtol=1e-9)


def test_ali_converges_faster():
    """Optically thick cube around a star: both iterations raise the temperatures toward the
    same equilibrium from below; after 8 steps the accelerated one is well ahead."""
    lam = np.logspace(0, 3, 12)
    dust = gen.Dust(lam, 30.0 * lam ** -1.5, np.full(12, 0.1), np.zeros(12))
    tree = gen.uniform_refined_tree((4, 4, 4), 1, rho=1.0, cell_cm=1.0)
    nu = brute.CL / (lam * 1e-4)
    star = [gen.Source(gen.SRC_POINT, 0, pos=(2.05, 1.95, 2.02),
                       power=brute.planck_nu(nu, 3000.0), packets=6000)]
    o = oracle.Model(tree, dust)
    leaf = o.leaf_mask
    mean = {}
    for ali in (False, True):
        hist, _, _ = oracle.lambda_iterate(o, star, seed=5, n_fixed=8, dust_packets=6000, ali=ali)
        mean[ali] = [float(np.mean(h[leaf])) for h in hist]
        assert all(b > a for a, b in zip(mean[ali][:-1], mean[ali][1:]))  # rising
    assert mean[True][-1] > 1.08 * mean[False][-1], (mean[True][-1], mean[False][-1])


def test_self_absorption_with_splitting_stays_below_emission():
    """With package splitting the branches split off a package start counting their cells at 0
    where they split; only the package as emitted, before its first crossing, is in its birth
    cell.  Per cell the tally then never exceeds what the cell's own packets absorbed or emitted,
    and it equals the unsplit tally in expectation (the first segment is never split)."""
    lam = np.logspace(0, 3, 8)
    dust = gen.Dust(lam, 5.0 * lam ** -1.2, np.full(8, 0.6), np.full(8, 0.3))
    tree = gen.uniform_refined_tree((4, 4, 4), 2, rho=1.0, cell_cm=1.0)
    # refine only part of the cube, so that crossings into deeper leaves (splits) happen
    o = oracle.Model(tree, dust)
    rng = np.random.default_rng(12)
    leaf = o.leaf_mask
    t = np.where(leaf, rng.uniform(30.0, 120.0, o.n_nodes), 0.0)
    rb = gen.refined_block(2, n=4, rho=1.0)
    ob = oracle.Model(rb, dust)
    tb = np.where(ob.leaf_mask, rng.uniform(30.0, 120.0, ob.n_nodes), 0.0)
    for model, temps in ((o, t), (ob, tb)):
        _, _, s1, _ = model.trace(_dust_source(4000), seed=9, t_node=temps, self_absorption=True)
        _, _, s4, _ = model.trace(_dust_source(4000), seed=9, t_node=temps, self_absorption=True,
                                  split_n=4)
        assert np.all(s4["e_self"] <= s4["e_emit_node"] * (1.0 + 1e-12))
        # the package as emitted deposits the same before its first crossing with or without
        # splitting (a split happens only at a crossing)
        np.testing.assert_allclose(s4["e_self"], s1["e_self"], rtol=1e-12, atol=0.0)
    assert s4["splits"] > 0
