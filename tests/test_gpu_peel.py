"""GPU parity of the peel-off images (paper Sect. 2.4) against the oracle on the same seeded
inputs: the plain FP64 form follows the oracle's histories exactly, so its images agree per
pixel to FP64 rounding, marched to the border and with extinction tables; the FP32-local region
schedule agrees to its relative-RMS bar, below the Monte Carlo noise of the images."""
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


DIRS = np.array([[0.0, 0.0, 1.0], [0.3, -0.5, 0.81], [-1.0, 0.2, 0.1], [0.0, 1.0, 0.0]])


def _scattering_box():
    tree = gen.refined_block(2)
    rng = np.random.default_rng(4)
    # non-uniform densities so that the tables are an approximation
    tree.child_rho = [rng.uniform(0.3, 2.0, len(c)) for c in tree.child_rho]
    dust = gen.Dust(np.array([0.5, 1.0]), np.array([0.3, 0.2]), np.array([0.6, 0.5]),
                    np.array([0.5, 0.3]))
    src = [gen.Source(gen.SRC_BACKGROUND, 0, power=np.array([1.0, 2.0]), packets=20000),
           gen.Source(gen.SRC_POINT, 0, pos=(0.5, 3.2, 1.7), power=np.array([5.0, 1.0]), packets=20000)]
    return tree, dust, src


def _random_tree_case():
    rng = np.random.default_rng(17)
    tree = gen.random_tree(rng, (3, 4, 2), 3, 0.45, rho_range=(0.2, 1.5))
    dust = gen.Dust(np.array([1.0]), np.array([0.6]), np.array([0.7]), np.array([0.6]))
    src = [gen.Source(gen.SRC_BACKGROUND, 0, power=np.array([1.0]), packets=30000)]
    return tree, dust, src


def _ctx(tree, dust):
    ctx = rt.Context(0)
    m = ctx.build_tree(tree)
    ctx.set_dust(m, dust)
    return ctx


def rel_rms(a, ref):
    return float(np.sqrt(((a - ref) ** 2).sum() / (ref ** 2).sum()))


@pytest.mark.parametrize("case,split_n", [("box", 1), ("random", 1), ("random", 4)])
@pytest.mark.parametrize("tiles", [0, 3])
def test_peel_fp64_against_oracle(torch, case, tiles, split_n):
    """Per pixel |I_gpu - I_ora| <= 1e-9 |I_ora| + 1e-12 max I_ora; as many events peeled as
    the oracle scattered (with splitting: the events of the split-off packages too, peeled
    after each launch over their queue)."""
    tree, dust, src = _scattering_box() if case == "box" else _random_tree_case()
    kw = dict(rr_threshold=0.05, rr_prob=0.5, split_n=split_n)
    ora = oracle.Model(tree, dust)
    _, _, sto, _ = ora.trace(src, seed=9, peel=dict(n_obs=DIRS, npix=12, width=6.0, tiles=tiles), **kw)
    ctx = _ctx(tree, dust)
    img, st = ctx.peel_map(src, seed=9, n_obs=DIRS, npix=12, width=6.0, tiles=tiles,
                           precision=rt.FP64, **kw)
    ctx.close()
    g, o = img.cpu().numpy(), sto["peel_image"]
    assert st["peel_events"] == sto["scatterings"] > 0
    assert np.count_nonzero(o) > 0.25 * o.size
    tol = 1e-9 * np.abs(o) + 1e-12 * np.abs(o).max()
    bad = np.abs(g - o) > tol
    assert not bad.any(), (int(bad.sum()), float(np.max(np.abs(g - o) / np.maximum(np.abs(o), 1e-300))))


@pytest.mark.parametrize("tiles,per_cu", [(0, 0), (3, 0), (3, 16)])
def test_peel_fp32_regions_against_oracle(torch, tiles, per_cu):
    """Region schedule (also with small regions, many sweeps): relative RMS over all pixels
    <= 1e-3 and below the Monte Carlo noise of the oracle's images."""
    tree, dust, src = _scattering_box()
    peel = dict(n_obs=DIRS, npix=12, width=6.0, tiles=tiles)
    ora = oracle.Model(tree, dust)
    _, _, sto, _ = ora.trace(src, seed=9, peel=peel)
    _, _, stb, _ = ora.trace(src, seed=1009, peel=peel)
    ctx = _ctx(tree, dust)
    img, st = ctx.peel_map(src, seed=9, n_obs=DIRS, npix=12, width=6.0, tiles=tiles,
                           precision=rt.FP32_LOCAL, blocks_per_cu=per_cu)
    ctx.close()
    o = sto["peel_image"]
    err = rel_rms(img.cpu().numpy(), o)
    noise = rel_rms(stb["peel_image"], o) / math.sqrt(2.0)
    assert err <= 1e-3 and err < noise, (err, noise)
    assert abs(st["peel_events"] - sto["scatterings"]) <= 1e-3 * sto["scatterings"]


def test_peel_tables_change_little_and_are_built(torch):
    """The tabled images differ from the marched ones by the tile approximation only (a few
    per cent here), and the table build is timed."""
    tree, dust, src = _scattering_box()
    ctx = _ctx(tree, dust)
    a, sa = ctx.peel_map(src, seed=2, n_obs=DIRS, npix=12, width=6.0, tiles=0, precision=rt.FP64)
    b, sb = ctx.peel_map(src, seed=2, n_obs=DIRS, npix=12, width=6.0, tiles=4, precision=rt.FP64)
    ctx.close()
    d = rel_rms(b.cpu().numpy(), a.cpu().numpy())
    assert 0.0 < d < 0.05, d
    assert sb["table_ms"] > 0.0 and sa["table_ms"] == 0.0


def test_peel_event_buffer_overflow_is_an_error(torch):
    """A batch with more events than the buffer holds fails with the count; the context stays
    usable."""
    tree, dust, src = _scattering_box()
    ctx = _ctx(tree, dust)
    with pytest.raises(rt.RTError, match="event buffer"):
        ctx.peel_map(src, seed=2, n_obs=DIRS[:1], npix=8, precision=rt.FP64, event_buffer=16)
    img, st = ctx.peel_map(src, seed=2, n_obs=DIRS[:1], npix=8, precision=rt.FP64)
    assert st["peel_events"] > 16 and float(img.sum()) > 0.0
    ctx.close()


def test_peel_argument_errors(torch):
    tree, dust, src = _scattering_box()
    ctx = _ctx(tree, dust)
    bad = [dict(n_obs=np.zeros((17, 3)) + 1.0, npix=8),
           dict(n_obs=DIRS, npix=0),
           dict(n_obs=DIRS, npix=8, tiles=65),
           dict(n_obs=[[0.0, 0.0, 0.0]], npix=8),
           dict(n_obs=DIRS, npix=8, precision=rt.FP32_LOCAL, schedule=rt.SCHED_GLOBAL)]
    for kw in bad:
        with pytest.raises(rt.RTError):
            ctx.peel_map(src, seed=1, **kw)
    img, _ = ctx.peel_map(src, seed=1, n_obs=DIRS[:2], npix=8)
    assert float(img.sum()) > 0.0
    ctx.close()
