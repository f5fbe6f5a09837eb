"""The allocation-free map entry point (rt_render_map_noalloc) through the C ABI against
rt_render_map, which runs the same kernels from context buffers: maps and crossing counts must
be identical, on two calls in a row (the second smaller, so that the shared scratch array's
previous contents would show), in both precisions; inputs beyond the scratch limit and host
images are refused without changing what a following call computes."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

rt = pytest.importorskip("paper_1206_3710_amd")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def test_render_map_noalloc_matches_render_map(torch):
    w = gen.c1("A", packets=20_000)
    dust = gen.shared_dust(24, kappa_v=1.0)
    src = [gen.Source(gen.SRC_BACKGROUND, 0, power=gen.background_spectrum(dust.lambda_um) * 1e12,
                      packets=20_000)]
    ctx = rt.Context(0)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, dust)
    r = ctx.trace_packets(src, seed=w.seed, precision=rt.FP32_LOCAL)
    ctx.solve_temperature(m, r["e_abs_node"], 2.0, 3000.0)
    cases = [  # first call: every wavelength (two passes of the kernel), then a smaller one
        dict(n_obs=(1.0, 0.3, 0.2), npix=64, lam=list(range(24)), precision=rt.FP64),
        dict(n_obs=(0.0, 0.0, 1.0), npix=24, lam=[3, 17, 0, 9, 22], precision=rt.FP32_LOCAL),
    ]
    for c in cases:
        ref, cr_ref = ctx.render_map(m, c["n_obs"], c["npix"], c["lam"], precision=c["precision"])
        img, cr = ctx.render_map_noalloc(m, c["n_obs"], c["npix"], c["lam"], precision=c["precision"])
        assert cr == cr_ref and cr > 0
        a, b = img.cpu().numpy(), ref.cpu().numpy()
        assert float(b.max()) > 0.0
        assert np.array_equal(a, b)
    # beyond the scratch limit, and a host image: refused
    with pytest.raises(rt.RTError) as e:
        ctx.render_map_noalloc(m, (1.0, 0.0, 0.0), 8, [0] * 513)
    assert e.value.code == rt.RT_EINVAL
    with pytest.raises(rt.RTError) as e:
        ctx.render_map_noalloc(m, (1.0, 0.0, 0.0), 8, [0], image=np.zeros((1, 8, 8)))
    assert e.value.code == rt.RT_EINVAL
    c = cases[1]
    ref, cr_ref = ctx.render_map(m, c["n_obs"], c["npix"], c["lam"], precision=c["precision"])
    img, cr = ctx.render_map_noalloc(m, c["n_obs"], c["npix"], c["lam"], precision=c["precision"])
    assert cr == cr_ref and np.array_equal(img.cpu().numpy(), ref.cpu().numpy())
    ctx.close()


def test_render_map_noalloc_needs_current_device_copies(torch):
    """After rt_build_tree the device copies are stale until an allocating call uploads them."""
    w = gen.c1("A", packets=1000)
    ctx = rt.Context(0)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, w.dusts[0])
    ctx.set_temperature(m, np.full(w.trees[0].n_nodes, 20.0))
    with pytest.raises(rt.RTError) as e:
        ctx.render_map_noalloc(m, (1.0, 0.0, 0.0), 8, [0])
    assert e.value.code == rt.RT_ESTATE
    ref, _ = ctx.render_map(m, (1.0, 0.0, 0.0), 8, [0])
    img, _ = ctx.render_map_noalloc(m, (1.0, 0.0, 0.0), 8, [0])
    assert np.array_equal(img.cpu().numpy(), ref.cpu().numpy())
    ctx.close()
