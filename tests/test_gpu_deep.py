"""GPU parity on the large deep-hierarchy cloud: root 256^3, 5 levels, 1.13e8 nodes (1.0e8
leaves), 64 dense cores reaching a central column tau_V of 1e3, 100 wavelengths, roulette on.

The tree is traced at its full size with 1e5 packets per wavelength; 10 packets per
wavelength are replayed one by one by the oracle from their packet ids (without deposit
arrays), and the two forms are compared with each other and against the Monte Carlo noise.
The full packet count (1e7 per wavelength) is the benchmark's."""
import math

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

rt = pytest.importorskip("paper_1206_3710_amd")

PACKETS = 100_000
SAMPLES = 10


@pytest.fixture(scope="module")
def deep():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = gen.c5(packets=PACKETS)
    print(f"deep cloud: {w.trees[0].n_nodes} nodes, {w.trees[0].n_leaves} leaves", flush=True)
    ctx = rt.Context(0)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, w.dusts[0])
    stride = PACKETS // SAMPLES
    kw = dict(seed=w.seed, rr_threshold=w.rr_threshold, rr_prob=w.rr_prob)
    r64 = ctx.trace_packets(w.sources, precision=rt.FP64, rec_stride=stride, **kw)
    r32 = ctx.trace_packets(w.sources, precision=rt.FP32_LOCAL, rec_stride=stride, **kw)
    r32b = ctx.trace_packets(w.sources, precision=rt.FP32_LOCAL, iteration=1, **kw)
    out = {k: {"stats": v["stats"], "records": v.get("records"),
               "e": v["e_abs_node"].cpu().numpy()} for k, v in
           (("r64", r64), ("r32", r32), ("r32b", r32b))}
    ctx.close()
    del r64, r32, r32b
    print("traced", flush=True)
    ora = oracle.Model(w.trees[0], w.dusts[0])
    nl = w.dusts[0].n_lambda
    reco = np.zeros(nl * SAMPLES, dtype=oracle.RECORD_DTYPE)
    for i in range(nl):
        for k in range(SAMPLES):
            j = k * stride
            _, _, _, rec = ora.trace(w.sources, pid_begin=j, pid_end=j + 1, lam_sel=i,
                                     rec_stride=1, deposits=False, **kw)
            reco[i * SAMPLES + k] = rec[i]
    print("replayed", flush=True)
    out["reco"] = reco
    return out


def _conserved(st, rel):
    lhs = st["e_emit"] + st["e_rr_gain"]
    rhs = st["e_abs"] + st["e_esc"] + st["e_killed"] + st["e_trunc"]
    assert abs(lhs - rhs) <= rel * lhs, (lhs, rhs)


def test_deep_fp64_sampled_packets_exact(deep):
    rg, reco = deep["r64"]["records"], deep["reco"]
    for f in ("status", "crossings", "events", "node", "birth"):
        assert np.array_equal(rg[f], reco[f]), f
    np.testing.assert_allclose(rg["w"], reco["w"], rtol=1e-9)
    st = deep["r64"]["stats"]
    assert st["packets"] == 100 * PACKETS and st["truncated"] == 0
    _conserved(st, 1e-9)


def test_deep_fp32_local_sampled_packets(deep):
    """Same bar as on the molecular cloud: 99 % of the sampled packets reproduce the replay's
    fate, counts and end node, with the weight within 2^-24 (8 n + n^2 / 2)."""
    rg, reco = deep["r32"]["records"], deep["reco"]
    assert np.array_equal(rg["birth"], reco["birth"])
    same = ((rg["status"] == reco["status"]) & (rg["crossings"] == reco["crossings"])
            & (rg["events"] == reco["events"]) & (rg["node"] == reco["node"]))
    assert same.mean() >= 0.99, same.mean()
    steps = rg["crossings"].astype(np.float64) + rg["events"] + 1.0
    tol = 2.0 ** -24 * (8.0 * steps + 0.5 * steps * steps) * np.abs(reco["w"])
    bad = same & (np.abs(rg["w"] - reco["w"]) > tol)
    assert not bad.any(), (rg[bad], reco[bad])
    st = deep["r32"]["stats"]
    assert st["packets"] == 100 * PACKETS and st["truncated"] == 0
    _conserved(st, 1e-4)


def test_deep_fp32_local_error_below_noise(deep):
    e64, e32, e32b = deep["r64"]["e"], deep["r32"]["e"], deep["r32b"]["e"]

    def rel_rms(a, ref):
        return float(np.sqrt(((a - ref) ** 2).sum() / (ref ** 2).sum()))
    err, noise = rel_rms(e32, e64), rel_rms(e32b, e32) / math.sqrt(2.0)
    print(f"deep cloud FP32-local vs FP64: {err:.3e}, noise {noise:.3e}")
    assert err <= 1e-3 and err < noise
    c64, c32 = deep["r64"]["stats"]["crossings"], deep["r32"]["stats"]["crossings"]
    assert abs(c32 - c64) <= 1e-3 * c64


def test_deep_global_key_sort_matches_lds_sort():
    """Per-wavelength output on the deep tree with 3 wavelengths: 3 x (about 9100 regions) keys
    are too many for the sweeps' LDS counters, so the queue is sorted with global atomics.  The
    histories (sampled records) equal those of the wavelength-integrated trace of the same
    packets, whose keys fit in LDS; the absorbed energy agrees to the FP32 summation order, and
    the per-wavelength arrays sum to it."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = gen.c5(packets=20_000)
    d = w.dusts[0]
    sel = [30, 50, 70]
    d3 = gen.Dust(d.lambda_um[sel], d.kappa_ext[sel], d.albedo[sel], d.hg_g[sel])
    src = [gen.Source(s.kind, s.model, s.pos, s.dir, np.asarray(s.power)[sel], s.packets)
           for s in w.sources]
    ctx = rt.Context(0)
    m = ctx.build_tree(w.trees[0])
    ctx.set_dust(m, d3)
    kw = dict(seed=w.seed, rr_threshold=w.rr_threshold, rr_prob=w.rr_prob, precision=rt.FP32_LOCAL,
              rec_stride=97)
    a = ctx.trace_packets(src, **kw)
    b = ctx.trace_packets(src, per_lambda=True, **kw)
    for f in ("status", "crossings", "events", "node", "birth", "w"):
        assert np.array_equal(a["records"][f], b["records"][f]), f
    ea, eb = a["e_abs_node"].cpu().numpy(), b["e_abs_node"].cpu().numpy()
    assert np.sqrt(((eb - ea) ** 2).sum() / (ea ** 2).sum()) < 1e-6
    el = b["e_abs_lambda_node"].cpu().numpy().reshape(3, -1)
    assert np.abs(el.sum(axis=0) - eb).max() <= 1e-12 * np.abs(eb).max()
    assert a["stats"]["crossings"] == b["stats"]["crossings"]
    ctx.close()
