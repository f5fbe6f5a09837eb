"""Benchmark on one MI355X.  Prints one JSON line.

Default workload: the deep-hierarchy cloud (root 256^3, up to 5 levels, 1.13e8 nodes, 100
wavelengths, 1e7 packets per wavelength, dust temperatures, 512^2 maps toward the 8 body
diagonals), the largest configuration that fits one GPU.  A step is one pass of the whole path
over the resident model: trace all packets (FP32-local form, region schedule), reduce the
absorbed energy to FP64, solve the temperatures, render the maps.  The plain FP64 form and the
one-queue FP32-local form are timed on the same inputs, which splits the gain over the FP64
form into its schedule and precision parts.  The molecular cloud (root 64^3, 3 levels, 32
wavelengths, 3.2e8 packets) is measured the same way after it and reported under "cloud".
Before anything touches the GPU the oracle is timed on the host cores (cpu_baseline: one
thread; cpu_all_cores: one thread per core of the host's share, on one shared model).

--workload cloud: the molecular cloud alone.  --workload disc: the circumstellar disc (root
96x96x32, 6 levels, 50 wavelengths); the star is traced once before timing, and a step is one
Lambda-iteration step from those temperatures: trace the dust emission (3e7 packets per
wavelength), solve the temperatures of A_stars + A_dust.  --workload clouds: 64 uneven clouds,
16 wavelengths, 1e6 packets per (model, wavelength), all traced in one call; a step is that
trace.

--split-study (cloud and deep workloads) adds, after the timed steps, the package-splitting
study of Sect. 4.1 (Table 1): the radiation field at the wavelength nearest 4 um, traced 20
times with and 20 times without splitting (factor 4) from the same small number of packets,
once for the external field and once for a star embedded in the densest deepest cell; the RMS
difference per hierarchy level (Eq. 7) from the mean of all runs, normalised to the largest
value, and the time per run.  It is reported in "splitting" and is not part of the timed
steps (it is off by default so that a kernel profile of the default run covers the timed
steps only).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_CROSSING_FP32 = 12.0   # packed density/subgrid word 4 B + FP32 accumulator RMW 8 B
BYTES_PER_CROSSING_FP64 = 28.0   # FP64 density 8 B + child 4 B + FP64 accumulator RMW 16 B
HBM_PEAK_GBS = 8000.0
# VALU issue: 256 CUs x 4 SIMDs, one wave64 vector instruction per 4 cycles each (16 lanes per
# SIMD; no packed FP32), 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4.0

# HBM traffic of the region pass kernel per workload, from two rocprofv3 --pmc runs of one
# trace step (FETCH_SIZE, then WRITE_SIZE), each scaled by what the same counter reads for a
# 4 GiB device-to-device copy (fetch x2.0, write x1.0), per leaf crossing; its VALU
# wave-instructions per leaf crossing (SQ_INSTS_VALU) and lane utilisation
# (SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU)) in the same step, at the launch settings the
# autotuner picks for the workload (given explicitly to those runs).  Valid only for the kernel
# sources the counters were taken on.
PASS_TRAFFIC = {"sources": ["blocked.hip", "device.h", "internal.h"],
                "sha256": "14afdc5f6ed60dab4e9b5d223999d99594a2e9a37d0d6a85be91c99c12377c96",
                "per_workload": {
                    # profiles/blk_pass_kernel_deep_hierarchy_cloud.md
                    "deep": {"fetch_bytes_per_crossing": 10.9418, "write_bytes_per_crossing": 4.9506,
                             "valu_per_crossing": 2.8701, "lane_utilisation": 0.6084},
                    # profiles/blk_pass_kernel_molecular_cloud.md
                    "cloud": {"fetch_bytes_per_crossing": 10.8368, "write_bytes_per_crossing": 6.3967,
                              "valu_per_crossing": 4.2469, "lane_utilisation": 0.4659}}}


WORKLOADS = {
    "cloud": "molecular cloud: root 64^3, 3 levels, 32 wavelengths 0.1-1000 um, %d packets/"
             "wavelength (isotropic field), roulette 1e-3/0.9, dust temperatures, 256^2 maps "
             "toward +x,+y,+z at 32 wavelengths",
    "disc": "circumstellar disc: root 96x96x32, 6 levels, 50 wavelengths; one Lambda-iteration "
            "step: dust emission of T_0 (%d packets/wavelength), roulette 1e-3/0.9, FP64 "
            "temperatures of A_stars + A_dust",
    "clouds": "64 uneven clouds (roots 16^3-48^3, 1-4 levels), 16 wavelengths, %d packets per "
              "(model, wavelength), one trace call",
    "deep": "deep-hierarchy cloud: root 256^3, 5 levels (1.13e8 nodes, 1.0e8 leaves), 64 cores of "
            "central tau_V 1e3, 100 wavelengths, %d packets/wavelength, roulette 1e-3/0.9, dust "
            "temperatures, 512^2 maps toward the 8 body diagonals at 100 wavelengths",
}


def node_geometry(tree):
    """Level, leaf flag, density and integer coordinates (at the node's level) of every
    canonical node of a tree description: root cells in x-fastest order, then each level's octs
    in the ascending order of their parents, cell b = bx + 2 by + 4 bz within its oct."""
    import numpy as np
    nx, ny, nz = tree.nx, tree.ny, tree.nz
    idx = np.arange(nx * ny * nz, dtype=np.int64)
    coords = [np.stack([idx % nx, (idx // nx) % ny, idx // (nx * ny)], axis=1)]
    rho = [np.asarray(tree.root_rho, dtype=np.float64)]
    leaf = [np.ones(len(idx), dtype=bool)]
    b = np.arange(8)
    off = np.stack([b & 1, (b >> 1) & 1, (b >> 2) & 1], axis=1)
    for l, (ref, kids) in enumerate(zip(tree.refined, tree.child_rho)):
        leaf[l][ref] = False
        parent = coords[l][ref]
        coords.append((2 * parent[:, None, :] + off[None, :, :]).reshape(-1, 3))
        rho.append(np.asarray(kids, dtype=np.float64))
        leaf.append(np.ones(8 * len(ref), dtype=bool))
    level = np.concatenate([np.full(len(r), l, dtype=np.int32) for l, r in enumerate(rho)])
    return level, np.concatenate(leaf), np.concatenate(rho), np.concatenate(coords)


def split_study(rt, gen, w, kw32, runs=20, packets=1_000_000, split_n=4, lam_um=4.0):
    """Noise per hierarchy level (Eq. 7) with and without package splitting, Sect. 4.1.  The
    per-run fields stay on the GPU (20 x 2 runs of the deep cloud's 1e8 leaves fit easily)."""
    import numpy as np
    import torch
    tree, dust = w.trees[0], w.dusts[0]
    i = int(np.argmin(np.abs(np.log(dust.lambda_um / lam_um))))
    d1 = gen.Dust(dust.lambda_um[i:i + 1], dust.kappa_ext[i:i + 1], dust.albedo[i:i + 1],
                  dust.hg_g[i:i + 1])
    level, leaf, rho, coords = node_geometry(tree)
    # J ~ absorbed power / cell mass at one wavelength (kappa_abs is the same in every cell)
    mass = rho * 8.0 ** (-level.astype(np.float64))
    use = leaf & (mass > 0)
    deep = use & (level == level.max())
    k = np.flatnonzero(deep)[np.argmax(rho[deep])]
    star = tuple(float(c) for c in (coords[k] + 0.5) * 2.0 ** -int(level[k]))
    n_lev = int(level.max()) + 1
    dev = torch.device("cuda", 0)
    p_bg = float(w.sources[0].power[i])
    use_idx = torch.from_numpy(np.flatnonzero(use)).to(dev)
    # dimensionless: absorbed power per unit source power, per mean cell mass
    inv_mass = torch.from_numpy(mass[use].mean() / mass[use] / p_bg).to(dev)
    lv = torch.from_numpy(level[use].astype(np.int64)).to(dev)
    n_cells = torch.bincount(lv, minlength=n_lev).double()
    del level, leaf, rho, coords, mass, use, deep
    ctx = rt.Context(0)
    m = ctx.build_tree(tree)
    ctx.set_dust(m, d1)
    cases = {"external": [gen.Source(gen.SRC_BACKGROUND, m, power=np.array([p_bg]), packets=packets)],
             "internal": [gen.Source(gen.SRC_POINT, m, pos=star, power=np.array([p_bg]), packets=packets)]}
    kw = {k_: v for k_, v in kw32.items() if k_ != "sweep_graph"}
    out = {"wavelength_um": float(dust.lambda_um[i]), "packets": packets, "runs": runs,
           "split_n": split_n, "star_root_cell_units": star,
           "cells_per_level": [int(v) for v in n_cells.tolist()]}
    # three estimators: no splitting, every oct a grid, and the coarser reading in which a
    # refined root cell's whole subtree is one grid (split_depth 1)
    variants = {"none": (1, 0), "oct": (split_n, 0), "root_subtree": (split_n, 1)}
    for name, src in cases.items():
        js = {v: [] for v in variants}
        ms = {v: [] for v in variants}
        cr = {v: [] for v in variants}
        sp = {v: [] for v in variants}
        for r in range(runs):
            for v, (n, depth) in variants.items():
                res = ctx.trace_packets(src, seed=w.seed + 7919 * r, precision=rt.FP32_LOCAL,
                                        split_n=n, split_depth=depth, **kw)
                js[v].append((res["e_abs_node"][use_idx] * inv_mass).float())
                ms[v].append(res["stats"]["kernel_ms"])
                cr[v].append(res["stats"]["crossings"])
                sp[v].append(res["stats"]["splits"])
        ref = torch.stack([j for v in variants for j in js[v]]).double().mean(dim=0)
        noise = {}
        for v in variants:
            acc = torch.zeros(n_lev, dtype=torch.float64, device=dev)
            for j in js[v]:
                d2 = (j.double() - ref) ** 2
                acc += torch.sqrt(torch.bincount(lv, weights=d2, minlength=n_lev) / n_cells)
            noise[v] = (acc / len(js[v])).tolist()
        del js, ref
        top = max(max(noise[v]) for v in variants)
        t = {v: float(np.mean(ms[v])) for v in variants}
        out[name] = {
            "noise_per_level_split": [x / top for x in noise["oct"]],
            "noise_per_level_no_split": [x / top for x in noise["none"]],
            "noise_per_level_split_root_subtree": [x / top for x in noise["root_subtree"]],
            "ms_per_run_split": t["oct"], "ms_per_run_no_split": t["none"],
            "ms_per_run_split_root_subtree": t["root_subtree"],
            "crossings_per_run_split": float(np.mean(cr["oct"])),
            "crossings_per_run_no_split": float(np.mean(cr["none"])),
            "crossings_per_run_split_root_subtree": float(np.mean(cr["root_subtree"])),
            "splits_per_run": float(np.mean(sp["oct"])),
            "splits_per_run_root_subtree": float(np.mean(sp["root_subtree"])),
            # packets needed for equal noise scale as noise^2: speed-up at the deepest level
            "gain_deepest_level": (noise["none"][-1] / noise["oct"][-1]) ** 2 * t["none"] / t["oct"],
            "gain_deepest_level_root_subtree":
                (noise["none"][-1] / noise["root_subtree"][-1]) ** 2 * t["none"] / t["root_subtree"],
        }
    ctx.close()
    return out


def peel_study(rt, gen, w, kw32, workload, packets=1_000_000, runs=3, tiles=4, lam_um=0.55):
    """Peel-off toward 5 observers (Sect. 2.4; the paper times its accelerated peel-off this
    way): time per run of the plain trace, of the trace with the columns marched to the border,
    and with extinction tables; the tables' effect on the images against their noise."""
    import numpy as np
    import torch
    tree, dust = w.trees[0], w.dusts[0]
    i = int(np.argmin(np.abs(np.log(dust.lambda_um / lam_um))))
    d1 = gen.Dust(dust.lambda_um[i:i + 1], dust.kappa_ext[i:i + 1], dust.albedo[i:i + 1],
                  dust.hg_g[i:i + 1])
    s0 = w.sources[0]
    src = [gen.Source(s0.kind, 0, pos=s0.pos, dir=s0.dir, power=np.array([float(s0.power[i])]),
                      packets=packets)]
    if workload == "disc":
        el = np.radians(2.0)  # 2 degrees above the disc plane, five azimuths
        dirs = [[np.cos(el) * np.cos(a), np.cos(el) * np.sin(a), np.sin(el)]
                for a in np.radians([0.0, 72.0, 144.0, 216.0, 288.0])]
    else:
        dirs = [[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1], [1, -1, 0.5]]
    ctx = rt.Context(0)
    m = ctx.build_tree(tree)
    ctx.set_dust(m, d1)
    kw = {k_: v for k_, v in kw32.items() if k_ not in ("sweep_graph", "batch_packets")}
    kw.update(rr_threshold=w.rr_threshold, rr_prob=w.rr_prob, precision=rt.FP32_LOCAL,
              batch_packets=1 << 18)
    npix = 256

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, 1e3 * (time.perf_counter() - t0)
    fn_plain = lambda r_: ctx.trace_packets(src, seed=w.seed + r_, **kw)
    fn_peel = lambda r_, t_: ctx.peel_map(src, seed=w.seed + r_, n_obs=dirs, npix=npix, tiles=t_,
                                          event_buffer=1 << 26, **kw)
    fn_plain(99)
    fn_peel(99, 0)
    fn_peel(99, tiles)
    ms = {"plain": [], "marched": [], "tabled": []}
    imgs = {"marched": [], "tabled": []}
    events = 0
    for r_ in range(runs):
        ms["plain"].append(timed(lambda: fn_plain(r_))[1])
        (a, st), t_a = timed(lambda: fn_peel(r_, 0))
        (b, sb), t_b = timed(lambda: fn_peel(r_, tiles))
        ms["marched"].append(t_a)
        ms["tabled"].append(t_b)
        imgs["marched"].append(a.double().cpu().numpy())
        imgs["tabled"].append(b.double().cpu().numpy())
        events = st["peel_events"]
        table_ms = sb["table_ms"]
        print(f"# peel study: run {r_ + 1} of {runs} done", file=sys.stderr, flush=True)

    def rel(x, ref):
        return float(np.sqrt(((x - ref) ** 2).sum() / (ref ** 2).sum()))
    ref = imgs["marched"][0]
    out = {"wavelength_um": float(dust.lambda_um[i]), "packets": packets, "runs": runs,
           "observers": dirs if isinstance(dirs[0], list) else [list(map(float, d)) for d in dirs],
           "npix": npix, "tiles": tiles, "events_per_run": int(events),
           "ms_per_run": {k_: float(np.median(v)) for k_, v in ms.items()},
           "table_ms": float(table_ms),
           "peel_ms_marched": float(np.median(ms["marched"]) - np.median(ms["plain"])),
           "peel_ms_tabled": float(np.median(ms["tabled"]) - np.median(ms["plain"])),
           "speedup_total": float(np.median(ms["marched"]) / np.median(ms["tabled"])),
           "tables_rel_rms_vs_marched": rel(imgs["tabled"][0], ref),
           "noise_rel_rms": rel(imgs["marched"][1], ref) / float(np.sqrt(2.0)) if runs > 1 else None}
    ctx.close()
    return out


def ali_study(rt, gen, steps=24, ref_steps=60, packets=300_000):
    """Accelerated against plain Lambda iteration (Sect. 3.1, Eqs. 2 and 3) on an optically
    thick cube around a star (gen.thick_cube): the mass-weighted mean relative distance of the
    temperatures after k steps to a long accelerated run, and the time per step."""
    import numpy as np
    import torch
    w = gen.thick_cube(packets=packets)
    tree, dust = w.trees[0], w.dusts[0]
    level, leaf, rho, _ = node_geometry(tree)
    mass = (rho * 8.0 ** (-level.astype(np.float64)))[leaf]
    ctx = rt.Context(0)
    m = ctx.build_tree(tree)
    ctx.set_dust(m, dust)
    kw = dict(precision=rt.FP32_LOCAL)
    checkpoints = [k for k in (1, 2, 4, 8, 12, 16, 24, 32, 48) if k <= steps]

    def run(ali, ks):
        hist, ms = [], []
        for k in ks:  # every call starts again from the constant sources
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t_, _, _ = ctx.lambda_iterate(m, w.sources, seed=w.seed, dust_packets=packets, n_max=k,
                                          tol=0.0, ali=ali, **kw)
            torch.cuda.synchronize()
            ms.append(1e3 * (time.perf_counter() - t0))
            hist.append(t_.cpu().numpy()[leaf])
        return hist, ms
    ref = run(True, [ref_steps])[0][-1]
    out = {"model": "optically thick cube: root 16^3 refined once (32768 leaves), 12 wavelengths, "
                    "3000 K star at the centre",
           "packets_per_lambda": packets, "checkpoints": checkpoints,
           "reference": f"{ref_steps} accelerated steps"}
    for name, ali in (("plain", False), ("accelerated", True)):
        hist, ms = run(ali, checkpoints)
        dist = [float((mass * np.abs(h - ref) / ref).sum() / mass.sum()) for h in hist]
        out[name] = {"distance_to_reference": dist,
                     "ms_per_step": float((ms[-1] - ms[0]) / max(checkpoints[-1] - checkpoints[0], 1))}
    ctx.close()
    return out


def subiter_study(rt, gen, ref_steps=40, packets=200_000, frac=0.5, stall=0.8):
    """Subiterations (Sect. 3.1, 3.3, App. B) against whole-model iterations on a thin cloud with
    one dense core around a star (gen.core_cloud), in the FP64 form and in the FP32-local region
    schedule: after k steps, the mass-weighted mean relative distance of the temperatures to a
    long whole-model run (FP64 form), over all leaves and over the core's, against the cell
    crossings and the time spent.  The subiterations follow the automatic iteration
    (rt_subiter_run)."""
    import numpy as np
    import torch
    w = gen.core_cloud(packets=packets)
    tree, dust = w.trees[0], w.dusts[0]
    level, leaf, rho, _ = node_geometry(tree)
    mass = (rho * 8.0 ** (-level.astype(np.float64)))[leaf]
    core = (level > 0)[leaf]
    ctx = rt.Context(0)
    m = ctx.build_tree(tree)
    ctx.set_dust(m, dust)
    rr = dict(rr_threshold=w.rr_threshold, rr_prob=w.rr_prob)

    def dist(h, ref, sel):
        return float((mass[sel] * np.abs(h[sel] - ref[sel]) / ref[sel]).sum() / mass[sel].sum())

    ctx.subiter_begin(m, w.sources, seed=w.seed, **rr)
    for k in range(1, ref_steps + 1):
        t_, _, _ = ctx.subiter_step(m, -1, dust_packets=packets, seed=w.seed, iteration=k, **rr)
    ref = t_.cpu().numpy()[leaf]
    print("# subiteration study: reference done", file=sys.stderr, flush=True)
    checkpoints = [1, 2, 3, 4, 6, 8, 12, 16]
    res = {"model": "thin cloud 15^3 with one dense core refined 3 levels around a 5000 K star",
           "packets_per_lambda": packets, "frac": frac, "stall": stall, "checkpoints": checkpoints,
           "reference": f"{ref_steps} whole-model steps, FP64 form"}
    all_leaves = np.ones(len(ref), dtype=bool)
    forms = {"fp64": dict(precision=rt.FP64),
             "fp32_regions": dict(precision=rt.FP32_LOCAL, schedule=rt.SCHED_REGIONS)}
    for form, kw in forms.items():
        res[form] = {}
        for name in ("whole_model", "subiterations"):
            rows = {"crossings": [], "seconds": [], "distance_all": [], "distance_core": []}
            roots = None
            for n in checkpoints:
                ctx.subiter_begin(m, w.sources, seed=w.seed, **rr, **kw)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if name == "whole_model":
                    cross = 0
                    for k in range(1, n + 1):
                        t_, _, st = ctx.subiter_step(m, -1, dust_packets=packets, seed=w.seed, iteration=k,
                                                     **rr, **kw)
                        cross += st["crossings"]
                else:
                    t_, roots, _, cs = ctx.subiter_run(m, n, dust_packets=packets, seed=w.seed, frac=frac,
                                                       stall=stall, **rr, **kw)
                    cross = int(cs.sum())
                h = t_.cpu().numpy()[leaf]
                rows["seconds"].append(time.perf_counter() - t0)
                rows["crossings"].append(int(cross))
                rows["distance_all"].append(dist(h, ref, all_leaves))
                rows["distance_core"].append(dist(h, ref, core))
            rows["roots_of_longest_run"] = [int(r) for r in roots] if roots is not None else None
            res[form][name] = rows
        print(f"# subiteration study: {form} done", file=sys.stderr, flush=True)
    ctx.close()
    return res


def lambda_graph_study(rt, gen, kw32, packets=1_000_000, steps=6):
    """Lambda iteration on the circumstellar disc (Sect. 3.1 Eq. 2), FP32-local region schedule,
    with every step launched directly against every step after the first replayed from one
    captured HIP graph: time per step (the difference between a run of `steps` steps and a run
    of one, both from the star's trace) and the temperature difference between the two."""
    import numpy as np
    import torch
    w = gen.c3(packets=packets)
    tree, dust = w.trees[0], w.dusts[0]
    level, leaf, rho, _ = node_geometry(tree)
    mass = (rho * 8.0 ** (-level.astype(np.float64)))[leaf]
    ctx = rt.Context(0)
    m = ctx.build_tree(tree)
    ctx.set_dust(m, dust)
    base = {k_: v for k_, v in kw32.items() if k_ != "sweep_graph"}
    base.update(precision=rt.FP32_LOCAL, rr_threshold=w.rr_threshold, rr_prob=w.rr_prob)
    out = {"model": "circumstellar disc, root 96x96x32, 6 levels, 50 wavelengths",
           "dust_packets_per_lambda": packets, "steps": steps}
    temps = {}
    for name, g in (("direct", 0), ("graph", 1)):
        times = {}
        for n in (1, steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t_, nd, crit = ctx.lambda_iterate(m, w.sources, seed=w.seed, dust_packets=packets, n_max=n, tol=0.0,
                                              sweep_graph=g, **base)
            torch.cuda.synchronize()
            times[n] = time.perf_counter() - t0
        temps[name] = t_.cpu().numpy()[leaf]
        out[name] = {"ms_per_step": 1e3 * (times[steps] - times[1]) / (steps - 1),
                     "criteria": [float(c) for c in crit]}
        print(f"# Lambda-iteration graph study: {name} done", file=sys.stderr, flush=True)
    a, b = temps["direct"], temps["graph"]
    out["t_rel_diff_mass_weighted"] = float((mass * np.abs(a - b) / a).sum() / mass.sum())
    out["speedup"] = out["direct"]["ms_per_step"] / out["graph"]["ms_per_step"]
    ctx.close()
    return out


def pass_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in PASS_TRAFFIC["sources"]:
        with open(os.path.join(ROOT, "paper_1206_3710_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["cloud", "disc", "clouds", "deep"], default="deep")
    ap.add_argument("--packets", type=int, default=0,
                    help="packets per wavelength (0: 1e7 cloud and deep, 3e7 disc, 1e6 clouds)")
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--global-steps", type=int, default=1,
                    help="steps of the one-queue FP32-local form (schedule-vs-precision split)")
    ap.add_argument("--cloud-steps", type=int, default=5,
                    help="deep workload: timed steps of the molecular cloud kept beside it (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-packets", type=int, default=0,
                    help="oracle sample: packets per wavelength (0: 4096 deep, 2^18 cloud, 2^16 "
                         "disc and clouds)")
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="threads for the all-core oracle figure (1: skip it)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--refill", type=float, default=0.0)
    ap.add_argument("--schedule", type=int, default=0, help="0: regions, 1: one global queue")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--tail-park", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (it runs, untimed, unless launch parameters are given)")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file")
    ap.add_argument("--graph", action="store_true",
                    help="replay captured graphs of the sweeps (no per-launch durations)")
    ap.add_argument("--trace-only", action="store_true", help="time only the transport step")
    ap.add_argument("--split-study", action="store_true",
                    help="add the package-splitting noise study (cloud and deep workloads)")
    ap.add_argument("--ali-study", action="store_true",
                    help="add the accelerated-iteration convergence study (a thick cube)")
    ap.add_argument("--subiter-study", action="store_true",
                    help="add the subiteration study (a thin cloud with a dense core)")
    ap.add_argument("--lambda-graph-study", action="store_true",
                    help="add Lambda-iteration steps on the disc launched directly against replayed "
                         "from a captured graph")
    ap.add_argument("--peel-study", action="store_true",
                    help="add the peel-off timing study (cloud, disc and deep workloads)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="no effect: the 4 GiB device-to-device copy always runs first")
    return ap.parse_args()


def cpu_info():
    """CPU model (from /proc/cpuinfo), the processor count the OS reports and the count this
    process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    return {"model": model or platform.machine(), "nproc": os.cpu_count(), "affinity": affinity}


def cpu_baselines(a, gen, w, tree, dust, nl, threads_max=16):
    """The oracle on the host cores, before anything touches the GPU: one thread on a packet-id
    prefix of every wavelength (the reported baseline), then the same oracle in several threads
    on a prefix that many times longer, split into one packet range per thread.  The threads
    share the one oracle model (its trace only reads it) and each adds its deposits to an array
    of its own, allocated and touched before the clock starts."""
    import threading
    import numpy as np
    import oracle
    info = cpu_info()
    src0 = [gen.Source(w.sources[0].kind, 0, pos=w.sources[0].pos, power=w.sources[0].power,
                       packets=w.sources[0].packets)]
    what = {"cloud": "", "disc": " of the star", "clouds": " of the first model",
            "deep": ""}[a.workload]
    n1 = a.cpu_packets or {"deep": 4096, "cloud": 1 << 18, "disc": 1 << 16, "clouds": 1 << 16}[a.workload]
    n1 = min(n1, int(w.sources[0].packets))
    kw = dict(seed=w.seed, rr_threshold=w.rr_threshold, rr_prob=w.rr_prob)
    ora = oracle.Model(tree, dust)
    out = np.zeros(ora.n_nodes)
    out.fill(0.0)
    t2 = time.perf_counter()
    _, _, sto, _ = ora.trace(src0, pid_end=n1, e_abs_out=out, **kw)
    dc = time.perf_counter() - t2
    cpu = {"value": sto["crossings"] / dc, "unit": "cell-crossings/s", "cores": 1,
           "kind": "oracle",
           "sample": f"first {n1} packets{what} at each of the {nl} wavelengths "
                     f"({sto['crossings']} crossings, {dc:.1f} s, single thread, {info['model']})"}
    threads = min(a.cpu_threads, info["affinity"], threads_max)
    if threads <= 1:
        return cpu, None
    n_all = min(threads * n1, int(w.sources[0].packets))
    edges = [n_all * k // threads for k in range(threads + 1)]
    outs = [np.zeros(ora.n_nodes) for _ in range(threads)]
    for o_ in outs:
        o_.fill(0.0)
    cross = [0] * threads
    errors = []

    def work(k):
        try:
            _, _, st, _ = ora.trace(src0, pid_begin=edges[k], pid_end=edges[k + 1], e_abs_out=outs[k], **kw)
            cross[k] = st["crossings"]
        except Exception as e:  # reported below
            errors.append(e)
    th = [threading.Thread(target=work, args=(k,)) for k in range(threads)]
    t3 = time.perf_counter()
    for t_ in th:
        t_.start()
    for t_ in th:
        t_.join()
    d3 = time.perf_counter() - t3
    if errors:
        raise errors[0]
    cr = sum(cross)
    cpu_all = {"value": cr / d3, "unit": "cell-crossings/s", "cores": threads, "kind": "oracle",
               "nproc": info["nproc"], "affinity": info["affinity"],
               "sample": f"first {n_all} packets{what} at each of the {nl} wavelengths, one packet "
                         f"range per thread over {threads} threads sharing one model ({cr} "
                         f"crossings, {d3:.1f} s, {info['model']}; the host's CPU share for one "
                         f"GPU is 16 cores)"}
    return cpu, cpu_all


def load_workload(gen, name, packets):
    if name == "cloud":
        return gen.c2(packets=packets or 10_000_000)
    if name == "disc":
        return gen.c3(packets=packets or 30_000_000)
    if name == "deep":
        return gen.c5(packets=packets or 10_000_000)
    return gen.c4(packets=packets or 1_000_000)


def measure(a, rt, gen, torch, w, workload, steps, warmup, copy_gbs, fp64_steps, global_steps,
            explicit):
    """Time `steps` whole-path steps of one workload in the FP32-local region schedule (after
    `warmup` untimed ones), then the plain FP64 form and the one-queue FP32-local form on the same
    inputs; returns the bench record's body for it."""
    import numpy as np
    ctx = rt.Context(0)
    for t_, d_ in zip(w.trees, w.dusts):
        m = ctx.build_tree(t_)
        ctx.set_dust(m, d_)
    m = 0
    nl = w.dusts[0].n_lambda
    lam_all = list(range(nl))
    # launch parameters given on the command line are the FP32-local form's; the FP64 form
    # keeps its own defaults
    kw = dict(rr_threshold=w.rr_threshold, rr_prob=w.rr_prob)
    kw32 = dict(kw, block_size=a.block, blocks_per_cu=a.blocks_per_cu, refill_threshold=a.refill,
                schedule=a.schedule, chunk_packets=a.chunk, batch_packets=a.batch,
                tail_park=a.tail_park, sweep_graph=1 if a.graph else 0)
    if workload == "disc":
        # constant sources once (FP64 form), then every timed step re-emits from T_0
        a_stars = ctx.trace_packets(w.sources, seed=w.seed, iteration=0, precision=rt.FP64,
                                    **kw)["e_abs_node"]
        t0_disc = ctx.solve_temperature(m, a_stars, 2.0, 3000.0)
        dust_src = [gen.Source(gen.SRC_DUST, 0, packets=w.sources[0].packets)]

    tuned = None
    if not a.no_autotune and not explicit:
        # launch parameters from the autotuner (packet-id prefix of the workload, untimed)
        t_tune = time.perf_counter()
        if workload == "disc":
            ctx.set_temperature(m, t0_disc)
        tune_src = dust_src if workload == "disc" else w.sources
        frac = 0.25
        params, rate = ctx.autotune(tune_src, seed=w.seed, precision=rt.FP32_LOCAL,
                                    schedule=a.schedule, sample_fraction=frac,
                                    cache=a.tune_cache, rr_threshold=w.rr_threshold,
                                    rr_prob=w.rr_prob)
        tuned = dict(params, sample_fraction=frac, sample_crossings_per_s=rate,
                     seconds=time.perf_counter() - t_tune)
        kw32.update(params)

    def step(precision, it, extra=None):
        kwp = dict(kw32 if precision == rt.FP32_LOCAL else kw)
        if extra:
            kwp.update(extra)
        if workload == "disc":
            ctx.set_temperature(m, t0_disc)
            r = ctx.trace_packets(dust_src, seed=w.seed, iteration=1 + it, precision=precision, **kwp)
        else:
            r = ctx.trace_packets(w.sources, seed=w.seed, iteration=it, precision=precision, **kwp)
        t = time.perf_counter()
        out = {"stats": r["stats"], "e_abs": r["e_abs_node"]}
        if not a.trace_only:
            if workload in ("cloud", "deep"):
                ctx.solve_temperature(m, r["e_abs_node"], 2.0, 3000.0)
                for d in w.map_dirs:
                    ctx.render_map(m, d, w.map_npix, lam_all, precision=precision)
            elif workload == "disc":
                ctx.solve_temperature(m, a_stars + r["e_abs_node"], 2.0, 3000.0)
        torch.cuda.synchronize()
        out["post_s"] = time.perf_counter() - t
        return out

    e_warm = None
    for i in range(warmup):
        e_warm = step(rt.FP32_LOCAL, 1000 + i)["e_abs"]
        print(f"# {workload}: warm-up step {i + 1} of {warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    crossings = 0
    kernel_ms, main_ms, main_n, post = [], [], [], []
    e32 = None
    for i in range(steps):
        o = step(rt.FP32_LOCAL, i)
        if i == 0:
            e32 = o["e_abs"]
        crossings += o["stats"]["crossings"]
        kernel_ms.append(o["stats"]["kernel_ms"])
        main_ms.append(o["stats"]["main_ms"])
        main_n.append(o["stats"]["main_launches"])
        post.append(o["post_s"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"# {workload}: {steps} timed steps done ({dt:.1f} s)", file=sys.stderr, flush=True)
    value = crossings / dt
    k_avg = sum(kernel_ms) / len(kernel_ms) / 1e3
    cr_step = crossings / steps
    # dominant kernel: per-launch durations from HIP events on its own stream (summed by the
    # library), algorithmic bytes = crossings handled x bytes per crossing
    launches = sum(main_n) / steps
    bytes_per_launch = cr_step / launches * BYTES_PER_CROSSING_FP32
    if sum(main_ms) > 0:
        main_launch_s = sum(main_ms) / sum(main_n) / 1e3
        achieved = bytes_per_launch / main_launch_s / 1e9
    else:  # replayed sweep graphs report no per-launch durations
        main_launch_s, achieved = float("nan"), float("nan")
    counters = PASS_TRAFFIC["per_workload"].get(workload)
    traffic, measured_gbs, issue = None, None, None
    if counters and a.schedule == 0 and pass_sources_sha() == PASS_TRAFFIC["sha256"]:
        per_cross = counters["fetch_bytes_per_crossing"] + counters["write_bytes_per_crossing"]
        traffic = cr_step / launches * per_cross
        if main_launch_s == main_launch_s:
            measured_gbs = traffic / main_launch_s / 1e9
            # the limit the kernel actually meets: VALU issue (measured instructions per
            # crossing x crossings per second while the pass kernel runs)
            v = counters["valu_per_crossing"] * cr_step / launches / main_launch_s
            issue = {"unit": "VALU wave-instructions/s", "valu_per_crossing": counters["valu_per_crossing"],
                     "lane_utilisation": counters.get("lane_utilisation"),
                     "achieved": v, "peak": VALU_ISSUE_PEAK, "frac": v / VALU_ISSUE_PEAK}

    def rel_rms(x, ref):
        x, ref = x.double().cpu().numpy(), ref.double().cpu().numpy()
        return float(np.sqrt(((x - ref) ** 2).sum() / (ref ** 2).sum()))

    def other_form(precision, n_steps, extra, label):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        c_, k_, e_ = 0, [], None
        for i in range(n_steps):
            o = step(precision, i, extra)
            if i == 0:
                e_ = o["e_abs"]
            c_ += o["stats"]["crossings"]
            k_.append(o["stats"]["kernel_ms"])
        torch.cuda.synchronize()
        d_ = time.perf_counter() - t1
        print(f"# {workload}: {label} done ({d_:.1f} s)", file=sys.stderr, flush=True)
        ka = sum(k_) / len(k_) / 1e3
        return e_, {"crossings_per_s": c_ / d_, "ms_per_step": 1e3 * d_ / n_steps,
                    "trace_kernel_ms": 1e3 * ka, "trace_crossings_per_s": (c_ / n_steps) / ka}

    fp64, acc, one_queue, gain = None, None, None, None
    if fp64_steps > 0:
        e64, fp64 = other_form(rt.FP64, fp64_steps, None, "plain FP64 form")
        fp64["hbm_frac_algorithmic"] = (fp64["trace_crossings_per_s"] * BYTES_PER_CROSSING_FP64
                                        / 1e9 / HBM_PEAK_GBS)
        # same Philox streams (iteration 0) in both forms: the difference is the FP32-local
        # rounding; an independent realisation (the warm-up) gives the Monte Carlo noise
        acc = {"rel_rms_fp32_local_vs_fp64": rel_rms(e32, e64),
               "mc_noise_rel_rms": rel_rms(e_warm, e64) / float(np.sqrt(2.0)) if e_warm is not None else None,
               "definition": "sqrt(sum (E32 - E64)^2 / sum E64^2) over nodes, absorbed power per node"}
    if global_steps > 0 and a.schedule == 0:
        e_g, one_queue = other_form(rt.FP32_LOCAL, global_steps, {"schedule": 1, "sweep_graph": 0,
                                                                 "block_size": 0, "blocks_per_cu": 0,
                                                                 "refill_threshold": 0.0},
                                    "one-queue FP32-local form")
        one_queue["rel_rms_vs_fp64"] = rel_rms(e_g, e64) if fp64_steps > 0 else None
    if fp64 and one_queue:
        tr = cr_step / k_avg
        gain = {"definition": "trace crossings/s ratios on the same inputs: precision = one-queue "
                              "FP32-local form over the plain FP64 form (same one-packet-per-lane "
                              "walk over the whole tree); schedule = the region (grid-by-grid, "
                              "LDS) schedule over the one-queue form, both FP32-local",
                "precision": one_queue["trace_crossings_per_s"] / fp64["trace_crossings_per_s"],
                "schedule": tr / one_queue["trace_crossings_per_s"],
                "total": tr / fp64["trace_crossings_per_s"]}
    body = {
        "value": value,
        "ms_per_step": 1e3 * dt / steps,
        "steps": steps,
        "config": {"workload": WORKLOADS[workload] % w.sources[0].packets
                               + (" (trace only)" if a.trace_only else ""),
                   "nodes": sum(t_.n_nodes for t_ in w.trees),
                   "leaves": sum(t_.n_leaves for t_ in w.trees),
                   "packets_per_step": int(sum(s.packets for s in w.sources) * nl),
                   "crossings_per_step": cr_step},
        "trace_kernel_ms": 1e3 * k_avg,
        "trace_crossings_per_s": cr_step / k_avg,
        "post_trace_ms": 1e3 * sum(post) / len(post),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "measured_gbs": measured_gbs,
                     "copy_gbs": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs if copy_gbs else None,
                     "kernel": "blk_pass_kernel<%d>" % (kw32["block_size"] or 768) if a.schedule == 0
                               else "trace_fp32_kernel<%d>" % (kw32["block_size"] or 256),
                     "launches_per_step": launches, "avg_launch_ms": 1e3 * main_launch_s,
                     "bytes_per_crossing": BYTES_PER_CROSSING_FP32,
                     "limiter": "VALU issue (see issue): the HBM figure is the method's roofline, "
                                "the issue figure is what the kernel meets" if issue else None,
                     "issue": issue},
        "autotune": tuned,
        "fp64": fp64,
        "fp32_one_queue": one_queue,
        "gain": gain,
        "accuracy": acc,
    }
    ctx.close()
    return body, kw32


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only: the library has no multi-GPU "
                                   "path (--gpus must be 1)"}))
        sys.exit(2)
    import gen

    w = load_workload(gen, a.workload, a.packets)
    tree, dust = w.trees[0], w.dusts[0]
    cpu, cpu_all = None, None
    if not a.no_cpu_baseline:
        cpu, cpu_all = cpu_baselines(a, gen, w, tree, dust, dust.n_lambda)
        print("# CPU baselines done", file=sys.stderr, flush=True)

    import torch
    import paper_1206_3710_amd as rt
    # 4 GiB device-to-device copy: reads and writes exceed every cache level; its rate is the
    # measured bandwidth the roofline is also reported against, and its counters calibrate the
    # traffic figures
    src_t = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
    dst_t = torch.empty_like(src_t)
    dst_t.copy_(src_t)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    dst_t.copy_(src_t)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 2.0 * 4.0 * (1 << 30) / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del src_t, dst_t
    torch.cuda.empty_cache()
    explicit = a.block or a.blocks_per_cu or a.refill or a.chunk or a.batch or a.tail_park
    body, kw32 = measure(a, rt, gen, torch, w, a.workload, a.steps, a.warmup, copy_gbs, a.fp64_steps,
                         a.global_steps, explicit)

    extra = None
    if a.workload == "deep" and a.cloud_steps > 0:
        # the molecular cloud, the previous default workload, kept beside the headline
        del w
        wc = load_workload(gen, "cloud", 0)
        b2, _ = measure(a, rt, gen, torch, wc, "cloud", a.cloud_steps, 1, copy_gbs, 1, 1, explicit)
        extra = {k: b2[k] for k in ("value", "ms_per_step", "steps", "config", "trace_crossings_per_s",
                                    "roofline", "fp64", "fp32_one_queue", "gain", "accuracy")}
        del wc

    splitting = None
    if a.workload in ("cloud", "deep") and a.schedule == 0 and a.split_study:
        splitting = split_study(rt, gen, load_workload(gen, a.workload, a.packets), kw32)

    accel = None
    if a.schedule == 0 and a.ali_study:
        accel = ali_study(rt, gen)

    subiters = None
    if a.subiter_study:
        subiters = subiter_study(rt, gen)

    lgraph = None
    if a.schedule == 0 and a.lambda_graph_study:
        lgraph = lambda_graph_study(rt, gen, kw32)

    peeling = None
    if a.workload in ("cloud", "disc", "deep") and a.schedule == 0 and a.peel_study:
        peeling = peel_study(rt, gen, load_workload(gen, a.workload, a.packets), kw32, a.workload)

    res = {
        "metric": "cell-crossings/s (FP32-local form; FP64 form in fp64)",
        "value": body["value"],
        "unit": "cell-crossings/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": body["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": body["config"],
        "trace_kernel_ms": body["trace_kernel_ms"],
        "trace_crossings_per_s": body["trace_crossings_per_s"],
        "post_trace_ms": body["post_trace_ms"],
        "roofline": body["roofline"],
        "autotune": body["autotune"],
        "fp64": body["fp64"],
        "fp32_one_queue": body["fp32_one_queue"],
        "gain": body["gain"],
        "accuracy": body["accuracy"],
        "cpu_baseline": cpu,
        "cpu_all_cores": cpu_all,
        "cloud": extra,
        "splitting": splitting,
        "peel_off": peeling,
        "accelerated_iteration": accel,
        "subiterations": subiters,
        "lambda_graph": lgraph,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
