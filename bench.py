"""Benchmark on one MI355X.  Prints one JSON line.

Default workload: the molecular cloud (root 64^3, up to 3 levels, 32 wavelengths, 1e7 packets
per wavelength, dust temperatures, 256^2 maps toward 3 axes).  A step is one pass of the whole
path over the resident model: trace all packets (FP32-local form, region schedule), reduce the
absorbed energy to FP64, solve the temperatures, render the maps.  The plain FP64 form is timed
on the same inputs for comparison.

--workload disc: the circumstellar disc (root 96x96x32, 6 levels, 50 wavelengths); the star is
traced once before timing, and a step is one Lambda-iteration step from those temperatures:
trace the dust emission (3e7 packets per wavelength), solve the temperatures of A_stars +
A_dust.  --workload clouds: 64 uneven clouds, 16 wavelengths, 1e6 packets per (model,
wavelength), all traced in one call; a step is that trace.

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

# HBM traffic of the region pass kernel, from two rocprofv3 --pmc runs of one trace step
# (FETCH_SIZE, then WRITE_SIZE), each scaled by what the same counter reads for a 4 GiB
# device-to-device copy (fetch x2.0, write x1.0), per leaf crossing; and its VALU wave-instructions
# per leaf crossing (SQ_INSTS_VALU of the same step), at the launch settings the autotuner picked
# in that run.  Valid only for the kernel sources the counters were taken on.
PASS_TRAFFIC = {"sources": ["blocked.hip", "device.h", "internal.h"],
                "sha256": "8be39f5aa2ab71ef8f102d850368f1f8ad6375446d60393939c6f6fbb6a00fb0",
                "fetch_bytes_per_crossing": 11.005, "write_bytes_per_crossing": 6.535,
                "valu_per_crossing": 5.34}


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
    for name, src in cases.items():
        js, ms, cr, sp = {1: [], split_n: []}, {1: [], split_n: []}, {1: [], split_n: []}, []
        for r in range(runs):
            for n in (1, split_n):
                res = ctx.trace_packets(src, seed=w.seed + 7919 * r, precision=rt.FP32_LOCAL,
                                        split_n=n, **kw)
                js[n].append((res["e_abs_node"][use_idx] * inv_mass).float())
                ms[n].append(res["stats"]["kernel_ms"])
                cr[n].append(res["stats"]["crossings"])
                if n > 1:
                    sp.append(res["stats"]["splits"])
        ref = torch.stack(js[1] + js[split_n]).double().mean(dim=0)
        noise = {}
        for n in (1, split_n):
            acc = torch.zeros(n_lev, dtype=torch.float64, device=dev)
            for j in js[n]:
                d2 = (j.double() - ref) ** 2
                acc += torch.sqrt(torch.bincount(lv, weights=d2, minlength=n_lev) / n_cells)
            noise[n] = (acc / len(js[n])).tolist()
        del js, ref
        top = max(max(noise[1]), max(noise[split_n]))
        t1, tn = float(np.mean(ms[1])), float(np.mean(ms[split_n]))
        out[name] = {
            "noise_per_level_split": [v / top for v in noise[split_n]],
            "noise_per_level_no_split": [v / top for v in noise[1]],
            "ms_per_run_split": tn, "ms_per_run_no_split": t1,
            "crossings_per_run_split": float(np.mean(cr[split_n])),
            "crossings_per_run_no_split": float(np.mean(cr[1])),
            "splits_per_run": float(np.mean(sp)),
            # packets needed for equal noise scale as noise^2: speed-up at the deepest level
            "gain_deepest_level": (noise[1][-1] / noise[split_n][-1]) ** 2 * t1 / tn,
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
    ap.add_argument("--workload", choices=["cloud", "disc", "clouds", "deep"], default="cloud")
    ap.add_argument("--packets", type=int, default=0,
                    help="packets per wavelength (0: 1e7 cloud and deep, 3e7 disc, 1e6 clouds)")
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-packets", type=int, default=1 << 18,
                    help="oracle sample: packets per wavelength")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="processes for the all-core oracle figure (1: skip it)")
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
    ap.add_argument("--peel-study", action="store_true",
                    help="add the peel-off timing study (cloud, disc and deep workloads)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="no effect: the 4 GiB device-to-device copy always runs first")
    return ap.parse_args()


_ORA = {}


def _oracle_init(tree, dust):
    import oracle
    _ORA["model"] = oracle.Model(tree, dust)


def _oracle_chunk(args):
    src, seed, rr_t, rr_p, b, e = args
    _, _, st, _ = _ORA["model"].trace(src, seed=seed, rr_threshold=rr_t, rr_prob=rr_p,
                                      pid_begin=b, pid_end=e)
    return st["crossings"]


def cpu_baselines(a, gen, w, tree, dust, nl):
    """The oracle on the host cores: one thread on a packet prefix (the reported baseline), and
    the same oracle in one process per core on a prefix 16 times longer.  Runs before anything
    touches the GPU (the worker processes are started fresh, not forked)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    import oracle
    src0 = [gen.Source(w.sources[0].kind, 0, pos=w.sources[0].pos, power=w.sources[0].power,
                       packets=w.sources[0].packets)]
    what = {"cloud": "", "disc": " of the star", "clouds": " of the first model",
            "deep": ""}[a.workload]
    cpu_name = platform.processor() or platform.machine()
    ora = oracle.Model(tree, dust)
    t2 = time.perf_counter()
    _, _, sto, _ = ora.trace(src0, seed=w.seed, rr_threshold=w.rr_threshold,
                             rr_prob=w.rr_prob, pid_end=a.cpu_packets)
    dc = time.perf_counter() - t2
    del ora
    cpu = {"value": sto["crossings"] / dc, "unit": "cell-crossings/s", "cores": 1,
           "kind": "oracle",
           "sample": f"first {a.cpu_packets} packets{what} at each of the {nl} wavelengths "
                     f"({sto['crossings']} crossings, {dc:.1f} s, single thread, {cpu_name})"}
    workers = min(a.cpu_workers, os.cpu_count() or 1)
    if workers <= 1:
        return cpu, None
    n_all = min(16 * a.cpu_packets, int(w.sources[0].packets))
    edges = [n_all * k // (4 * workers) for k in range(4 * workers + 1)]
    tasks = [(src0, w.seed, w.rr_threshold, w.rr_prob, edges[k], edges[k + 1])
             for k in range(4 * workers) if edges[k + 1] > edges[k]]
    # a pool whose workers die raises instead of waiting
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"), initializer=_oracle_init,
                             initargs=(tree, dust)) as pool:
        list(pool.map(_oracle_chunk, [(src0, w.seed, w.rr_threshold, w.rr_prob, 0, 1)] * workers))
        t3 = time.perf_counter()
        cr = sum(pool.map(_oracle_chunk, tasks))
        d3 = time.perf_counter() - t3
    cpu_all = {"value": cr / d3, "unit": "cell-crossings/s", "cores": workers, "kind": "oracle",
               "sample": f"first {n_all} packets{what} at each of the {nl} wavelengths, "
                         f"{len(tasks)} packet ranges over {workers} processes ({cr} crossings, "
                         f"{d3:.1f} s, {cpu_name})"}
    return cpu, cpu_all


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "bench.py runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import gen

    if a.workload == "cloud":
        w = gen.c2(packets=a.packets or 10_000_000)
    elif a.workload == "disc":
        w = gen.c3(packets=a.packets or 30_000_000)
    elif a.workload == "deep":
        w = gen.c5(packets=a.packets or 10_000_000)
    else:
        w = gen.c4(packets=a.packets or 1_000_000)
    tree, dust = w.trees[0], w.dusts[0]
    cpu, cpu_all = None, None
    if not a.no_cpu_baseline:
        cpu, cpu_all = cpu_baselines(a, gen, w, tree, dust, dust.n_lambda)

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
    ctx = rt.Context(0)
    for t_, d_ in zip(w.trees, w.dusts):
        m = ctx.build_tree(t_)
        ctx.set_dust(m, d_)
    m = 0
    nl = dust.n_lambda
    lam_all = list(range(nl))
    kw = dict(rr_threshold=w.rr_threshold, rr_prob=w.rr_prob, block_size=a.block,
              blocks_per_cu=a.blocks_per_cu, refill_threshold=a.refill)
    kw32 = dict(kw, schedule=a.schedule, chunk_packets=a.chunk, batch_packets=a.batch,
                tail_park=a.tail_park, sweep_graph=1 if a.graph else 0)
    if a.workload == "disc":
        # constant sources once (FP64 form), then every timed step re-emits from T_0
        a_stars = ctx.trace_packets(w.sources, seed=w.seed, iteration=0, precision=rt.FP64,
                                    **kw)["e_abs_node"]
        t0_disc = ctx.solve_temperature(m, a_stars, 2.0, 3000.0)
        dust_src = [gen.Source(gen.SRC_DUST, 0, packets=w.sources[0].packets)]

    tuned = None
    explicit = a.block or a.blocks_per_cu or a.refill or a.chunk or a.batch or a.tail_park
    if not a.no_autotune and not explicit:
        # launch parameters from the autotuner (packet-id prefix of the workload, untimed)
        t_tune = time.perf_counter()
        if a.workload == "disc":
            ctx.set_temperature(m, t0_disc)
        tune_src = dust_src if a.workload == "disc" else w.sources
        params, rate = ctx.autotune(tune_src, seed=w.seed, precision=rt.FP32_LOCAL,
                                    schedule=a.schedule, sample_fraction=0.125,
                                    cache=a.tune_cache, rr_threshold=w.rr_threshold,
                                    rr_prob=w.rr_prob)
        tuned = dict(params, sample_crossings_per_s=rate, seconds=time.perf_counter() - t_tune)
        kw32.update(params)

    def step(precision, it):
        kwp = kw32 if precision == rt.FP32_LOCAL else kw
        if a.workload == "disc":
            ctx.set_temperature(m, t0_disc)
            r = ctx.trace_packets(dust_src, seed=w.seed, iteration=1 + it, precision=precision, **kwp)
        else:
            r = ctx.trace_packets(w.sources, seed=w.seed, iteration=it, precision=precision, **kwp)
        t = time.perf_counter()
        out = {"stats": r["stats"], "e_abs": r["e_abs_node"]}
        if not a.trace_only:
            if a.workload in ("cloud", "deep"):
                ctx.solve_temperature(m, r["e_abs_node"], 2.0, 3000.0)
                for d in w.map_dirs:
                    ctx.render_map(m, d, w.map_npix, lam_all, precision=precision)
            elif a.workload == "disc":
                ctx.solve_temperature(m, a_stars + r["e_abs_node"], 2.0, 3000.0)
        out["post_s"] = time.perf_counter() - t
        return out

    e_warm = None
    for i in range(a.warmup):
        e_warm = step(rt.FP32_LOCAL, 1000 + i)["e_abs"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    crossings = 0
    kernel_ms = []
    main_ms, main_n = [], []
    post = []
    for i in range(a.steps):
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
    value = crossings / dt
    k_avg = sum(kernel_ms) / len(kernel_ms) / 1e3
    cr_step = crossings / a.steps
    # dominant kernel: per-launch durations from HIP events on its own stream (summed by the
    # library), algorithmic bytes = crossings handled x bytes per crossing
    launches = sum(main_n) / a.steps
    bytes_per_launch = cr_step / launches * BYTES_PER_CROSSING_FP32
    if sum(main_ms) > 0:
        main_launch_s = sum(main_ms) / sum(main_n) / 1e3
        achieved = bytes_per_launch / main_launch_s / 1e9
    else:  # replayed sweep graphs report no per-launch durations
        main_launch_s, achieved = float("nan"), float("nan")
    traffic = None
    issue = None
    if a.workload == "cloud" and a.schedule == 0 and pass_sources_sha() == PASS_TRAFFIC["sha256"]:
        traffic = cr_step / launches * (PASS_TRAFFIC["fetch_bytes_per_crossing"]
                                        + PASS_TRAFFIC["write_bytes_per_crossing"])
        # the limit the kernel actually meets: VALU issue (measured instructions per crossing x
        # crossings per second while the pass kernel runs)
        if main_launch_s == main_launch_s:
            v = PASS_TRAFFIC["valu_per_crossing"] * cr_step / launches / main_launch_s
            issue = {"unit": "VALU wave-instructions/s", "valu_per_crossing": PASS_TRAFFIC["valu_per_crossing"],
                     "achieved": v, "peak": VALU_ISSUE_PEAK, "frac": v / VALU_ISSUE_PEAK}

    # plain FP64 form on the same inputs
    fp64 = None
    if a.fp64_steps > 0:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        c64 = 0
        k64 = []
        for i in range(a.fp64_steps):
            o = step(rt.FP64, i)
            if i == 0:
                e64 = o["e_abs"]
            c64 += o["stats"]["crossings"]
            k64.append(o["stats"]["kernel_ms"])
        torch.cuda.synchronize()
        d64 = time.perf_counter() - t1
        k64a = sum(k64) / len(k64) / 1e3
        # same Philox streams (iteration 0) in both forms: the difference is the FP32-local
        # rounding; an independent realisation (the warm-up) gives the Monte Carlo noise
        def rel_rms(x, ref):
            x, ref = x.double().cpu().numpy(), ref.double().cpu().numpy()
            return float(np.sqrt(((x - ref) ** 2).sum() / (ref ** 2).sum()))
        acc = {"rel_rms_fp32_local_vs_fp64": rel_rms(e32, e64),
               "mc_noise_rel_rms": rel_rms(e_warm, e64) / float(np.sqrt(2.0)) if e_warm is not None else None,
               "definition": "sqrt(sum (E32 - E64)^2 / sum E64^2) over nodes, absorbed power per node"}
        fp64 = {"crossings_per_s": c64 / d64, "ms_per_step": 1e3 * d64 / a.fp64_steps,
                "trace_kernel_ms": 1e3 * k64a,
                "trace_crossings_per_s": (c64 / a.fp64_steps) / k64a,
                "hbm_frac_algorithmic": (c64 / a.fp64_steps) * BYTES_PER_CROSSING_FP64 / k64a / 1e9 / HBM_PEAK_GBS}

    splitting = None
    if a.workload in ("cloud", "deep") and a.schedule == 0 and a.split_study:
        splitting = split_study(rt, gen, w, kw32)

    accel = None
    if a.schedule == 0 and a.ali_study:
        accel = ali_study(rt, gen)

    subiters = None
    if a.subiter_study:
        subiters = subiter_study(rt, gen)

    peeling = None
    if a.workload in ("cloud", "disc", "deep") and a.schedule == 0 and a.peel_study:
        peeling = peel_study(rt, gen, w, kw32, a.workload)

    res = {
        "metric": "cell-crossings/s (FP32-local form; FP64 form in fp64)",
        "value": value,
        "unit": "cell-crossings/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[a.workload] % w.sources[0].packets
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
                     "copy_gbs": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs if copy_gbs else None,
                     "kernel": "blk_pass_kernel<%d>" % (kw32["block_size"] or 768) if a.schedule == 0
                               else "trace_fp32_kernel<%d>" % (kw32["block_size"] or 256),
                     "launches_per_step": launches, "avg_launch_ms": 1e3 * main_launch_s,
                     "bytes_per_crossing": BYTES_PER_CROSSING_FP32, "issue": issue},
        "autotune": tuned,
        "fp64": fp64,
        "accuracy": acc if fp64 is not None else None,
        "cpu_baseline": cpu,
        "cpu_all_cores": cpu_all,
        "splitting": splitting,
        "peel_off": peeling,
        "accelerated_iteration": accel,
        "subiterations": subiters,
    }
    print(json.dumps(res))
    ctx.close()


if __name__ == "__main__":
    main()
