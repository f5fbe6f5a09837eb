"""ctypes shim around the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow, obviously-correct reference the GPU
library is checked against; it shares no code with the library.  Only ``tests/``, the smoke
check and the benchmark's CPU-baseline leg import this module.

Functions mirror the library's calls: ``Model`` (build_tree + set_dust), ``Model.locate``,
``Model.trace``, ``Model.solve_temperature``, ``Model.render``, and ``lambda_iterate`` (the
Lambda iteration of the paper's Eq. 2 driven from the oracle's own pieces).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no fp contraction)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class Stats(C.Structure):
    _fields_ = [("crossings", C.c_uint64), ("scatterings", C.c_uint64), ("kills", C.c_uint64),
                ("truncated", C.c_uint64), ("packets", C.c_uint64), ("dropped_zero_q", C.c_uint64),
                ("e_emit", C.c_double), ("e_abs", C.c_double), ("e_esc", C.c_double),
                ("e_killed", C.c_double), ("e_rr_gain", C.c_double), ("e_trunc", C.c_double),
                ("splits", C.c_uint64), ("split_kills", C.c_uint64), ("e_split_killed", C.c_double),
                ("e_split_gain", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


RECORD_DTYPE = np.dtype([("status", "<u4"), ("crossings", "<u4"), ("events", "<u4"),
                         ("pad", "<u4"), ("node", "<i8"), ("birth", "<i8"), ("w", "<f8")])


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_SO)
        P = C.c_void_p
        L.om_build.restype = P
        L.om_build.argtypes = [C.c_int32] * 3 + [C.c_double, C.c_int32, P, P, P, P]
        L.om_free.argtypes = [P]
        L.om_error.restype = C.c_char_p
        L.om_n_nodes.restype = C.c_int64
        L.om_n_nodes.argtypes = [P]
        L.om_n_levels.restype = C.c_int32
        L.om_n_levels.argtypes = [P]
        L.om_level_offsets.argtypes = [P, P]
        L.om_child.argtypes = [P, P]
        L.om_node_rho.argtypes = [P, P]
        L.om_locate.argtypes = [P, C.c_int64, P, P, P]
        L.om_philox.argtypes = [C.c_uint32, C.c_uint32, C.c_int64, P, P]
        L.om_set_dust.restype = C.c_int
        L.om_set_dust.argtypes = [P, C.c_int32, P, P, P, P]
        L.om_dnu.argtypes = [P, P]
        L.om_trace.restype = C.c_int
        L.om_trace.argtypes = [P, C.c_int32, C.c_int32, P, P, P, P, P, P, C.c_uint64, C.c_uint32,
                               C.c_double, C.c_double, C.c_int64, C.c_int32, C.c_int64, C.c_int64,
                               C.c_int32, P, P, P, C.c_int64, P, C.c_int32, P, P, P, P, C.c_int64, P, C.c_int32]
        L.om_node_coords.argtypes = [P, P]
        L.om_emission_all.argtypes = [P, P, P]
        L.om_hg_phase.restype = C.c_double
        L.om_hg_phase.argtypes = [C.c_double, C.c_double]
        L.om_peel_column.restype = C.c_int
        L.om_peel_column.argtypes = [P, P, C.c_int32, C.c_int64, P, P]
        L.om_branch_id.restype = C.c_uint32
        L.om_branch_id.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32]
        L.om_solve_temperature.argtypes = [P, P, C.c_double, C.c_double, P]
        L.om_emission.restype = C.c_double
        L.om_emission.argtypes = [P, C.c_int64, C.c_double]
        L.om_render.restype = C.c_int
        L.om_render.argtypes = [P, P, C.c_int32, C.c_double, C.c_int32, P, P, P, P]
        L.om_hg_mu.restype = C.c_double
        L.om_hg_mu.argtypes = [C.c_double, C.c_double]
        L.om_rotate.argtypes = [P, C.c_double, C.c_double]
        L.om_uniform.restype = C.c_double
        L.om_uniform.argtypes = [C.c_uint32]
        L.om_cdf_pick.restype = C.c_int64
        L.om_cdf_pick.argtypes = [P, C.c_int64, C.c_uint64]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    pass


class PeelOpts(C.Structure):
    _fields_ = [("n_dir", C.c_int32), ("n_obs", C.c_void_p), ("npix", C.c_int32),
                ("width", C.c_double), ("tiles", C.c_int32), ("image", C.c_void_p)]


def hg_phase(g, mu):
    return lib().om_hg_phase(float(g), float(mu))


class Model:
    """One oct-tree model with its dust table, held by the oracle."""

    def __init__(self, tree, dust=None):
        L = lib()
        self._keep = []
        nl = tree.n_levels
        root = np.ascontiguousarray(tree.root_rho, dtype=np.float64)
        nref = np.array([len(r) for r in tree.refined] or [0], dtype=np.int64)
        refs = [np.ascontiguousarray(r, dtype=np.int64) for r in tree.refined]
        kids = [np.ascontiguousarray(k, dtype=np.float64) for k in tree.child_rho]
        rp = (C.c_void_p * max(nl, 1))(*[_p(r).value for r in refs] or [None])
        kp = (C.c_void_p * max(nl, 1))(*[_p(k).value for k in kids] or [None])
        h = L.om_build(tree.nx, tree.ny, tree.nz, float(tree.root_cell_cm), nl, _p(root),
                       _p(nref), C.cast(rp, C.c_void_p), C.cast(kp, C.c_void_p))
        if not h:
            raise OracleError(L.om_error().decode())
        self.h = h
        self.tree = tree
        self.n_nodes = int(L.om_n_nodes(h))
        self.n_levels = nl
        off = np.zeros(nl + 2, dtype=np.int64)
        L.om_level_offsets(h, _p(off))
        self.offsets = off
        ch = np.zeros(self.n_nodes, dtype=np.int64)
        L.om_child(h, _p(ch))
        self.child = ch
        self.n_lambda = 0
        if dust is not None:
            self.set_dust(dust)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().om_free(self.h)
                self.h = None
        except Exception:
            pass

    @property
    def leaf_mask(self):
        return self.child < 0

    def level_of_nodes(self):
        lv = np.zeros(self.n_nodes, dtype=np.int32)
        for l in range(self.n_levels + 1):
            lv[self.offsets[l]:self.offsets[l + 1]] = l
        return lv

    def node_rho(self):
        r = np.zeros(self.n_nodes)
        lib().om_node_rho(self.h, _p(r))
        return r

    def set_dust(self, dust):
        L = lib()
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in
                (dust.lambda_um, dust.kappa_ext, dust.albedo, dust.hg_g)]
        if L.om_set_dust(self.h, len(arrs[0]), *[_p(a) for a in arrs]) != 0:
            raise OracleError(L.om_error().decode())
        self.n_lambda = len(arrs[0])
        self.dust = dust

    def dnu(self):
        d = np.zeros(self.n_lambda)
        lib().om_dnu(self.h, _p(d))
        return d

    def locate(self, xyz):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        n = len(xyz)
        lev = np.zeros(n, dtype=np.int32)
        node = np.zeros(n, dtype=np.int64)
        lib().om_locate(self.h, n, _p(xyz), _p(lev), _p(node))
        return lev, node

    def trace(self, sources, seed, iteration=0, model_index=0, rr_threshold=0.0, rr_prob=0.0,
              max_events=0, per_lambda=False, pid_begin=0, pid_end=-1, lam_sel=-1,
              t_node=None, rec_stride=0, deposits=True, split_n=1, peel=None, self_absorption=False,
              level_arrays=False, subtree=-1, e_abs_out=None, flux=False, split_depth=0):
        """Follow packets of ``sources`` (gen.Source list) -> (e_abs, e_esc, stats, records).
        ``peel``: dict(n_obs=[[x, y, z], ...], npix=, width=0.0, tiles=0) turns on the peel-off
        images, returned in stats["peel_image"] as [n_dir, n_lambda, npix, npix].
        ``self_absorption``: stats["e_self"] and stats["e_emit_node"] per node (the diagonal
        part of the accelerated Lambda iteration).  ``level_arrays``: stats["e_lvl"]
        [n_levels + 1, n_nodes], the deposits by the shallowest level visited; ``subtree``: a
        refined node whose subtree alone emits and holds the packages (subiterations).
        ``e_abs_out``: a caller-owned float64 array the deposits are added to (instead of a new
        zeroed one), so that repeated or concurrent calls need no new allocation.  ``flux``:
        stats["e_flux"] per node, the weight of the packages leaving each refined node's subtree
        (the energy flow from each grid to its parent, Sect. 3.3).  ``split_depth``: the reading
        of "grid" for splitting, 0 every oct, d > 0 all levels below d one grid with their
        level-d ancestor (1: the root grid and one grid per refined root cell)."""
        L = lib()
        ns = len(sources)
        nl = self.n_lambda
        kind = np.array([s.kind for s in sources], dtype=np.int32)
        pos = np.array([s.pos for s in sources], dtype=np.float64).reshape(-1)
        dirs = np.array([s.dir for s in sources], dtype=np.float64).reshape(-1)
        power = np.zeros(ns * nl)
        for i, s in enumerate(sources):
            if s.power is not None:
                power[i * nl:(i + 1) * nl] = s.power
        packets = np.array([s.packets for s in sources], dtype=np.int64)
        if e_abs_out is not None:
            if (e_abs_out.dtype != np.float64 or not e_abs_out.flags.c_contiguous
                    or e_abs_out.size != self.n_nodes * (nl if per_lambda else 1)):
                raise OracleError("e_abs_out must be a contiguous float64 array of the output size")
            e_abs = e_abs_out
        else:
            e_abs = np.zeros(self.n_nodes * (nl if per_lambda else 1)) if deposits else None
        e_esc = np.zeros(nl)
        st = Stats()
        tn = None if t_node is None else np.ascontiguousarray(t_node, dtype=np.float64)
        rec = None
        pid_end = pid_end if pid_end >= 0 else int(packets.max())
        if rec_stride > 0:
            nrec = (pid_end - pid_begin + rec_stride - 1) // rec_stride
            rec = np.zeros(ns * nl * nrec, dtype=RECORD_DTYPE)
        e_lvl = np.zeros((self.n_levels + 1) * self.n_nodes) if level_arrays else None
        e_self = np.zeros(self.n_nodes) if self_absorption else None
        e_flux = np.zeros(self.n_nodes) if flux else None
        e_emit_node = np.zeros(self.n_nodes) if self_absorption else None
        po, img = None, None
        if peel is not None:
            nobs = np.ascontiguousarray(peel["n_obs"], dtype=np.float64).reshape(-1, 3)
            npix = int(peel["npix"])
            img = np.zeros((len(nobs), nl, npix, npix))
            po = PeelOpts(len(nobs), _p(nobs).value, npix, float(peel.get("width", 0.0)),
                          int(peel.get("tiles", 0)), _p(img).value)
        rc = L.om_trace(self.h, model_index, ns, _p(kind), _p(pos), _p(dirs), _p(power),
                        _p(packets), None if tn is None else _p(tn), C.c_uint64(seed),
                        iteration, rr_threshold, rr_prob, max_events, int(per_lambda),
                        pid_begin, pid_end, lam_sel, None if e_abs is None else _p(e_abs),
                        _p(e_esc), C.byref(st),
                        rec_stride, None if rec is None else _p(rec), split_n,
                        None if po is None else C.byref(po),
                        None if e_self is None else _p(e_self),
                        None if e_emit_node is None else _p(e_emit_node),
                        None if e_lvl is None else _p(e_lvl), int(subtree),
                        None if e_flux is None else _p(e_flux), int(split_depth))
        if rc != 0:
            raise OracleError(L.om_error().decode())
        if img is not None or e_self is not None or e_lvl is not None or e_flux is not None:
            out = st.as_dict()
            if e_flux is not None:
                out["e_flux"] = e_flux
            if img is not None:
                out["peel_image"] = img
            if e_self is not None:
                out["e_self"] = e_self
                out["e_emit_node"] = e_emit_node
            if e_lvl is not None:
                out["e_lvl"] = e_lvl.reshape(self.n_levels + 1, self.n_nodes)
            if per_lambda and e_abs is not None:
                e_abs = e_abs.reshape(nl, self.n_nodes)
            return e_abs, e_esc, out, rec
        if per_lambda and e_abs is not None:
            e_abs = e_abs.reshape(nl, self.n_nodes)
        return e_abs, e_esc, st.as_dict(), rec

    def peel_column(self, n_obs, xyz, tiles=0):
        """Column (density x length, root-cell units) from each point toward n_obs."""
        nv = np.ascontiguousarray(n_obs, dtype=np.float64)
        x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        col = np.zeros(len(x))
        lib().om_peel_column(self.h, _p(nv), int(tiles), len(x), _p(x), _p(col))
        return col

    def node_coords(self):
        """Integer coordinates of every node at its own level, [n_nodes, 3]."""
        out = np.zeros(3 * self.n_nodes, dtype=np.int32)
        lib().om_node_coords(self.h, _p(out))
        return out.reshape(-1, 3)

    def subtree_mask(self, root):
        """Nodes of the subtree below refined node ``root`` (all nodes for -1)."""
        if root < 0:
            return np.ones(self.n_nodes, dtype=bool)
        lv = self.level_of_nodes()
        xyz = self.node_coords().astype(np.int64)
        lr, cr = int(lv[root]), xyz[root]
        sh = np.maximum(lv - lr, 0)[:, None]
        return (lv > lr) & np.all((xyz >> sh) == cr[None, :], axis=1)

    def emission_all(self, t_node):
        """Emitted power of every leaf at temperatures t_node (0 for refined nodes)."""
        tn = np.ascontiguousarray(t_node, dtype=np.float64)
        out = np.zeros(self.n_nodes)
        lib().om_emission_all(self.h, _p(tn), _p(out))
        return out

    def solve_temperature(self, a_node, t_min=2.0, t_max=3000.0):
        a = np.ascontiguousarray(a_node, dtype=np.float64)
        t = np.zeros(self.n_nodes)
        lib().om_solve_temperature(self.h, _p(a), t_min, t_max, _p(t))
        return t

    def emission(self, node, t):
        return lib().om_emission(self.h, int(node), float(t))

    def render(self, n_obs, npix, t_node, lambda_idx, width=0.0):
        L = lib()
        nv = np.ascontiguousarray(n_obs, dtype=np.float64)
        li = np.ascontiguousarray(lambda_idx, dtype=np.int32)
        tn = np.ascontiguousarray(t_node, dtype=np.float64)
        img = np.zeros((len(li), npix, npix))
        cr = C.c_uint64(0)
        rc = L.om_render(self.h, _p(nv), npix, width, len(li), _p(li), _p(tn), _p(img),
                         C.byref(cr))
        if rc != 0:
            raise OracleError(L.om_error().decode())
        return img, int(cr.value)


def philox(key0, key1, ctr):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.zeros_like(ctr)
    lib().om_philox(key0, key1, len(ctr), _p(ctr), _p(out))
    return out


def hg_mu(g, u):
    return lib().om_hg_mu(float(g), float(u))


def rotate(d, mu, phi):
    v = np.ascontiguousarray(d, dtype=np.float64).copy()
    lib().om_rotate(_p(v), float(mu), float(phi))
    return v


def cdf_pick(q, r):
    q = np.ascontiguousarray(q, dtype=np.uint64)
    return int(lib().om_cdf_pick(_p(q), len(q), C.c_uint64(int(r))))


def branch_id(b, n, c):
    return int(lib().om_branch_id(b, n, c))


def uniform(x):
    """The oracle's uniform mapping (2 (x >> 9) + 1) 2^-24, for tests."""
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(9)).astype(np.float64) * 2.0 + 1.0) * 2.0 ** -24


def ali_step_absorbed(a_stars, a_dust, e_self, e_emit_node):
    """Absorbed power that the accelerated Lambda iteration (Sect. 3.1 Eq. 3) balances with the
    new emission E(T): with lambda* = e_self / e_emit the fraction of a cell's own emission it
    absorbs before its packets first leave it, E(T)(1 - lambda*) = A_stars + A_dust - e_self,
    i.e. E(T) = (A_stars + A_dust - e_self) / (1 - lambda*)."""
    lam = np.where(e_emit_node > 0.0, e_self / np.where(e_emit_node > 0.0, e_emit_node, 1.0), 0.0)
    lam = np.minimum(lam, 1.0 - 1e-9)
    return (a_stars + a_dust - e_self) / (1.0 - lam)


def subtree_ali_absorbed(a_tot, mask, st):
    """The absorbed power a subiteration step balances with the new emission when it uses the
    accelerated iteration (Sect. 3.1 Eq. 3 inside the subtree, Sect. 3.2): for the cells of the
    subtree, whose emission the step traced, ali_step_absorbed with A_stars + A_dust replaced by
    the sum of the cell's arrays (e_self, the part of its own emission it absorbed before the
    packets first left it, lies in its own level's array); elsewhere a_tot unchanged."""
    lam = np.where(st["e_emit_node"] > 0.0,
                   st["e_self"] / np.where(st["e_emit_node"] > 0.0, st["e_emit_node"], 1.0), 0.0)
    lam = np.minimum(lam, 1.0 - 1e-9)
    return np.where(mask, (a_tot - st["e_self"]) / (1.0 - lam), a_tot)


def subiterate(model, star_sources, seed, schedule, dust_packets, rr_threshold=0.0, rr_prob=0.0,
               t_min=2.0, t_max=3000.0, split_n=1, split_depth=0, ali=False):
    """Lambda iteration with subiterations on complete subtrees (paper Sect. 3.1 and App. B).
    ``schedule``: the subtree root of each step, a refined node or -1 for the whole model.  Each
    cell keeps one absorbed-energy array per hierarchy level above or at its own; a step with
    root r (level l_r) traces the dust emission of r's subtree only, keeps its packages inside
    it, and replaces the arrays of levels > l_r (all levels for the whole model) of the cells in
    the subtree with what it deposits; the temperatures of those cells then follow from
    A_stars + the sum of their arrays (Eq. 9).  Key iteration of step k is k.  ``split_n`` > 1:
    package splitting (Sect. 2.3) in every trace, a split-off package filing its deposits under
    the shallowest level of the package it split from.  ``ali``: every step uses the
    accelerated iteration inside its subtree (subtree_ali_absorbed).  Returns (temperature
    after each step, A_stars, per-step trace statistics)."""
    import gen
    sp = dict(split_n=split_n, split_depth=split_depth)
    a_stars, _, _, _ = model.trace(star_sources, seed, iteration=0, rr_threshold=rr_threshold,
                                   rr_prob=rr_prob, **sp)
    t = model.solve_temperature(a_stars, t_min, t_max)
    lv = model.level_of_nodes()
    arrays = np.zeros((model.n_levels + 1, model.n_nodes))
    hist, stats = [t.copy()], []
    for it, root in enumerate(schedule, start=1):
        lo = 0 if root < 0 else int(lv[root]) + 1
        mask = model.subtree_mask(root)
        src = [gen.Source(gen.SRC_DUST, 0, packets=dust_packets)]
        _, _, st, _ = model.trace(src, seed, iteration=it, rr_threshold=rr_threshold,
                                  rr_prob=rr_prob, t_node=t, level_arrays=True, subtree=root,
                                  self_absorption=ali, **sp)
        stats.append(st)
        arrays[lo:, mask] = st["e_lvl"][lo:, mask]
        a_tot = a_stars + arrays.sum(axis=0)
        t_new = model.solve_temperature(subtree_ali_absorbed(a_tot, mask, st) if ali else a_tot,
                                         t_min, t_max)
        t = np.where(mask, t_new, t)
        hist.append(t.copy())
    return hist, a_stars, stats


def canonical_parents(model):
    """Canonical parent of every node (-1 for a root cell)."""
    tree = model.tree
    par = np.full(model.n_nodes, -1, dtype=np.int64)
    for l, ref in enumerate(tree.refined):
        lo = model.offsets[l + 1]
        kids = np.arange(8 * len(ref), dtype=np.int64)
        par[lo + kids] = model.offsets[l] + np.asarray(ref, dtype=np.int64)[kids // 8]
    return par


def subtree_select(imb, frac, parent, tagged, tag_root):
    """The next subtree of the automatic iteration (Sect. 3.3): the lowest common ancestor of the
    parents of every leaf whose imbalance is within ``frac`` of the largest, and of every tagged
    grid (a refined node, which the subtree must hold); -1 for the whole model (no refined cell
    holds them all, or the root grid is tagged)."""
    mx = float(imb.max()) if len(imb) else 0.0
    nodes = [int(parent[c]) for c in np.flatnonzero(imb >= frac * mx)] if mx > 0.0 else []
    nodes += [int(g) for g in np.flatnonzero(tagged)]
    if tag_root or not nodes:
        return -1, mx

    def chain(c):  # c and its ancestors, deepest first
        out = []
        while c >= 0:
            out.append(c)
            c = int(parent[c])
        return out
    common = None
    for c in nodes:
        if c < 0:
            return -1, mx
        ch = chain(c)
        common = ch if common is None else [a for a in ch if a in set(common)]
        if not common:
            return -1, mx
    return common[0], mx


def subiterate_auto(model, star_sources, seed, n_steps, dust_packets, frac=0.5, stall=0.8,
                    flux_frac=0.0, rr_threshold=0.0, rr_prob=0.0, t_min=2.0, t_max=3000.0,
                    split_n=1, split_depth=0, ali=False):
    """The automatic iteration of Sect. 3.3 over subiterations on complete subtrees (Sect. 3.1,
    App. B), step by step from the oracle's own bookkeeping:
      * per leaf, the energy imbalance |A - E(T_old)| / E(T_old) recorded at its last step, with
        E the emission at the temperatures that step started from;
      * the first step takes the whole model; each later one the subtree subtree_select picks
        (leaves within ``frac`` of the largest imbalance, and the tagged grids);
      * a repeat of the previous subtree without the largest imbalance dropping below ``stall``
        times its previous value is the noise limit of that subtree: the whole model instead;
      * flux_frac > 0: the energy flowing out of every refined node's subtree is measured in each
        step; when a step below r changes the flow out of r's subtree by more than flux_frac
        times the energy absorbed in its parent's subtree (since the parent last took part), the
        parent grid is tagged until a step includes it.
    Key iteration of step k is k; ``split_n``, ``split_depth`` and ``ali`` as for subiterate
    (the imbalances and the flows use the absorbed power itself).  Returns (temperatures after
    each step, the roots taken)."""
    import gen
    sp = dict(split_n=split_n, split_depth=split_depth)
    a_stars, _, _, _ = model.trace(star_sources, seed, iteration=0, rr_threshold=rr_threshold,
                                   rr_prob=rr_prob, **sp)
    t = model.solve_temperature(a_stars, t_min, t_max)
    lv = model.level_of_nodes()
    leaf = model.leaf_mask
    parent = canonical_parents(model)
    arrays = np.zeros((model.n_levels + 1, model.n_nodes))
    imb = np.zeros(model.n_nodes)
    flux_ref = np.zeros(model.n_nodes)
    tagged = np.zeros(model.n_nodes, dtype=bool)
    tag_root = False
    hist, roots = [t.copy()], []
    prev_root, prev_max = -2, 0.0
    for k in range(n_steps):
        root = -1
        if k > 0:
            root, mx = subtree_select(imb, frac, parent, tagged, tag_root)
            if root >= 0 and root == prev_root and mx > stall * prev_max:
                root = -1
            prev_max = mx
        lo = 0 if root < 0 else int(lv[root]) + 1
        mask = model.subtree_mask(root)
        src = [gen.Source(gen.SRC_DUST, 0, packets=dust_packets)]
        _, _, st, _ = model.trace(src, seed, iteration=k + 1, rr_threshold=rr_threshold,
                                  rr_prob=rr_prob, t_node=t, level_arrays=True, subtree=root,
                                  flux=flux_frac > 0.0, self_absorption=ali, **sp)
        arrays[lo:, mask] = st["e_lvl"][lo:, mask]
        a_tot = a_stars + arrays.sum(axis=0)
        e_old = model.emission_all(t)
        upd = mask & leaf
        imb[upd] = np.where(e_old[upd] > 0.0, np.abs(a_tot[upd] - e_old[upd]) / np.where(e_old[upd] > 0.0,
                                                                                        e_old[upd], 1.0), 0.0)
        t_new = model.solve_temperature(subtree_ali_absorbed(a_tot, mask, st) if ali else a_tot,
                                         t_min, t_max)
        t = np.where(mask, t_new, t)
        if flux_frac > 0.0:
            flow = st["e_flux"]
            if root >= 0:
                par = int(parent[root])
                absorbed = float(a_tot[model.subtree_mask(par) & leaf].sum())
                if abs(flow[root] - flux_ref[root]) > flux_frac * absorbed:
                    if par < 0:
                        tag_root = True
                    else:
                        tagged[par] = True
            inner = mask & ~leaf
            flux_ref[inner] = flow[inner]
            tagged[inner] = False
            if root >= 0:
                tagged[root] = False
            else:
                tag_root = False
        prev_root = root
        roots.append(root)
        hist.append(t.copy())
    return hist, roots


def lambda_iterate(model, star_sources, seed, n_max=30, tol=1e-3, n_fixed=None,
                   dust_packets=None, rr_threshold=0.0, rr_prob=0.0, t_min=2.0, t_max=3000.0,
                   ali=False, split_n=1):
    """Lambda iteration (paper Sect. 3.1 Eq. 2; constant-source field kept, Sect. 3.2), or with
    ali=True the accelerated iteration with the diagonal operator (Eq. 3, ali_step_absorbed):
    A_stars from the constant sources once, T_0 = f(A_stars); then for n >= 1 the dust
    emission of T_{n-1} is traced with key iteration n, T_n = f(A_stars + A_dust).
    Stops when the mass-weighted mean |T_n - T_{n-1}|/T_{n-1} < tol, or after n_max steps
    (or exactly n_fixed steps).  ``split_n`` > 1: package splitting in every trace.  Returns
    (T history list, A_stars, per-step dust-trace stats)."""
    import gen
    a_stars, _, _, _ = model.trace(star_sources, seed, iteration=0, rr_threshold=rr_threshold,
                                   rr_prob=rr_prob, split_n=split_n)
    t = model.solve_temperature(a_stars, t_min, t_max)
    hist = [t]
    leaf = model.leaf_mask
    lv = model.level_of_nodes()
    mass = model.node_rho() * (model.tree.root_cell_cm * 2.0 ** -lv) ** 3
    n_steps = n_fixed if n_fixed is not None else n_max
    npk = dust_packets if dust_packets is not None else star_sources[0].packets
    stats = []
    for it in range(1, n_steps + 1):
        src = [gen.Source(gen.SRC_DUST, 0, packets=npk)]
        a_dust, _, st, _ = model.trace(src, seed, iteration=it, rr_threshold=rr_threshold,
                                       rr_prob=rr_prob, t_node=t, self_absorption=ali,
                                       split_n=split_n)
        stats.append(st)
        if ali:
            a_new = ali_step_absorbed(a_stars, a_dust, st["e_self"], st["e_emit_node"])
        else:
            a_new = a_stars + a_dust
        t_new = model.solve_temperature(a_new, t_min, t_max)
        hist.append(t_new)
        w = mass[leaf]
        rel = np.abs(t_new[leaf] - t[leaf]) / t[leaf]
        crit = float((w * rel).sum() / w.sum()) if w.sum() > 0 else 0.0
        t = t_new
        if n_fixed is None and crit < tol:
            break
    return hist, a_stars, stats
