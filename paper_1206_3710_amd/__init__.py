"""Python binding of the gfx950 hierarchical-grid Monte Carlo radiative-transfer library.

Argument marshalling only: every step of the transport, the temperature solve and the maps
runs in the HIP kernels of ``libhiert.so`` (C ABI in ``include/rt.h``).  PyTorch provides
device memory and the current stream.  There is no CPU fallback: if the library is not built,
or no gfx950 device is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhiert.so")

RT_OK, RT_EINVAL, RT_ENOMEM, RT_EDEVICE, RT_ESTATE = 0, -1, -2, -3, -4
RT_MAX_LEVELS = 24
SRC_BACKGROUND, SRC_POINT, SRC_DUST, SRC_BEAM = 0, 1, 2, 3
FP64, FP32_LOCAL = 0, 1
SCHED_REGIONS, SCHED_GLOBAL = 0, 1

EXPORTS = ["rt_last_error", "rt_create", "rt_destroy", "rt_build_tree", "rt_get_model_info",
           "rt_get_sizes", "rt_locate", "rt_set_dust", "rt_set_temperature", "rt_trace_packets",
           "rt_solve_temperature", "rt_lambda_iterate", "rt_ali_iterate", "rt_subiter_begin",
           "rt_subiter_step", "rt_subiter_select", "rt_subiter_run", "rt_render_map",
           "rt_render_map_noalloc", "rt_peel_map",
           "rt_autotune", "rt_philox"]


class RTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rt error {code}: {msg}")
        self.code = code


class TreeDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("root_cell_cm", C.c_double), ("n_levels", C.c_int32),
                ("root_rho", C.c_void_p), ("n_refined", C.c_void_p), ("refined", C.c_void_p),
                ("child_rho", C.c_void_p)]


class ModelInfo(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_leaves", C.c_int64), ("n_levels", C.c_int32),
                ("n_lambda", C.c_int32), ("level_offset", C.c_int64 * (RT_MAX_LEVELS + 2)),
                ("node_base", C.c_int64), ("lambda_base", C.c_int64),
                ("lambda_node_base", C.c_int64)]


class Source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("model", C.c_int32), ("pos", C.c_double * 3),
                ("dir", C.c_double * 3), ("power", C.c_void_p), ("packets_per_lambda", C.c_int64)]


class TraceOpts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("iteration", C.c_uint32), ("precision", C.c_int32),
                ("rr_threshold", C.c_double), ("rr_prob", C.c_double), ("max_events", C.c_int64),
                ("block_size", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("refill_threshold", C.c_float), ("schedule", C.c_int32),
                ("chunk_packets", C.c_int32), ("tail_park", C.c_int32), ("batch_packets", C.c_int64),
                ("rec_stride", C.c_int64), ("records", C.c_void_p), ("sweep_graph", C.c_int32),
                ("split_n", C.c_int32), ("split_depth", C.c_int32)]


class PeelOpts(C.Structure):
    _fields_ = [("n_dir", C.c_int32), ("npix", C.c_int32), ("n_obs", C.c_void_p),
                ("width", C.c_double), ("tiles", C.c_int32), ("pad", C.c_int32),
                ("event_buffer", C.c_int64), ("image", C.c_void_p)]


class TraceStats(C.Structure):
    _fields_ = [("crossings", C.c_uint64), ("scatterings", C.c_uint64), ("kills", C.c_uint64),
                ("truncated", C.c_uint64), ("packets", C.c_uint64), ("e_emit", C.c_double),
                ("e_abs", C.c_double), ("e_esc", C.c_double), ("e_killed", C.c_double),
                ("e_rr_gain", C.c_double), ("e_trunc", C.c_double), ("kernel_ms", C.c_double),
                ("reduce_ms", C.c_double), ("main_ms", C.c_double), ("main_launches", C.c_uint64),
                ("splits", C.c_uint64), ("split_kills", C.c_uint64), ("split_skips", C.c_uint64),
                ("e_split_killed", C.c_double), ("e_split_gain", C.c_double),
                ("peel_events", C.c_uint64), ("table_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


RECORD_DTYPE = np.dtype([("status", "<u4"), ("crossings", "<u4"), ("events", "<u4"),
                         ("pad", "<u4"), ("node", "<i8"), ("birth", "<i8"), ("w", "<f8")])

_lib = None


def lib():
    """Load libhiert.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1206_3710_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        I32, I64, U32, U64, D = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
        sig = {
            "rt_last_error": (C.c_char_p, [P]),
            "rt_create": (I32, [P, I32, P]),
            "rt_destroy": (I32, [P]),
            "rt_build_tree": (I32, [P, P, P, P]),
            "rt_get_model_info": (I32, [P, I32, P]),
            "rt_get_sizes": (I32, [P, P, P, P]),
            "rt_locate": (I32, [P, I32, I64, P, P, P]),
            "rt_set_dust": (I32, [P, I32, I32, P, P, P, P]),
            "rt_set_temperature": (I32, [P, I32, P]),
            "rt_trace_packets": (I32, [P, I32, P, P, P, P, P, P]),
            "rt_solve_temperature": (I32, [P, I32, P, D, D, P]),
            "rt_lambda_iterate": (I32, [P, I32, I32, P, P, I64, I32, D, D, D, P, P, P]),
            "rt_ali_iterate": (I32, [P, I32, I32, P, P, I64, I32, D, D, D, P, P, P]),
            "rt_subiter_begin": (I32, [P, I32, I32, P, P, D, D, D, I32]),
            "rt_subiter_step": (I32, [P, I32, I64, I64, U32, P, P, P, P]),
            "rt_subiter_select": (I32, [P, I32, D, P, P]),
            "rt_subiter_run": (I32, [P, I32, I32, D, D, I64, U32, P, P, P, P, P]),
            "rt_render_map": (I32, [P, I32, P, I32, D, I32, P, I32, P, P]),
            "rt_render_map_noalloc": (I32, [P, I32, P, I32, D, I32, P, I32, P, P]),
            "rt_peel_map": (I32, [P, I32, P, P, P, P]),
            "rt_autotune": (I32, [P, I32, P, P, D, C.c_char_p, P, P]),
            "rt_philox": (I32, [P, U32, U32, I64, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _source_array(sources):
    """ctypes array of rt_source for gen.Source-like objects, and the power arrays it points to."""
    n = len(sources)
    arr = (Source * n)()
    keep = []
    for i, s in enumerate(sources):
        pw = None
        if s.power is not None:
            pw = np.ascontiguousarray(s.power, dtype=np.float64)
            keep.append(pw)
        arr[i] = Source(int(s.kind), int(s.model), (C.c_double * 3)(*s.pos),
                        (C.c_double * 3)(*s.dir), None if pw is None else _ptr(pw).value,
                        int(s.packets))
    return arr, keep


def _ptr(a):
    """Address of a numpy array or torch tensor."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _torch():
    import torch
    return torch


class Context:
    """A library context on one GPU.  Arrays returned are torch tensors on that GPU."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU available: the library runs only on a gfx950 device")
        self.device = device
        self.tdev = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.tdev)
        self.stream = stream
        h = C.c_void_p()
        handle = C.c_void_p(stream.cuda_stream) if hasattr(stream, "cuda_stream") else C.c_void_p(stream)
        rc = lib().rt_create(C.byref(h), device, handle)
        if rc != RT_OK:
            raise RTError(rc, lib().rt_last_error(None).decode())
        self.h = h
        self.models = []

    def close(self):
        if getattr(self, "h", None):
            lib().rt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != RT_OK:
            raise RTError(rc, lib().rt_last_error(self.h).decode())

    # ------------------------------------------------------------------ tree and dust
    def build_tree(self, tree) -> int:
        nl = tree.n_levels
        root = np.ascontiguousarray(tree.root_rho, dtype=np.float64)
        nref = np.array([len(r) for r in tree.refined] or [0], dtype=np.int64)
        refs = [np.ascontiguousarray(r, dtype=np.int64) for r in tree.refined]
        kids = [np.ascontiguousarray(k, dtype=np.float64) for k in tree.child_rho]
        rp = (C.c_void_p * max(nl, 1))(*[_ptr(r).value for r in refs] or [None])
        kp = (C.c_void_p * max(nl, 1))(*[_ptr(k).value for k in kids] or [None])
        d = TreeDesc(tree.nx, tree.ny, tree.nz, float(tree.root_cell_cm), nl, _ptr(root).value,
                     _ptr(nref).value, C.cast(rp, C.c_void_p).value, C.cast(kp, C.c_void_p).value)
        model = C.c_int32()
        nn = C.c_int64()
        self._check(lib().rt_build_tree(self.h, C.byref(d), C.byref(model), C.byref(nn)))
        self.models.append(int(nn.value))
        return int(model.value)

    def model_info(self, model: int) -> dict:
        mi = ModelInfo()
        self._check(lib().rt_get_model_info(self.h, model, C.byref(mi)))
        d = {k: getattr(mi, k) for k, _ in mi._fields_ if k != "level_offset"}
        d["level_offset"] = list(mi.level_offset)[: mi.n_levels + 2]
        return d

    def sizes(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(lib().rt_get_sizes(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return int(a.value), int(b.value), int(c.value)

    def set_dust(self, model: int, dust):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in
                (dust.lambda_um, dust.kappa_ext, dust.albedo, dust.hg_g)]
        self._check(lib().rt_set_dust(self.h, model, len(arrs[0]), *[_ptr(a) for a in arrs]))

    def set_temperature(self, model: int, t_node):
        t = self._dev(t_node, _torch().float64)
        self._check(lib().rt_set_temperature(self.h, model, _ptr(t)))

    def _dev(self, a, dtype):
        torch = _torch()
        if isinstance(a, torch.Tensor):
            return a.to(device=self.tdev, dtype=dtype).contiguous()
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=self.tdev)

    # ------------------------------------------------------------------ calls
    def locate(self, model: int, xyz):
        torch = _torch()
        x = self._dev(xyz, torch.float64).reshape(-1, 3)
        n = x.shape[0]
        lev = torch.empty(n, dtype=torch.int32, device=self.tdev)
        node = torch.empty(n, dtype=torch.int64, device=self.tdev)
        self._check(lib().rt_locate(self.h, model, n, _ptr(x), _ptr(lev), _ptr(node)))
        return lev, node

    def trace_packets(self, sources: Sequence, seed: int, iteration: int = 0, precision: int = FP64,
                      rr_threshold: float = 0.0, rr_prob: float = 0.0, max_events: int = 0,
                      block_size: int = 0, blocks_per_cu: int = 0, refill_threshold: float = 0.0,
                      rec_stride: int = 0, per_lambda: bool = False, schedule: int = SCHED_REGIONS,
                      chunk_packets: int = 0, batch_packets: int = 0, tail_park: int = 0,
                      sweep_graph: int = 0, split_n: int = 1, split_depth: int = 0):
        """Trace the packets of ``sources`` (objects with kind, model, pos, dir, power,
        packets).  ``split_n`` > 1 turns on package splitting at subgrid entry with the
        roulette at subgrid exit (region schedule); ``split_depth`` > 0 makes all levels below
        it one grid with their ancestor at that level (0: every oct is a grid).  Returns a dict of device tensors and the
        statistics."""
        torch = _torch()
        n = len(sources)
        arr, keep = _source_array(sources)
        n_rec = 0
        tn, tl, tln = self.sizes()
        e_node = torch.zeros(tn, dtype=torch.float64, device=self.tdev)
        e_lam = torch.zeros(max(tln, 1), dtype=torch.float64, device=self.tdev) if per_lambda else None
        e_esc = torch.zeros(max(tl, 1), dtype=torch.float64, device=self.tdev)
        rec = None
        if rec_stride > 0:
            for s in sources:
                nl = self.model_info(int(s.model))["n_lambda"]
                n_rec += nl * ((int(s.packets) + rec_stride - 1) // rec_stride)
            rec = torch.zeros(max(n_rec, 1) * RECORD_DTYPE.itemsize, dtype=torch.uint8,
                              device=self.tdev)
        opts = TraceOpts(seed, iteration, precision, rr_threshold, rr_prob, max_events, block_size,
                         blocks_per_cu, refill_threshold, schedule, chunk_packets, tail_park,
                         batch_packets, rec_stride, None if rec is None else rec.data_ptr(),
                         sweep_graph, split_n, split_depth)
        st = TraceStats()
        self._check(lib().rt_trace_packets(self.h, n, arr, C.byref(opts), _ptr(e_node),
                                           _ptr(e_lam), _ptr(e_esc), C.byref(st)))
        out = {"e_abs_node": e_node, "e_esc": e_esc[:tl], "stats": st.as_dict()}
        if per_lambda:
            out["e_abs_lambda_node"] = e_lam[:tln]
        if rec is not None:
            out["records"] = np.frombuffer(rec.cpu().numpy().tobytes(), dtype=RECORD_DTYPE)[:n_rec]
        return out

    def peel_map(self, sources: Sequence, seed: int, n_obs, npix: int, width: float = 0.0,
                 tiles: int = 0, event_buffer: int = 0, iteration: int = 0, precision: int = FP64,
                 rr_threshold: float = 0.0, rr_prob: float = 0.0, max_events: int = 0,
                 block_size: int = 0, blocks_per_cu: int = 0, refill_threshold: float = 0.0,
                 schedule: int = SCHED_REGIONS, chunk_packets: int = 0, batch_packets: int = 0,
                 tail_park: int = 0, split_n: int = 1, split_depth: int = 0):
        """Peel-off images of the scattered light toward the directions ``n_obs`` ([n_dir, 3]):
        a device tensor [n_dir, n_lambda, npix, npix] and the statistics."""
        torch = _torch()
        n = len(sources)
        arr, keep = _source_array(sources)
        nv = np.ascontiguousarray(n_obs, dtype=np.float64).reshape(-1, 3)
        nl = self.model_info(int(sources[0].model))["n_lambda"]
        img = torch.zeros((len(nv), nl, npix, npix), dtype=torch.float64, device=self.tdev)
        po = PeelOpts(len(nv), npix, _ptr(nv).value, width, tiles, 0, event_buffer, img.data_ptr())
        opts = TraceOpts(seed, iteration, precision, rr_threshold, rr_prob, max_events, block_size,
                         blocks_per_cu, refill_threshold, schedule, chunk_packets, tail_park,
                         batch_packets, 0, None, 0, split_n, split_depth)
        st = TraceStats()
        self._check(lib().rt_peel_map(self.h, n, arr, C.byref(opts), C.byref(po), C.byref(st)))
        return img, st.as_dict()

    def solve_temperature(self, model: int, a_node, t_min: float = 2.0, t_max: float = 3000.0):
        """Temperatures for absorbed power ``a_node``; None takes the last trace's result."""
        torch = _torch()
        a = None if a_node is None else self._dev(a_node, torch.float64)
        t = torch.empty(self.models[model], dtype=torch.float64, device=self.tdev)
        self._check(lib().rt_solve_temperature(self.h, model, _ptr(a), t_min, t_max, _ptr(t)))
        return t

    def autotune(self, sources: Sequence, seed: int, precision: int = FP32_LOCAL,
                 schedule: int = SCHED_REGIONS, sample_fraction: float = 0.125,
                 cache: Optional[str] = None, iteration: int = 0, rr_threshold: float = 0.0,
                 rr_prob: float = 0.0, **start):
        """Tune the launch parameters of trace_packets on a packet prefix of ``sources``.
        Returns (keyword arguments for trace_packets, crossings per second of the sample)."""
        n = len(sources)
        arr = (Source * n)()
        keep = []
        for i, s in enumerate(sources):
            pw = None
            if s.power is not None:
                pw = np.ascontiguousarray(s.power, dtype=np.float64)
                keep.append(pw)
            arr[i] = Source(int(s.kind), int(s.model), (C.c_double * 3)(*s.pos),
                            (C.c_double * 3)(*s.dir), None if pw is None else _ptr(pw).value,
                            int(s.packets))
        base = TraceOpts(seed, iteration, precision, rr_threshold, rr_prob,
                         start.get("max_events", 0), start.get("block_size", 0),
                         start.get("blocks_per_cu", 0), start.get("refill_threshold", 0.0),
                         schedule, start.get("chunk_packets", 0), start.get("tail_park", 0),
                         start.get("batch_packets", 0), 0, None, 0, start.get("split_n", 0))
        best = TraceOpts()
        rate = C.c_double()
        self._check(lib().rt_autotune(self.h, n, arr, C.byref(base), sample_fraction,
                                      None if cache is None else cache.encode(), C.byref(best),
                                      C.byref(rate)))
        tuned = {"block_size": best.block_size, "blocks_per_cu": best.blocks_per_cu,
                 "refill_threshold": round(best.refill_threshold, 6),
                 "chunk_packets": best.chunk_packets, "tail_park": best.tail_park,
                 "batch_packets": best.batch_packets}
        return tuned, rate.value

    def lambda_iterate(self, model: int, sources: Sequence, seed: int, dust_packets: int,
                       n_max: int = 30, tol: float = 1e-3, t_min: float = 2.0,
                       t_max: float = 3000.0, precision: int = FP64, rr_threshold: float = 0.0,
                       rr_prob: float = 0.0, iteration: int = 0, ali: bool = False, **kw):
        """Lambda iteration (ali=True: the accelerated one with the diagonal operator).
        Returns (temperatures, steps taken, stopping statistic per step)."""
        torch = _torch()
        n = len(sources)
        arr = (Source * max(n, 1))()
        keep = []
        for i, s in enumerate(sources):
            pw = np.ascontiguousarray(s.power, dtype=np.float64)
            keep.append(pw)
            arr[i] = Source(int(s.kind), int(s.model), (C.c_double * 3)(*s.pos),
                            (C.c_double * 3)(*s.dir), _ptr(pw).value, int(s.packets))
        opts = TraceOpts(seed, iteration, precision, rr_threshold, rr_prob, kw.get("max_events", 0),
                         kw.get("block_size", 0), kw.get("blocks_per_cu", 0),
                         kw.get("refill_threshold", 0.0), kw.get("schedule", SCHED_REGIONS),
                         kw.get("chunk_packets", 0), kw.get("tail_park", 0),
                         kw.get("batch_packets", 0), 0, None, kw.get("sweep_graph", 0),
                         kw.get("split_n", 0), kw.get("split_depth", 0))
        t = torch.empty(self.models[model], dtype=torch.float64, device=self.tdev)
        nd = C.c_int32()
        crit = np.zeros(max(n_max, 1))
        fn = lib().rt_ali_iterate if ali else lib().rt_lambda_iterate
        self._check(fn(self.h, model, n, arr, C.byref(opts), dust_packets, n_max, tol, t_min, t_max,
                       _ptr(t), C.byref(nd), _ptr(crit)))
        return t, int(nd.value), crit[: nd.value]

    @staticmethod
    def _sub_opts(seed, iteration, precision, rr_threshold, rr_prob, kw):
        return TraceOpts(seed, iteration, precision, rr_threshold, rr_prob, kw.get("max_events", 0),
                         kw.get("block_size", 0), kw.get("blocks_per_cu", 0),
                         kw.get("refill_threshold", 0.0), kw.get("schedule", SCHED_REGIONS),
                         kw.get("chunk_packets", 0), kw.get("tail_park", 0),
                         kw.get("batch_packets", 0), 0, None, 0, kw.get("split_n", 0),
                         kw.get("split_depth", 0))

    def subiter_begin(self, model: int, sources: Sequence, seed: int, t_min: float = 2.0,
                      t_max: float = 3000.0, iteration: int = 0, rr_threshold: float = 0.0,
                      rr_prob: float = 0.0, precision: int = FP64, flux_frac: float = 0.0,
                      ali: bool = False, **kw):
        """Subiterations (FP64 form, or FP32_LOCAL with the region schedule): trace the
        constant sources, T_0, clear the level arrays; flux_frac > 0 tracks the energy flow
        from each grid to its parent and tags grids whose inflow changed; ali: the steps use
        the accelerated iteration inside their subtree (FP64 form)."""
        arr, keep = _source_array(sources) if sources else ((Source * 1)(), [])
        opts = self._sub_opts(seed, iteration, precision, rr_threshold, rr_prob, kw)
        self._check(lib().rt_subiter_begin(self.h, model, len(sources), arr, C.byref(opts), t_min, t_max,
                                           float(flux_frac), 1 if ali else 0))

    def subiter_step(self, model: int, root: int, dust_packets: int, seed: int, iteration: int,
                     rr_threshold: float = 0.0, rr_prob: float = 0.0, precision: int = FP64, **kw):
        """One (sub)iteration step below refined node ``root`` (-1: the whole model).
        Returns (temperatures, stopping statistic, trace statistics)."""
        torch = _torch()
        opts = self._sub_opts(seed, 0, precision, rr_threshold, rr_prob, kw)
        t = torch.empty(self.models[model], dtype=torch.float64, device=self.tdev)
        crit = C.c_double()
        st = TraceStats()
        self._check(lib().rt_subiter_step(self.h, model, int(root), int(dust_packets), int(iteration),
                                          C.byref(opts), C.byref(crit), _ptr(t), C.byref(st)))
        return t, float(crit.value), st.as_dict()

    def subiter_select(self, model: int, frac: float = 0.25):
        """Next subtree root from the recorded energy imbalance: (root, largest imbalance)."""
        root = C.c_int64()
        mx = C.c_double()
        self._check(lib().rt_subiter_select(self.h, model, frac, C.byref(root), C.byref(mx)))
        return int(root.value), float(mx.value)

    def subiter_run(self, model: int, n_steps: int, dust_packets: int, seed: int, frac: float = 0.5,
                    stall: float = 0.8, first_iteration: int = 1, rr_threshold: float = 0.0,
                    rr_prob: float = 0.0, precision: int = FP64, **kw):
        """Automatic iteration after subiter_begin: (temperatures after the last step, roots,
        stopping statistics, crossings per step)."""
        torch = _torch()
        opts = self._sub_opts(seed, 0, precision, rr_threshold, rr_prob, kw)
        roots = np.zeros(n_steps, dtype=np.int64)
        crit = np.zeros(n_steps)
        cross = np.zeros(n_steps, dtype=np.uint64)
        t = torch.empty(self.models[model], dtype=torch.float64, device=self.tdev)
        self._check(lib().rt_subiter_run(self.h, model, n_steps, frac, stall, int(dust_packets),
                                         int(first_iteration), C.byref(opts), _ptr(roots), _ptr(crit),
                                         _ptr(cross), _ptr(t)))
        return t, roots, crit, cross

    def render_map(self, model: int, n_obs, npix: int, lambda_idx, width: float = 0.0,
                   precision: int = FP64):
        torch = _torch()
        nv = np.ascontiguousarray(n_obs, dtype=np.float64)
        li = np.ascontiguousarray(lambda_idx, dtype=np.int32)
        img = torch.empty((len(li), npix, npix), dtype=torch.float64, device=self.tdev)
        cr = C.c_uint64()
        self._check(lib().rt_render_map(self.h, model, _ptr(nv), npix, width, len(li), _ptr(li),
                                        precision, _ptr(img), C.byref(cr)))
        return img, int(cr.value)

    def render_map_noalloc(self, model: int, n_obs, npix: int, lambda_idx, image=None,
                           width: float = 0.0, precision: int = FP64):
        """rt_render_map_noalloc: the map into ``image`` (a device tensor [n_sel, npix, npix]
        float64, allocated here when None); returns (image, crossings)."""
        torch = _torch()
        nv = np.ascontiguousarray(n_obs, dtype=np.float64)
        li = np.ascontiguousarray(lambda_idx, dtype=np.int32)
        if image is None:
            image = torch.empty((len(li), npix, npix), dtype=torch.float64, device=self.tdev)
        cr = C.c_uint64()
        self._check(lib().rt_render_map_noalloc(self.h, model, _ptr(nv), npix, width, len(li), _ptr(li),
                                                precision, _ptr(image), C.byref(cr)))
        return image, int(cr.value)

    def philox(self, key0: int, key1: int, ctr):
        torch = _torch()
        c = self._dev(np.ascontiguousarray(ctr, dtype=np.uint32).view(np.int32), torch.int32)
        out = torch.empty_like(c)
        self._check(lib().rt_philox(self.h, key0, key1, c.numel() // 4, _ptr(c), _ptr(out)))
        return out.cpu().numpy().view(np.uint32).reshape(-1, 4)
