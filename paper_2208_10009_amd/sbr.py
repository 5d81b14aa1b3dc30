"""Thin Python binding of the HIP library (include/sbr.h).

Argument marshalling only: every stage of the method runs in the library's
HIP kernels.  ``torch`` is imported first so that the library and PyTorch share
one HIP runtime; PyTorch supplies the device and the stream.  If the library
has not been built, every entry point raises -- there is no fallback.

Names follow the C ABI: ``Context.launch_grid`` is ``sbr_launch_grid``,
``Scene.trace`` is ``sbr_trace``, ``Scene.candidates`` is ``sbr_candidates``,
``Scene.trace_rays`` is ``sbr_trace_rays``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbr.so")
MAX_ORDER = 8

OK = 0
E_INVALID_ARG = -1
E_NO_SCENE = -2
E_NO_BVH = -3
E_CAPACITY = -4
E_OOM = -5
E_DEVICE = -6
E_INTERNAL = -7
E_SCRATCH = -8

FLAG_KEEP_INVALID = 1
FLAG_FRESH_GRID = 2
FLAG_GRAPH = 4
PATH_STALLED = 1
PATH_INVALID = 2
PATH_TARGET_MET = 4

# every function declared in include/sbr.h
EXPORTS = (
    "sbr_context_create", "sbr_context_destroy", "sbr_scene_upload", "sbr_bvh_build",
    "sbr_scene_destroy", "sbr_trace", "sbr_trace_device", "sbr_candidates", "sbr_launch_grid",
    "sbr_trace_rays",
    "sbr_trace_counters", "sbr_trace_batch", "sbr_context_get_tuning", "sbr_context_set_tuning",
    "sbr_path_gradients", "sbr_status_string", "sbr_last_error", "sbr_trace_device_noalloc",
    "sbr_scene_wedges", "sbr_diffract", "sbr_diff_candidates",
)


class TraceParams(C.Structure):
    _fields_ = [
        ("max_order", C.c_int32),
        ("division_n", C.c_int32),
        ("iterations", C.c_int32),
        ("subrays", C.c_int32),
        ("target_err_deg", C.c_double),
        ("freq_hz", C.c_double),
        ("tx_power_dbm", C.c_double),
        ("flags", C.c_uint32),
        ("launch", C.c_int32),
    ]


class Job(C.Structure):
    _fields_ = [("scene", C.c_int32), ("rx_first", C.c_int32), ("n_rx", C.c_int32),
                ("reserved", C.c_int32), ("tx", C.c_double * 3), ("params", TraceParams)]


class Tuning(C.Structure):
    _fields_ = [("trace_chunk", C.c_int32), ("persist_blocks", C.c_int32),
                ("trace_block", C.c_int32), ("stack_depth", C.c_int32),
                ("lds_budget", C.c_int32), ("rx_tree_min", C.c_int32),
                ("lookahead_max_paths", C.c_int64), ("lookahead_depth", C.c_int32),
                ("lookahead3_max_paths", C.c_int32), ("grid_check_log2", C.c_int32),
                ("ray_order", C.c_int32), ("refine_segments", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Complex(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class BvhParams(C.Structure):
    _fields_ = [("max_leaf_size", C.c_int32), ("sah_bins", C.c_int32), ("split_pct", C.c_int32)]


class TraceStats(C.Structure):
    _fields_ = [
        ("n_rays", C.c_int64), ("n_candidates", C.c_int64), ("n_unique", C.c_int64),
        ("n_paths", C.c_int64),
        ("ms_launch", C.c_double), ("ms_trace", C.c_double), ("ms_dedup", C.c_double),
        ("ms_refine", C.c_double), ("ms_solve", C.c_double), ("ms_emit", C.c_double),
        ("ms_total", C.c_double),
        ("lds_bytes", C.c_int64), ("lds_nodes", C.c_int64), ("lds_tris", C.c_int64),
        ("lds_max", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


PATH_DTYPE = np.dtype([
    ("rx", np.int32), ("order", np.int32), ("face", np.int32, (MAX_ORDER,)),
    ("launch_ray", np.int64), ("iters_used", np.int32), ("flags", np.uint32),
    ("tan_err", np.float64), ("axis", np.float64, (3,)),
    ("delay_s", np.float64), ("aod", np.float64, (3,)), ("aoa", np.float64, (3,)),
    ("power_dbm", np.float64), ("err_angle_deg", np.float64), ("length_m", np.float64),
    ("exact_delay_s", np.float64), ("exact_aod", np.float64, (3,)),
    ("exact_aoa", np.float64, (3,)), ("exact_power_dbm", np.float64),
    ("exact_length_m", np.float64), ("init_tan_err", np.float64),
], align=True)
assert PATH_DTYPE.itemsize == 248

DPATH_DTYPE = np.dtype([
    ("rx", np.int32), ("wedge", np.int32), ("launch_ray", np.int64), ("iters_used", np.int32),
    ("flags", np.uint32), ("tan_err", np.float64), ("axis", np.float64, (3,)),
    ("point", np.float64, (3,)), ("delay_s", np.float64), ("aod", np.float64, (3,)),
    ("aoa", np.float64, (3,)), ("err_angle_deg", np.float64), ("length_m", np.float64),
    ("exact_point", np.float64, (3,)), ("exact_delay_s", np.float64),
    ("exact_aod", np.float64, (3,)), ("exact_aoa", np.float64, (3,)),
    ("exact_length_m", np.float64), ("init_tan_err", np.float64),
], align=True)
assert DPATH_DTYPE.itemsize == 248

WEDGE_DTYPE = np.dtype([("a", np.float64, (3,)), ("b", np.float64, (3,)), ("face", np.int32, (2,))],
                       align=True)
assert WEDGE_DTYPE.itemsize == 56

CAND_DTYPE = np.dtype([
    ("rx", np.int32), ("order", np.int32), ("face", np.int32, (MAX_ORDER,)),
    ("ray", np.int64), ("tan_err", np.float64),
], align=True)
assert CAND_DTYPE.itemsize == 56


class SbrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (_status_string(status), status, msg))
        self.status = status


_lib = None


def _status_string(st):
    try:
        return lib().sbr_status_string(st).decode()
    except Exception:  # pragma: no cover - only when the library is missing
        return "status"


def lib(load_torch: bool = True):
    """The loaded library.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            "HIP library %s is missing: build it with __graft_entry__.build() "
            "(there is no CPU fallback)" % LIB_PATH)
    if load_torch:
        import torch  # noqa: F401  (shares its HIP runtime with the library)
    L = C.CDLL(LIB_PATH)
    vp, dp, ip, lp = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    L.sbr_status_string.restype = C.c_char_p
    L.sbr_status_string.argtypes = [C.c_int32]
    L.sbr_last_error.restype = C.c_char_p
    L.sbr_last_error.argtypes = [vp]
    L.sbr_context_create.argtypes = [C.c_int32, vp, C.POINTER(vp)]
    L.sbr_context_destroy.argtypes = [vp]
    L.sbr_scene_upload.argtypes = [vp, dp, C.c_int64, ip, ip, ip, C.c_int64,
                                   C.POINTER(Complex), C.c_int32, C.POINTER(vp)]
    L.sbr_bvh_build.argtypes = [vp, C.POINTER(BvhParams)]
    L.sbr_scene_destroy.argtypes = [vp]
    L.sbr_trace.argtypes = [vp, dp, dp, C.c_int32, C.POINTER(TraceParams), vp, C.c_int64, lp,
                            C.POINTER(TraceStats)]
    L.sbr_trace_device.argtypes = [vp, dp, vp, C.c_int32, C.POINTER(TraceParams), vp, C.c_int64,
                                   lp, C.POINTER(TraceStats)]
    L.sbr_trace_device_noalloc.argtypes = [vp, dp, vp, C.c_int32, C.POINTER(TraceParams), vp,
                                           C.c_int64, lp, C.POINTER(TraceStats)]
    L.sbr_scene_wedges.argtypes = [vp, vp, C.c_int64, lp]
    L.sbr_diffract.argtypes = [vp, dp, dp, C.c_int32, C.POINTER(TraceParams), vp, C.c_int64, lp,
                               C.POINTER(TraceStats)]
    L.sbr_diff_candidates.argtypes = [vp, dp, dp, C.c_int32, C.POINTER(TraceParams), vp,
                                      C.c_int64, lp]
    L.sbr_candidates.argtypes = [vp, dp, dp, C.c_int32, C.POINTER(TraceParams), vp, C.c_int64,
                                 lp]
    L.sbr_launch_grid.argtypes = [vp, C.c_int32, C.c_int32, C.c_int64, C.c_int64, dp]
    L.sbr_trace_rays.argtypes = [vp, dp, C.c_int32, C.c_int32, C.c_int32, C.c_int64, C.c_int64,
                                 ip, dp]
    L.sbr_trace_counters.argtypes = [vp, dp, dp, C.c_int32, C.POINTER(TraceParams), lp]
    L.sbr_context_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
    L.sbr_context_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
    L.sbr_trace_batch.argtypes = [vp, C.POINTER(vp), C.c_int32, C.POINTER(Job), C.c_int32, dp,
                                  C.c_int32, vp, C.c_int64, lp, C.POINTER(TraceStats)]
    for name in EXPORTS:
        getattr(L, name).restype = getattr(L, name).restype or C.c_int32
    L.sbr_status_string.restype = C.c_char_p
    L.sbr_last_error.restype = C.c_char_p
    _lib = L
    return L


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


EQUIANGULAR, EQUIDISTANT_ICOSA, EQUIDISTANT_OCTA = 0, 1, 2


def num_rays(n: int, launch: int = EQUIANGULAR) -> int:
    """Launch rays of division n: 10 n^2 + 2 (icosahedron), 4 n^2 + 2 (octahedron)."""
    return (4 if launch == EQUIDISTANT_OCTA else 10) * n * n + 2


def make_params(max_order=3, division_n=20, iterations=3, subrays=6, target_err_deg=0.0,
                freq_hz=28e9, tx_power_dbm=0.0, keep_invalid=False, fresh_grid=False,
                launch=EQUIANGULAR, graph=False):
    flags = (FLAG_KEEP_INVALID if keep_invalid else 0) | (FLAG_FRESH_GRID if fresh_grid else 0) | \
        (FLAG_GRAPH if graph else 0)
    return TraceParams(max_order, division_n, iterations, subrays, target_err_deg, freq_hz,
                       tx_power_dbm, flags, launch)


class Context:
    """sbr_context_create on `device`, bound to torch's current stream there."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        L = lib()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible to torch")
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        h = C.c_void_p()
        st = L.sbr_context_create(device, C.c_void_p(handle), C.byref(h))
        if st != OK:
            raise SbrError(st, L.sbr_last_error(None).decode())
        self.h = h
        self.device = device
        self.scenes = []

    def _check(self, st):
        if st != OK:
            raise SbrError(st, lib().sbr_last_error(self.h).decode())

    def launch_grid(self, n: int, first: int = 0, count: int | None = None,
                    launch: int = EQUIANGULAR) -> np.ndarray:
        N = num_rays(n, launch)
        if count is None:
            count = N - first
        out = np.empty((count, 3), np.float64)
        self._check(lib().sbr_launch_grid(self.h, launch, n, first, count, _d(out)))
        return out

    def tuning(self) -> dict:
        """sbr_context_get_tuning"""
        t = Tuning()
        self._check(lib().sbr_context_get_tuning(self.h, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        """sbr_context_set_tuning: update some fields, keep the others."""
        cur = self.tuning()
        cur.update(kw)
        t = Tuning(**cur)
        self._check(lib().sbr_context_set_tuning(self.h, C.byref(t)))

    def scene(self, scene: dict, max_leaf_size: int = 4, sah_bins: int = 64,
              split_pct: int = 0) -> "Scene":
        return Scene(self, scene, max_leaf_size, sah_bins, split_pct)

    def trace_batch(self, scenes, jobs, rx, capacity: int | None = None):
        """sbr_trace_batch.  scenes: list of Scene; jobs: list of dicts with
        scene (index), tx, rx_first, n_rx and trace parameters (as for
        Scene.trace); rx: [n_rx_total, 3].  Returns (paths, stats)."""
        rxa = np.ascontiguousarray(rx, np.float64).reshape(-1, 3)
        sh = (C.c_void_p * len(scenes))(*[s.h for s in scenes])
        arr = (Job * max(len(jobs), 1))()
        for i, j in enumerate(jobs):
            prm = {k: v for k, v in j.items() if k not in ("scene", "tx", "rx_first", "n_rx")}
            arr[i] = Job(int(j["scene"]), int(j["rx_first"]), int(j["n_rx"]), 0,
                         (C.c_double * 3)(*[float(v) for v in j["tx"]]), make_params(**prm))
        cap = capacity if capacity is not None else 16384
        while True:
            out = np.zeros(max(cap, 1), PATH_DTYPE)
            n = C.c_int64()
            stats = TraceStats()
            st = lib().sbr_trace_batch(self.h, sh, len(scenes), arr, len(jobs), _d(rxa), len(rxa),
                                       out.ctypes.data_as(C.c_void_p), cap, C.byref(n),
                                       C.byref(stats))
            if st == E_CAPACITY and capacity is None:
                cap = n.value
                continue
            self._check(st)
            return out[: n.value].copy(), stats.as_dict()

    def close(self):
        for s in list(self.scenes):
            s.close()
        if self.h:
            self._check(lib().sbr_context_destroy(self.h))
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


class Scene:
    """sbr_scene_upload + sbr_bvh_build of a scene dict (see scenes.py)."""

    def __init__(self, ctx: Context, scene: dict, max_leaf_size=4, sah_bins=64, split_pct=0):
        self.ctx = ctx
        xyz = np.ascontiguousarray(scene["xyz"], np.float64).reshape(-1, 3)
        tri = np.ascontiguousarray(scene["tri"], np.int32).reshape(-1, 3)
        face = np.ascontiguousarray(scene["face_id"], np.int32)
        mat = np.ascontiguousarray(scene["mat_id"], np.int32)
        eps = np.asarray(scene["eps_r"], np.complex128).reshape(-1)
        ce = (Complex * max(len(eps), 1))(*[Complex(e.real, e.imag) for e in eps])
        h = C.c_void_p()
        ctx._check(lib().sbr_scene_upload(ctx.h, _d(xyz), len(xyz), _i(tri), _i(face), _i(mat),
                                          len(tri), ce, len(eps), C.byref(h)))
        self.h = h
        ctx.scenes.append(self)
        bp = BvhParams(max_leaf_size, sah_bins, split_pct)
        ctx._check(lib().sbr_bvh_build(self.h, C.byref(bp)))
        self.n_tri = len(tri)

    def trace(self, tx, rx, capacity: int | None = None, **params):
        """sbr_trace: returns (paths structured array, stats dict)."""
        txa = np.ascontiguousarray(tx, np.float64).reshape(3)
        rxa = np.ascontiguousarray(rx, np.float64).reshape(-1, 3)
        prm = make_params(**params)
        cap = capacity if capacity is not None else 4096
        while True:
            out = np.zeros(max(cap, 1), PATH_DTYPE)
            n = C.c_int64()
            stats = TraceStats()
            st = lib().sbr_trace(self.h, _d(txa), _d(rxa), len(rxa), C.byref(prm),
                                 out.ctypes.data_as(C.c_void_p), cap, C.byref(n),
                                 C.byref(stats))
            if st == E_CAPACITY and capacity is None:
                cap = n.value
                continue
            self.ctx._check(st)
            return out[: n.value].copy(), stats.as_dict()

    def trace_device(self, tx, rx, out=None, **params):
        """sbr_trace_device: rx is a float64 [n_rx, 3] tensor on the context's
        device; returns (paths as a uint8 [n, record] device tensor, stats).
        `out` (a uint8 device tensor of whole records) is reused when large
        enough; otherwise, or on SBR_E_CAPACITY, a larger one is allocated."""
        import torch
        txa = np.ascontiguousarray(tx, np.float64).reshape(3)
        assert rx.dtype == torch.float64 and rx.is_cuda and rx.dim() == 2 and rx.shape[1] == 3
        rx = rx.contiguous()
        prm = make_params(**params)
        rec = PATH_DTYPE.itemsize
        if out is None:
            out = torch.empty((4096, rec), dtype=torch.uint8, device=rx.device)
        while True:
            n = C.c_int64()
            stats = TraceStats()
            st = lib().sbr_trace_device(self.h, _d(txa), C.c_void_p(rx.data_ptr()), rx.shape[0],
                                        C.byref(prm), C.c_void_p(out.data_ptr()), out.shape[0],
                                        C.byref(n), C.byref(stats))
            if st == E_CAPACITY:
                out = torch.empty((n.value, rec), dtype=torch.uint8, device=rx.device)
                continue
            self.ctx._check(st)
            return out[: n.value], stats.as_dict()

    def trace_device_noalloc(self, tx, rx, out, **params):
        """sbr_trace_device_noalloc: as trace_device, into the caller's `out`
        (a uint8 [capacity, record] device tensor); nothing is allocated.
        Returns (paths view of out, stats); raises SbrError when out is too
        small or the call exceeds the fixed scratch."""
        import torch
        txa = np.ascontiguousarray(tx, np.float64).reshape(3)
        assert rx.dtype == torch.float64 and rx.is_cuda and rx.dim() == 2 and rx.shape[1] == 3
        assert rx.is_contiguous(), "rx must be contiguous (nothing is copied)"
        assert out.dtype == torch.uint8 and out.is_cuda and out.is_contiguous()
        assert out.dim() == 2 and out.shape[1] == PATH_DTYPE.itemsize
        prm = make_params(**params)
        n = C.c_int64()
        stats = TraceStats()
        st = lib().sbr_trace_device_noalloc(self.h, _d(txa), C.c_void_p(rx.data_ptr()),
                                            rx.shape[0], C.byref(prm), C.c_void_p(out.data_ptr()),
                                            out.shape[0], C.byref(n), C.byref(stats))
        self.ctx._check(st)
        return out[: n.value], stats.as_dict()

    def candidates(self, tx, rx, capacity: int | None = None, **params):
        """sbr_candidates: reception events before path test 1, sorted."""
        txa = np.ascontiguousarray(tx, np.float64).reshape(3)
        rxa = np.ascontiguousarray(rx, np.float64).reshape(-1, 3)
        prm = make_params(**params)
        cap = capacity if capacity is not None else 16384
        while True:
            out = np.zeros(max(cap, 1), CAND_DTYPE)
            n = C.c_int64()
            st = lib().sbr_candidates(self.h, _d(txa), _d(rxa), len(rxa), C.byref(prm),
                                      out.ctypes.data_as(C.c_void_p), cap, C.byref(n))
            if st == E_CAPACITY and capacity is None:
                cap = n.value
                continue
            self.ctx._check(st)
            return out[: n.value].copy()

    def wedges(self):
        """sbr_scene_wedges: structured array of (a, b, face)."""
        n = C.c_int64()
        st = lib().sbr_scene_wedges(self.h, None, 0, C.byref(n))
        if st != E_CAPACITY:  # the count query of a scene with wedges
            self.ctx._check(st)
        out = np.zeros(max(n.value, 1), WEDGE_DTYPE)
        self.ctx._check(lib().sbr_scene_wedges(self.h, out.ctypes.data_as(C.c_void_p), n.value,
                                               C.byref(n)))
        return out[: n.value]

    def diffract(self, tx, rx, capacity: int | None = None, **params):
        """sbr_diffract: order-1 diffraction paths (DPATH_DTYPE) and stats."""
        txa = np.ascontiguousarray(tx, np.float64).reshape(3)
        rxa = np.ascontiguousarray(rx, np.float64).reshape(-1, 3)
        prm = make_params(**params)
        cap = capacity if capacity is not None else 4096
        while True:
            out = np.zeros(max(cap, 1), DPATH_DTYPE)
            n = C.c_int64()
            stats = TraceStats()
            st = lib().sbr_diffract(self.h, _d(txa), _d(rxa), len(rxa), C.byref(prm),
                                    out.ctypes.data_as(C.c_void_p), cap, C.byref(n),
                                    C.byref(stats))
            if st == E_CAPACITY and capacity is None:
                cap = n.value
                continue
            self.ctx._check(st)
            return out[: n.value].copy(), stats.as_dict()

    def diff_candidates(self, tx, rx, capacity: int | None = None, **params):
        """sbr_diff_candidates: diffraction events before path test 1, sorted."""
        txa = np.ascontiguousarray(tx, np.float64).reshape(3)
        rxa = np.ascontiguousarray(rx, np.float64).reshape(-1, 3)
        prm = make_params(**params)
        cap = capacity if capacity is not None else 16384
        while True:
            out = np.zeros(max(cap, 1), CAND_DTYPE)
            n = C.c_int64()
            st = lib().sbr_diff_candidates(self.h, _d(txa), _d(rxa), len(rxa), C.byref(prm),
                                           out.ctypes.data_as(C.c_void_p), cap, C.byref(n))
            if st == E_CAPACITY and capacity is None:
                cap = n.value
                continue
            self.ctx._check(st)
            return out[: n.value].copy()

    def trace_rays(self, tx, n: int, max_order: int, first: int = 0, count: int | None = None,
                   launch: int = EQUIANGULAR):
        """sbr_trace_rays: (tri [count, K+1] input indices, t [count, K+1])."""
        N = num_rays(n, launch)
        if count is None:
            count = N - first
        txa = np.ascontiguousarray(tx, np.float64).reshape(3)
        ot = np.empty((count, max_order + 1), np.int32)
        oT = np.empty((count, max_order + 1), np.float64)
        self.ctx._check(lib().sbr_trace_rays(self.h, _d(txa), launch, n, max_order, first, count,
                                             _i(ot), _d(oT)))
        return ot, oT

    def trace_counters(self, tx, rx, **params):
        """sbr_trace_counters: dict of segments, nodes, tris, events,
        tris_run, wave_node_steps, wave_tri_steps, wave_seg_steps,
        wave_rx_steps, rx_nodes, rx_tests."""
        txa = np.ascontiguousarray(tx, np.float64).reshape(3)
        rxa = np.ascontiguousarray(rx, np.float64).reshape(-1, 3)
        prm = make_params(**params)
        out = np.zeros(12, np.int64)
        self.ctx._check(lib().sbr_trace_counters(self.h, _d(txa), _d(rxa), len(rxa), C.byref(prm),
                                                 out.ctypes.data_as(C.POINTER(C.c_int64))))
        return dict(zip(("segments", "nodes", "tris", "events", "tris_run", "wave_node_steps",
                         "wave_tri_steps", "wave_seg_steps", "wave_rx_steps", "rx_nodes",
                         "rx_tests"),
                        (int(v) for v in out)))

    def close(self):
        if self.h:
            self.ctx._check(lib().sbr_scene_destroy(self.h))
            self.h = None
            self.ctx.scenes.remove(self)
