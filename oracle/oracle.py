"""Python binding of the plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark import this module.  The product path never does: it shares no
code with the oracle and must fail loudly when its own HIP library is absent.

The C source (``sbr_oracle.c``) follows the paper's method step by step:
the equiangular icosahedral launch grid (Sec. II.B, eqs. (1)-(2)), SBR
tracing with specular reflection and reception (Sec. III.A, eq. (3)), path
test 1 (double counting), the iterative precise algorithm (Sec. III.B,
eqs. (4)-(6)), path test 2 (validity) and path delay, AOD, AOA and power.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sbr_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
MAX_ORDER = 8

FLAG_STALLED = 1
FLAG_INVALID = 2
FLAG_TARGET_MET = 4


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "sbr_oracle.h"))
    ):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = [
            "gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
            "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
            _SRC, "-o", tmp, "-lquadmath", "-lm",
        ]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("max_order", C.c_int32),
        ("division_n", C.c_int32),
        ("iterations", C.c_int32),
        ("subrays", C.c_int32),
        ("target_err_deg", C.c_double),
        ("freq_hz", C.c_double),
        ("tx_power_dbm", C.c_double),
        ("keep_invalid", C.c_int32),
        ("n_threads", C.c_int32),
        ("launch", C.c_int32),
    ]


class _Cand(C.Structure):
    _fields_ = [
        ("rx", C.c_int32),
        ("order", C.c_int32),
        ("face", C.c_int32 * MAX_ORDER),
        ("ray", C.c_int64),
        ("tan_err", C.c_double),
    ]


class _Path(C.Structure):
    _fields_ = [
        ("rx", C.c_int32),
        ("order", C.c_int32),
        ("face", C.c_int32 * MAX_ORDER),
        ("launch_ray", C.c_int64),
        ("iters_used", C.c_int32),
        ("flags", C.c_uint32),
        ("tan_err", C.c_double),
        ("axis", C.c_double * 3),
        ("delay_s", C.c_double),
        ("aod", C.c_double * 3),
        ("aoa", C.c_double * 3),
        ("power_dbm", C.c_double),
        ("err_angle_deg", C.c_double),
        ("length_m", C.c_double),
        ("exact_delay_s", C.c_double),
        ("exact_aod", C.c_double * 3),
        ("exact_aoa", C.c_double * 3),
        ("exact_power_dbm", C.c_double),
        ("exact_length_m", C.c_double),
        ("init_tan_err", C.c_double),
    ]


class _DPath(C.Structure):
    _fields_ = [
        ("rx", C.c_int32),
        ("wedge", C.c_int32),
        ("launch_ray", C.c_int64),
        ("iters_used", C.c_int32),
        ("flags", C.c_uint32),
        ("tan_err", C.c_double),
        ("axis", C.c_double * 3),
        ("point", C.c_double * 3),
        ("delay_s", C.c_double),
        ("aod", C.c_double * 3),
        ("aoa", C.c_double * 3),
        ("err_angle_deg", C.c_double),
        ("length_m", C.c_double),
        ("exact_point", C.c_double * 3),
        ("exact_delay_s", C.c_double),
        ("exact_aod", C.c_double * 3),
        ("exact_aoa", C.c_double * 3),
        ("exact_length_m", C.c_double),
        ("init_tan_err", C.c_double),
    ]


def _np_dtype(struct):
    fields = []
    for name, ct in struct._fields_:
        if hasattr(ct, "_length_"):
            fields.append((name, np.dtype(ct._type_), (ct._length_,)))
        else:
            fields.append((name, np.dtype(ct)))
    dt = np.dtype(fields, align=True)
    assert dt.itemsize == C.sizeof(struct), (dt.itemsize, C.sizeof(struct))
    return dt


CAND_DTYPE = _np_dtype(_Cand)
PATH_DTYPE = _np_dtype(_Path)
DPATH_DTYPE = _np_dtype(_DPath)

_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        lp = C.POINTER(C.c_int64)
        L.orc_num_rays.restype = C.c_int64
        L.orc_num_rays.argtypes = [C.c_int32]
        L.orc_launch_dirs.argtypes = [C.c_int32, lp, C.c_int64, dp]
        L.orc_num_rays_m.restype = C.c_int64
        L.orc_num_rays_m.argtypes = [C.c_int32, C.c_int32]
        L.orc_launch_dirs_m.argtypes = [C.c_int32, C.c_int32, lp, C.c_int64, dp]
        L.orc_sin_cr.restype = C.c_double
        L.orc_sin_cr.argtypes = [C.c_double]
        L.orc_acos_cr.restype = C.c_double
        L.orc_acos_cr.argtypes = [C.c_double]
        L.orc_fresnel_avg.restype = C.c_double
        L.orc_fresnel_avg.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_trace_rays.argtypes = [dp, ip, C.c_int64, dp, C.c_int32, C.c_int32, C.c_int32, lp,
                                     C.c_int64, C.c_int32, ip, ip, dp]
        L.orc_trace_dirs.argtypes = [dp, ip, C.c_int64, dp, dp, C.c_int64, C.c_int32, ip, ip,
                                     dp, dp]
        L.orc_run.argtypes = [dp, ip, ip, C.c_int64, dp, dp, C.c_int32, dp, dp, C.c_int32,
                              C.POINTER(Params),
                              C.POINTER(C.POINTER(_Cand)), lp,
                              C.POINTER(C.POINTER(_Cand)), lp,
                              C.POINTER(C.POINTER(_Path)), lp]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_refine_history.argtypes = [dp, ip, C.c_int64, dp, C.POINTER(Params), dp, ip, ip,
                                         dp, C.c_int64, dp]
        L.orc_ray_events.argtypes = [dp, ip, C.c_int64, dp, C.c_int32, C.c_int32, C.c_int32, dp,
                                     C.c_int32, lp, C.c_int64, C.c_int32,
                                     C.POINTER(C.POINTER(_Cand)), lp]
        L.orc_path_test1.argtypes = [C.c_void_p, C.c_int64, C.POINTER(C.POINTER(_Cand)), lp]
        L.orc_path_records.argtypes = [dp, ip, ip, C.c_int64, dp, dp, C.c_int32, dp, dp,
                                       C.c_int32, C.POINTER(Params), C.c_void_p, C.c_int64,
                                       C.c_void_p]
        L.orc_wedges.restype = C.c_int64
        L.orc_wedges.argtypes = [dp, ip, C.c_int64, dp, C.c_int64]
        L.orc_diffract.argtypes = [dp, ip, C.c_int64, dp, dp, C.c_int32, C.POINTER(Params),
                                   C.POINTER(C.POINTER(_Cand)), lp,
                                   C.POINTER(C.POINTER(_Cand)), lp,
                                   C.POINTER(C.POINTER(_DPath)), lp]
        L.orc_diffract_history.argtypes = [dp, ip, C.c_int64, dp, C.POINTER(Params), dp, ip, dp,
                                           C.c_int64, dp]
        L.orc_exact_path.argtypes = [dp, ip, ip, C.c_int64, dp, dp, dp, dp, C.c_int32, ip,
                                     C.c_double, C.c_double, dp, dp, dp, ip]
        L.orc_path_jacobian.argtypes = [dp, ip, ip, C.c_int64, dp, dp, C.c_int32, dp, dp,
                                        C.c_int32, ip, C.c_double, C.c_double, dp, dp]
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _l(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _scene_arrays(scene):
    xyz = np.ascontiguousarray(scene["xyz"], dtype=np.float64)
    tri = np.ascontiguousarray(scene["tri"], dtype=np.int64)
    tri_v = np.ascontiguousarray(xyz[tri].reshape(-1, 9)) if len(tri) else np.zeros((0, 9))
    face = np.ascontiguousarray(scene["face_id"], dtype=np.int32)
    mat = np.ascontiguousarray(scene["mat_id"], dtype=np.int32)
    eps = np.asarray(scene["eps_r"], dtype=np.complex128)
    er = np.ascontiguousarray(eps.real)
    ei = np.ascontiguousarray(eps.imag)
    return tri_v, face, mat, er, ei


EQUIANGULAR, EQUIDISTANT_ICOSA, EQUIDISTANT_OCTA = 0, 1, 2


def num_rays(n: int, launch: int = EQUIANGULAR) -> int:
    return int(lib().orc_num_rays_m(launch, n))


def launch_dirs(n: int, ids=None, launch: int = EQUIANGULAR) -> np.ndarray:
    if ids is None:
        m = num_rays(n, launch)
        out = np.empty((m, 3), np.float64)
        rc = lib().orc_launch_dirs_m(launch, n, None, 0, _d(out))
    else:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        out = np.empty((len(ids), 3), np.float64)
        rc = lib().orc_launch_dirs_m(launch, n, _l(ids), len(ids), _d(out))
    if rc:
        raise ValueError("orc_launch_dirs failed (%d)" % rc)
    return out


def sin_cr(x: float) -> float:
    return lib().orc_sin_cr(x)


def acos_cr(x: float) -> float:
    return lib().orc_acos_cr(x)


def fresnel_avg(cos_i: float, eps: complex) -> float:
    return lib().orc_fresnel_avg(cos_i, eps.real, eps.imag)


def trace_rays(scene, tx, n, max_order, ids=None, threads=0, launch=EQUIANGULAR):
    """Per-ray closest hits of segments 0..K: (tri, face, t) arrays [m, K+1]."""
    tri_v, face, _, _, _ = _scene_arrays(scene)
    txa = np.ascontiguousarray(tx, dtype=np.float64)
    if ids is None:
        m = num_rays(n, launch)
        idp = None
    else:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        m = len(ids)
        idp = _l(ids)
    ot = np.empty((m, max_order + 1), np.int32)
    of = np.empty((m, max_order + 1), np.int32)
    oT = np.empty((m, max_order + 1), np.float64)
    rc = lib().orc_trace_rays(_d(tri_v), _i(face), len(face), _d(txa), n, launch, max_order, idp,
                              m, threads, _i(ot), _i(of), _d(oT))
    if rc:
        raise ValueError("orc_trace_rays failed (%d)" % rc)
    return ot, of, oT


def trace_dirs(scene, tx, dirs, max_order):
    """Closest hits of segments 0..K for explicit directions: (tri, face, t, D)."""
    tri_v, face, _, _, _ = _scene_arrays(scene)
    txa = np.ascontiguousarray(tx, dtype=np.float64)
    dirs = np.ascontiguousarray(np.asarray(dirs, np.float64).reshape(-1, 3))
    m = len(dirs)
    ot = np.empty((m, max_order + 1), np.int32)
    of = np.empty((m, max_order + 1), np.int32)
    oT = np.empty((m, max_order + 1), np.float64)
    oD = np.empty((m, max_order + 1), np.float64)
    rc = lib().orc_trace_dirs(_d(tri_v), _i(face), len(face), _d(txa), _d(dirs), m, max_order,
                              _i(ot), _i(of), _d(oT), _d(oD))
    if rc:
        raise ValueError("orc_trace_dirs failed (%d)" % rc)
    return ot, of, oT, oD


def make_params(max_order=3, division_n=20, iterations=3, subrays=6, target_err_deg=0.0,
                freq_hz=28e9, tx_power_dbm=0.0, keep_invalid=False, threads=0,
                launch=EQUIANGULAR) -> Params:
    return Params(max_order, division_n, iterations, subrays, target_err_deg, freq_hz,
                  tx_power_dbm, int(bool(keep_invalid)), threads, launch)


def _take(ptr, n, dtype):
    if n == 0 or not ptr:
        out = np.zeros(0, dtype)
    else:
        buf = C.cast(ptr, C.POINTER(C.c_char * (n * dtype.itemsize))).contents
        out = np.frombuffer(bytes(buf), dtype=dtype).copy()
    lib().orc_free(C.cast(ptr, C.c_void_p))
    return out


def run(scene, tx, rx, **kw):
    """Whole method; returns dict(candidates, unique, paths) as structured arrays."""
    tri_v, face, mat, er, ei = _scene_arrays(scene)
    txa = np.ascontiguousarray(tx, dtype=np.float64)
    rxa = np.ascontiguousarray(np.asarray(rx, dtype=np.float64).reshape(-1, 3))
    prm = make_params(**kw)
    cp = C.POINTER(_Cand)()
    up = C.POINTER(_Cand)()
    pp = C.POINTER(_Path)()
    nc, nu, npth = C.c_int64(), C.c_int64(), C.c_int64()
    rc = lib().orc_run(_d(tri_v), _i(face), _i(mat), len(face), _d(er), _d(ei), len(er),
                       _d(txa), _d(rxa), len(rxa), C.byref(prm), C.byref(cp), C.byref(nc),
                       C.byref(up), C.byref(nu), C.byref(pp), C.byref(npth))
    if rc:
        raise ValueError("orc_run failed (%d)" % rc)
    return {
        "candidates": _take(cp, nc.value, CAND_DTYPE),
        "unique": _take(up, nu.value, CAND_DTYPE),
        "paths": _take(pp, npth.value, PATH_DTYPE),
    }


def ray_events(scene, tx, rx, n, max_order, ids, threads=0, launch=EQUIANGULAR):
    """Reception events of the launch rays `ids` only (step 1 of run())."""
    tri_v, face, _, _, _ = _scene_arrays(scene)
    txa = np.ascontiguousarray(tx, dtype=np.float64)
    rxa = np.ascontiguousarray(np.asarray(rx, dtype=np.float64).reshape(-1, 3))
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    cp = C.POINTER(_Cand)()
    nc = C.c_int64()
    rc = lib().orc_ray_events(_d(tri_v), _i(face), len(face), _d(txa), n, launch, max_order, _d(rxa),
                              len(rxa), _l(ids), len(ids), threads, C.byref(cp), C.byref(nc))
    if rc:
        raise ValueError("orc_ray_events failed (%d)" % rc)
    return _take(cp, nc.value, CAND_DTYPE)


def path_test1(events):
    """Path test 1 over reception events (a CAND_DTYPE array): one winner per
    (rx, order, face sequence), sorted by that key."""
    ev = np.ascontiguousarray(events, dtype=CAND_DTYPE)
    up = C.POINTER(_Cand)()
    nu = C.c_int64()
    rc = lib().orc_path_test1(ev.ctypes.data_as(C.c_void_p), len(ev), C.byref(up), C.byref(nu))
    if rc:
        raise ValueError("orc_path_test1 failed (%d)" % rc)
    return _take(up, nu.value, CAND_DTYPE)


def path_records(scene, tx, rx, winners, **kw):
    """Path records (steps 3-4 of run()) for given path-test-1 winners
    (a CAND_DTYPE array); invalid paths are flagged, not dropped."""
    tri_v, face, mat, er, ei = _scene_arrays(scene)
    txa = np.ascontiguousarray(tx, dtype=np.float64)
    rxa = np.ascontiguousarray(np.asarray(rx, dtype=np.float64).reshape(-1, 3))
    win = np.ascontiguousarray(winners, dtype=CAND_DTYPE)
    out = np.zeros(len(win), PATH_DTYPE)
    prm = make_params(**kw)
    rc = lib().orc_path_records(_d(tri_v), _i(face), _i(mat), len(face), _d(er), _d(ei), len(er),
                                _d(txa), _d(rxa), len(rxa), C.byref(prm),
                                win.ctypes.data_as(C.c_void_p), len(win),
                                out.ctypes.data_as(C.c_void_p))
    if rc:
        raise ValueError("orc_path_records failed (%d)" % rc)
    return out


def refine_history(scene, tx, rx_rows, orders, faces, axes, **kw):
    """tan(theta_error) after each iteration for the given path rows."""
    tri_v, face, _, _, _ = _scene_arrays(scene)
    prm = make_params(**kw)
    rx_rows = np.ascontiguousarray(rx_rows, dtype=np.float64).reshape(-1, 3)
    orders = np.ascontiguousarray(orders, dtype=np.int32)
    fz = np.full((len(orders), MAX_ORDER), -1, np.int32)
    faces = np.asarray(faces)
    fz[:, : faces.shape[1]] = faces
    axes = np.ascontiguousarray(axes, dtype=np.float64).reshape(-1, 3)
    hist = np.empty((len(orders), prm.iterations + 1), np.float64)
    txa = np.ascontiguousarray(tx, dtype=np.float64)
    rc = lib().orc_refine_history(_d(tri_v), _i(face), len(face), _d(txa), C.byref(prm),
                                  _d(rx_rows), _i(orders), _i(fz), _d(axes), len(orders),
                                  _d(hist))
    if rc:
        raise ValueError("orc_refine_history failed (%d)" % rc)
    return hist


def exact_path(scene, tx, rx, faces, freq_hz=28e9, tx_power_dbm=0.0):
    """Image-method path for one face sequence: (points, length, power_dbm, valid)."""
    tri_v, face, mat, er, ei = _scene_arrays(scene)
    faces = np.ascontiguousarray(faces, dtype=np.int32)
    k = len(faces)
    pts = np.zeros((max(k, 1), 3), np.float64)
    L, P, V = C.c_double(), C.c_double(), C.c_int32()
    txa = np.ascontiguousarray(tx, dtype=np.float64)
    rxa = np.ascontiguousarray(rx, dtype=np.float64)
    rc = lib().orc_exact_path(_d(tri_v), _i(face), _i(mat), len(face), _d(er), _d(ei),
                              _d(txa), _d(rxa), k, _i(faces) if k else None, freq_hz,
                              tx_power_dbm, _d(pts), C.byref(L), C.byref(P), C.byref(V))
    if rc:
        raise ValueError("orc_exact_path failed (%d)" % rc)
    return pts[:k], L.value, P.value, bool(V.value)


def path_jacobian(scene, tx, rx, faces, freq_hz=28e9, tx_power_dbm=0.0):
    """Image-method path quantities of one face sequence and their analytic
    Jacobian: (values [8] = delay, AOD (3), AOA (3), power;
    jac [8][6 + 2 M] over Tx (3), Rx (3), (re, im) of each material)."""
    tri_v, face, mat, er, ei = _scene_arrays(scene)
    faces = np.ascontiguousarray(faces, dtype=np.int32)
    k = len(faces)
    val = np.zeros(8, np.float64)
    jac = np.zeros((8, 6 + 2 * len(er)), np.float64)
    txa = np.ascontiguousarray(tx, dtype=np.float64)
    rxa = np.ascontiguousarray(rx, dtype=np.float64)
    rc = lib().orc_path_jacobian(_d(tri_v), _i(face), _i(mat), len(face), _d(er), _d(ei),
                                 len(er), _d(txa), _d(rxa), k, _i(faces) if k else None,
                                 freq_hz, tx_power_dbm, _d(val), _d(jac))
    if rc:
        raise ValueError("orc_path_jacobian failed (%d)" % rc)
    return val, jac


def wedges(scene):
    """Wedges of the scene (order-1 diffraction edges): dict of arrays a, b, e,
    u0, u1 [W, 3] and faces [W, 2]."""
    tri_v, face, _, _, _ = _scene_arrays(scene)
    n = lib().orc_wedges(_d(tri_v), _i(face), len(face), None, 0)
    if n < 0:
        raise ValueError("orc_wedges failed")
    out = np.zeros((max(n, 1), 17), np.float64)
    lib().orc_wedges(_d(tri_v), _i(face), len(face), _d(out), n)
    out = out[:n]
    return {"a": out[:, 0:3], "b": out[:, 3:6], "e": out[:, 6:9], "u0": out[:, 9:12],
            "u1": out[:, 12:15], "faces": out[:, 15:17].astype(np.int32)}


def diffract(scene, tx, rx, **kw):
    """Order-1 diffraction (events, winners, paths); events and winners are
    CAND_DTYPE with order 1 and face[0] = wedge index."""
    tri_v, face, _, _, _ = _scene_arrays(scene)
    txa = np.ascontiguousarray(tx, dtype=np.float64)
    rxa = np.ascontiguousarray(np.asarray(rx, dtype=np.float64).reshape(-1, 3))
    prm = make_params(**kw)
    cp = C.POINTER(_Cand)()
    up = C.POINTER(_Cand)()
    pp = C.POINTER(_DPath)()
    nc, nu, npth = C.c_int64(), C.c_int64(), C.c_int64()
    rc = lib().orc_diffract(_d(tri_v), _i(face), len(face), _d(txa), _d(rxa), len(rxa),
                            C.byref(prm), C.byref(cp), C.byref(nc), C.byref(up), C.byref(nu),
                            C.byref(pp), C.byref(npth))
    if rc:
        raise ValueError("orc_diffract failed (%d)" % rc)
    return {
        "candidates": _take(cp, nc.value, CAND_DTYPE),
        "unique": _take(up, nu.value, CAND_DTYPE),
        "paths": _take(pp, npth.value, DPATH_DTYPE),
    }


def diffract_history(scene, tx, rx_rows, wedge_ids, axes, **kw):
    """tan(theta_error) after each iteration for diffraction rows."""
    tri_v, face, _, _, _ = _scene_arrays(scene)
    prm = make_params(**kw)
    rx_rows = np.ascontiguousarray(rx_rows, dtype=np.float64).reshape(-1, 3)
    wid = np.ascontiguousarray(wedge_ids, dtype=np.int32)
    axes = np.ascontiguousarray(axes, dtype=np.float64).reshape(-1, 3)
    hist = np.empty((len(wid), prm.iterations + 1), np.float64)
    txa = np.ascontiguousarray(tx, dtype=np.float64)
    rc = lib().orc_diffract_history(_d(tri_v), _i(face), len(face), _d(txa), C.byref(prm),
                                    _d(rx_rows), _i(wid), _d(axes), len(wid), _d(hist))
    if rc:
        raise ValueError("orc_diffract_history failed (%d)" % rc)
    return hist
