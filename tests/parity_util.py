"""Shared comparison helpers of the GPU parity tests (the bars of the HIP
path against the FP64 oracle)."""
import numpy as np

DELAY_RTOL = 1e-6
ANGLE_TOL_DEG = 1e-4
POWER_TOL_DB = 1e-3


def angle_deg(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    c = np.cross(a, b)
    return np.degrees(np.arctan2(np.linalg.norm(c, axis=-1), np.sum(a * b, axis=-1)))


def bits(x):
    return np.ascontiguousarray(x, np.float64).view(np.uint64)


def key_of(rec):
    return (int(rec["rx"]), int(rec["order"])) + tuple(int(f) for f in rec["face"])


def compare_paths(g, o):
    assert len(g) == len(o)
    for f in ("rx", "order", "face", "launch_ray", "iters_used", "flags"):
        assert np.array_equal(g[f], o[f]), f
    # the refinement is decided in FP64 with the oracle's operation order
    assert np.array_equal(bits(g["tan_err"]), bits(o["tan_err"]))
    assert np.array_equal(bits(g["axis"]), bits(o["axis"]))
    assert np.array_equal(bits(g["init_tan_err"]), bits(o["init_tan_err"]))
    for f in ("delay_s", "exact_delay_s", "length_m", "exact_length_m"):
        assert np.all(np.abs(g[f] - o[f]) <= DELAY_RTOL * np.abs(o[f])), f
    for f in ("aod", "aoa", "exact_aod", "exact_aoa"):
        assert np.all(angle_deg(g[f], o[f]) <= ANGLE_TOL_DEG), f
    assert np.all(np.abs(g["err_angle_deg"] - o["err_angle_deg"]) <= ANGLE_TOL_DEG)
    for f in ("power_dbm", "exact_power_dbm"):
        assert np.all(np.abs(g[f] - o[f]) <= POWER_TOL_DB), f
