"""GPU parity of order-1 diffraction (Sec. III.A wedges, Sec. III.B, Sec. IV)
through the C ABI against the FP64 oracle on the same seeded inputs.

Bars: wedges, events (receiver, wedge, ray, tan of the error angle), path
sets, launch rays, iterations, flags, the refined axis and diffraction point
and the exact point bit-exact (every decision and every reported coordinate
is FP64 in the oracle's operation order); delays relative 1e-6 and angles
1e-4 degree (the reported angle error goes through atan)."""
import math

import numpy as np
import pytest

from paper_2208_10009_amd import scenes

pytestmark = pytest.mark.gpu

from parity_util import ANGLE_TOL_DEG, DELAY_RTOL, angle_deg, bits  # noqa: E402


def box_scene(*boxes):
    b = scenes.SceneBuilder()
    for lo, hi in boxes:
        b.box(lo, hi, 0)
    return b.scene([5.3 - 0.4j])


def sort_events(a):
    """Events in the canonical order (rx, order, face sequence, tan_err, ray)."""
    keys = [a["ray"], a["tan_err"]] + [a["face"][:, j] for j in range(7, -1, -1)] + \
        [a["order"], a["rx"]]
    return a[np.lexsort(keys)]


def compare_dpaths(g, o):
    assert len(g) == len(o)
    for f in ("rx", "wedge", "launch_ray", "iters_used", "flags"):
        assert np.array_equal(g[f], o[f]), f
    for f in ("tan_err", "axis", "point", "exact_point", "init_tan_err", "length_m",
              "exact_length_m"):
        assert np.array_equal(bits(g[f]), bits(o[f])), f
    for f in ("delay_s", "exact_delay_s"):
        assert np.all(np.abs(g[f] - o[f]) <= DELAY_RTOL * np.abs(o[f])), f
    for f in ("aod", "aoa", "exact_aod", "exact_aoa"):
        if len(g):
            assert angle_deg(g[f], o[f]).max() <= ANGLE_TOL_DEG, f
    assert np.all(np.abs(g["err_angle_deg"] - o["err_angle_deg"]) <= ANGLE_TOL_DEG)


@pytest.mark.parametrize("which", ["box", "two_boxes", "manhattan", "hinge"])
def test_wedges_bitexact(gpu, orc, which):
    if which == "box":
        sc = box_scene(((0, 0, 0), (10, 8, 20)))
    elif which == "two_boxes":
        sc = box_scene(((0, 0, 0), (10, 10, 20)), ((6, -5, 0), (8, -3, 30)))
    elif which == "manhattan":
        sc = scenes.manhattan(0)
    else:
        b = scenes.SceneBuilder()
        b.quad((0, 0, 0), (0, 1, 0), (-1, 1, 0), (-1, 0, 0), 0)
        t = math.radians(30.0)
        b.quad((0, 0, 0), (math.cos(t), 0, math.sin(t)), (math.cos(t), 1, math.sin(t)),
               (0, 1, 0), 0)
        sc = b.scene([4 + 0j])
    s = gpu.scene(sc)
    try:
        w = s.wedges()
    finally:
        s.close()
    o = orc.wedges(sc)
    assert len(w) == len(o["a"]) > 0
    assert np.array_equal(bits(w["a"]), bits(o["a"])) and np.array_equal(bits(w["b"]), bits(o["b"]))
    assert np.array_equal(w["face"], o["faces"])


CASES = [
    # (scene, tx, receivers, params)
    ("box", (-12.0, 6.0, 9.0), [(14.0, -9.0, 11.0), (20.0, -8.0, 4.0), (5.0, 5.0, 5.0),
                                (25.0, 3.0, 12.0), (-3.0, -4.0, 25.0)],
     dict(division_n=40, iterations=10, subrays=6)),
    ("two_boxes", (-12.0, 6.0, 9.0), [(14.0, -9.0, 11.0), (14.0, -2.0, 33.0), (-8.0, -15.0, 2.0)],
     dict(division_n=33, iterations=6, subrays=7, keep_invalid=True)),
    ("box_target", (-12.0, 6.0, 9.0), [(14.0, -9.0, 11.0), (20.0, -8.0, 4.0), (-3.0, -4.0, 25.0)],
     dict(division_n=24, iterations=40, subrays=6, target_err_deg=1e-5)),
]


def _scene(name):
    if name.startswith("two_boxes"):
        return box_scene(((0, 0, 0), (10, 10, 20)), ((6, -5, 0), (8, -3, 30)))
    return box_scene(((0, 0, 0), (10, 10, 20)))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_diffraction_small_scenes(gpu, orc, case):
    name, tx, rx, prm = case
    sc = _scene(name)
    rx = np.array(rx)
    s = gpu.scene(sc)
    try:
        ev = s.diff_candidates(tx, rx, **prm)
        got, st = s.diffract(tx, rx, **prm)
    finally:
        s.close()
    o = orc.diffract(sc, tx, rx, **prm)
    oc = sort_events(o["candidates"])
    assert len(ev) == len(oc) > 0
    assert ev.tobytes() == sort_events(ev).tobytes()
    assert ev.tobytes() == oc.tobytes()
    compare_dpaths(got, o["paths"])
    assert st["n_candidates"] == len(oc) and st["n_unique"] == len(o["unique"])
    assert len(got) > 0


@pytest.mark.parametrize("prm", [dict(iterations=10, subrays=6, keep_invalid=True),
                                 dict(iterations=30, subrays=6, target_err_deg=0.01),
                                 dict(iterations=5, subrays=7)],
                         ids=["i10_keep", "target", "s7"])
def test_diffraction_manhattan_full(gpu, orc, prm):
    """The Manhattan grid at n = 200 (400,002 rays, 768 wedges, 64 Rx): the
    whole event set, path set and every record."""
    cfg = scenes.manhattan_config(0)
    kw = dict(prm, division_n=200)
    s = gpu.scene(cfg["scene"])
    try:
        ev = s.diff_candidates(cfg["tx"], cfg["rx"], **kw)
        got, _ = s.diffract(cfg["tx"], cfg["rx"], **kw)
    finally:
        s.close()
    o = orc.diffract(cfg["scene"], cfg["tx"], cfg["rx"], **kw)
    oc = sort_events(o["candidates"])
    assert len(ev) == len(oc) > 1000
    assert ev.tobytes() == sort_events(ev).tobytes()
    assert ev.tobytes() == oc.tobytes()
    compare_dpaths(got, o["paths"])
    assert len(got) > 100


def test_diffraction_edge_cases(gpu, orc):
    """No receivers; a room seen from inside (its edges are concave from the
    receivers' side: no diffraction); a ground plane alone (no wedge); a
    receiver inside a building; a too-small output buffer."""
    from paper_2208_10009_amd import sbr
    prm = dict(division_n=30, iterations=3, subrays=6)
    cfg = scenes.shoebox_config(0)
    s = gpu.scene(cfg["scene"])
    try:
        assert len(s.wedges()) == 12
        got, st = s.diffract(cfg["tx"], cfg["rx"], **prm)
        assert len(got) == 0 and st["n_candidates"] == 0
        got, _ = s.diffract(cfg["tx"], np.zeros((0, 3)), **prm)
        assert len(got) == 0
    finally:
        s.close()
    s = gpu.scene(scenes.two_ray())
    try:
        assert len(s.wedges()) == 0
        got, st = s.diffract([0, 0, 10], [[50, 0, 2]], **prm)
        assert len(got) == 0 and st["n_candidates"] == 0
    finally:
        s.close()
    sc = box_scene(((0, 0, 0), (10, 10, 20)))
    s = gpu.scene(sc)
    try:
        assert len(s.diff_candidates([-12, 6, 9], [[5, 5, 5]], **prm)) == 0
        full, _ = s.diffract([-12, 6, 9], [[14, -9, 11], [20, -8, 4]], **prm)
        assert len(full) >= 2
        with pytest.raises(sbr.SbrError) as e:
            s.diffract([-12, 6, 9], [[14, -9, 11], [20, -8, 4]], capacity=1, **prm)
        assert e.value.status == sbr.E_CAPACITY
    finally:
        s.close()


def _hinge_long(normals_deg, L=4.0):
    t = math.radians(normals_deg)
    b = scenes.SceneBuilder()
    b.quad((0, 0, 0), (0, L, 0), (-L, L, 0), (-L, 0, 0), 0)
    c, s_ = math.cos(t), math.sin(t)
    b.quad((0, 0, 0), (L * c, 0, L * s_), (L * c, L, L * s_), (0, L, 0), 0)
    return b.scene([4 + 0j])


@pytest.mark.parametrize("normals_deg", [60.0, 120.0])
def test_diffraction_hinge_solid_side(gpu, orc, normals_deg):
    """An obtuse and an acute hinge (the wedge's solid side is not the set of
    points in front of both faces): receivers all around the edge, events and
    paths equal to the oracle's."""
    sc = _hinge_long(normals_deg)
    tx = (1.0, 2.0, -3.0)
    ang = np.radians(np.arange(5.0, 360.0, 10.0))
    rx = np.stack([6 * np.cos(ang), np.full(len(ang), 2.2), 6 * np.sin(ang)], axis=1)
    prm = dict(division_n=24, iterations=6, subrays=6, keep_invalid=True)
    s = gpu.scene(sc)
    try:
        ev = s.diff_candidates(tx, rx, **prm)
        got, _ = s.diffract(tx, rx, **prm)
    finally:
        s.close()
    o = orc.diffract(sc, tx, rx, **prm)
    oc = sort_events(o["candidates"])
    assert len(ev) == len(oc) > 0
    assert ev.tobytes() == oc.tobytes()
    compare_dpaths(got, o["paths"])
    # receivers strictly inside the solid sector get nothing
    inside = (np.degrees(ang) > normals_deg) & (np.degrees(ang) < 180.0)
    assert not np.isin(np.nonzero(inside)[0], ev["rx"]).any()


def test_diffraction_blocked_before_the_edge(gpu, orc):
    b = scenes.SceneBuilder()
    b.box((0, 0, 0), (10, 10, 20), 0)
    b.quad((-6, 0, 0), (-6, 12, 0), (-6, 12, 25), (-6, 0, 25), 0)
    sc = b.scene([5.3 - 0.4j])
    tx, rx = (-12.0, 6.0, 9.0), np.array([[14.0, -9.0, 11.0], [20.0, -8.0, 4.0]])
    prm = dict(division_n=40, iterations=4, subrays=6, keep_invalid=True)
    s = gpu.scene(sc)
    try:
        ev = s.diff_candidates(tx, rx, **prm)
        got, _ = s.diffract(tx, rx, **prm)
    finally:
        s.close()
    o = orc.diffract(sc, tx, rx, **prm)
    assert ev.tobytes() == sort_events(o["candidates"]).tobytes()
    compare_dpaths(got, o["paths"])
