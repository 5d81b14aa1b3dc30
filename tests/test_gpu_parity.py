"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.

Bars:
  * launch directions, per-ray triangle sequences and segment parameters,
    reception events, path sets, face sequences, winning launch rays,
    iteration counts and flags: bit-exact (the HIP path evaluates every
    decision in FP64 with the oracle's operation order);
  * refined and exact delay: relative error <= 1e-6; AOD/AOA: <= 1e-4 deg;
    power: <= 1e-3 dB (transcendentals on the GPU are not correctly rounded).
"""
import math

import numpy as np
import pytest

from paper_2208_10009_amd import scenes

pytestmark = pytest.mark.gpu

from parity_util import (ANGLE_TOL_DEG, DELAY_RTOL, POWER_TOL_DB, angle_deg, bits,  # noqa: F401
                         compare_paths as _compare_paths, key_of)


# ----------------------------------------------------------- launch grid --
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 20, 21, 200])
def test_launch_grid_bitexact(gpu, orc, n):
    g = gpu.launch_grid(n)
    o = orc.launch_dirs(n)
    assert g.shape == (10 * n * n + 2, 3)
    assert np.array_equal(bits(g), bits(o))


def test_launch_grid_large_n_sampled(gpu, orc):
    n = 1000
    rng = np.random.default_rng(7)
    N = 10 * n * n + 2
    ids = np.unique(np.concatenate([np.arange(64), N - 64 + np.arange(64),
                                    rng.integers(0, N, 4000)]))
    o = orc.launch_dirs(n, ids)
    for first in (0, N - 64):
        g = gpu.launch_grid(n, first, 64)
        assert np.array_equal(bits(g), bits(o[np.searchsorted(ids, first + np.arange(64))]))
    g = gpu.launch_grid(n)
    assert np.array_equal(bits(g[ids]), bits(o))


@pytest.mark.parametrize("check_log2", [200, 0])
def test_launch_grid_full_series_pass(gpu, orc, check_log2):
    """The grid setup accepts short-series values only when their error bound
    proves the rounding; with the bounds scaled by 2^200 every layer takes the
    full-series pass instead.  Both give the correctly rounded grid."""
    from paper_2208_10009_amd import sbr
    base = gpu.tuning()
    try:
        gpu.set_tuning(**dict(base, grid_check_log2=check_log2))
        assert gpu.tuning()["grid_check_log2"] == check_log2
        for n in (4, 7, 21, 200):
            assert np.array_equal(bits(gpu.launch_grid(n)), bits(orc.launch_dirs(n))), n
        n = 1000
        N = 10 * n * n + 2
        ids = np.unique(np.random.default_rng(8).integers(0, N, 3000))
        assert np.array_equal(bits(gpu.launch_grid(n)[ids]), bits(orc.launch_dirs(n, ids)))
        with pytest.raises(sbr.SbrError):
            gpu.set_tuning(grid_check_log2=201)
    finally:
        gpu.set_tuning(**base)


# ------------------------------------------------------- per-ray tracing --
def _compare_rays(gpu, orc, cfg, n, K, first=0, count=None):
    sc = gpu.scene(cfg["scene"])
    try:
        gt, gT = sc.trace_rays(cfg["tx"], n, K, first, count)
    finally:
        sc.close()
    N = 10 * n * n + 2
    ids = np.arange(first, first + (N - first if count is None else count))
    ot, _, oT = orc.trace_rays(cfg["scene"], cfg["tx"], n, K, ids=ids)
    assert np.array_equal(gt, ot)
    assert np.array_equal(bits(gT), bits(oT))
    return gt


@pytest.mark.parametrize("seed", [0, 1])
def test_trace_rays_shoebox_all(gpu, orc, seed):
    cfg = scenes.shoebox_config(seed)
    gt = _compare_rays(gpu, orc, cfg, 20, 3)
    assert (gt[:, 3] >= 0).all()  # closed room: every segment ends on a wall


def test_trace_rays_manhattan_all(gpu, orc):
    cfg = scenes.manhattan_config(0)
    gt = _compare_rays(gpu, orc, cfg, 60, 6)
    assert (gt[:, 0] >= 0).any() and (gt[:, 0] < 0).any()


def test_trace_rays_manhattan_full_size_chunks(gpu, orc):
    cfg = scenes.manhattan_config(0)
    n = 200
    N = 10 * n * n + 2
    for first in (0, 123457, N - 3001):
        _compare_rays(gpu, orc, cfg, n, 6, first, 3001)


def test_trace_rays_ragged_and_empty(gpu, orc):
    cfg = scenes.shoebox_config(0)
    sc = gpu.scene(cfg["scene"])
    try:
        t, T = sc.trace_rays(cfg["tx"], 20, 3, 4001, 1)
        assert t.shape == (1, 4)
        t0, _ = sc.trace_rays(cfg["tx"], 20, 3, 17, 0)
        assert t0.shape == (0, 4)
    finally:
        sc.close()
    ot, _, oT = orc.trace_rays(cfg["scene"], cfg["tx"], 20, 3, ids=[4001])
    assert np.array_equal(t, ot) and np.array_equal(bits(T), bits(oT))


def test_empty_scene_traces_nothing(gpu):
    empty = {"xyz": np.zeros((0, 3)), "tri": np.zeros((0, 3), np.int32),
             "face_id": np.zeros(0, np.int32), "mat_id": np.zeros(0, np.int32),
             "eps_r": np.array([5.0 + 0j])}
    sc = gpu.scene(empty)
    try:
        t, T = sc.trace_rays([0, 0, 0], 3, 2)
        assert (t == -1).all() and np.isinf(T).all()
        p, st = sc.trace([0, 0, 0], [[1.0, 2.0, 3.0]], max_order=2, division_n=3, iterations=2)
        # free space: only the line of sight
        assert len(p) == 1 and p[0]["order"] == 0
    finally:
        sc.close()


# ------------------------------------------------------- reception events --
def _sorted_oracle_cands(c):
    order = np.lexsort((c["ray"], c["tan_err"], *[c["face"][:, j] for j in range(7, -1, -1)],
                        c["order"], c["rx"]))
    return c[order]


def _compare_candidates(gpu, orc, cfg, **prm):
    sc = gpu.scene(cfg["scene"])
    try:
        g = sc.candidates(cfg["tx"], cfg["rx"], **prm)
    finally:
        sc.close()
    o = _sorted_oracle_cands(orc.run(cfg["scene"], cfg["tx"], cfg["rx"], **prm)["candidates"])
    assert len(g) == len(o)
    for f in ("rx", "order", "face", "ray"):
        assert np.array_equal(g[f], o[f]), f
    assert np.array_equal(bits(g["tan_err"]), bits(o["tan_err"]))
    return g


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_candidates_shoebox(gpu, orc, seed):
    cfg = scenes.shoebox_config(seed)
    g = _compare_candidates(gpu, orc, cfg, **cfg["params"])
    assert len(g) > 20


def test_candidates_manhattan_full(gpu, orc):
    cfg = scenes.manhattan_config(0)
    g = _compare_candidates(gpu, orc, cfg, **cfg["params"])
    assert len(g) > 50


@pytest.mark.parametrize("tree", [False, True])
def test_candidates_receivers_everywhere(gpu, orc, tree):
    """Receivers spread through the whole volume (at ground level, between
    and above the buildings, above the transmitter), tested one by one and
    through the receiver tree: a wave skips its receivers only where no
    receiver can be captured, so the events equal the oracle's bit for bit."""
    rng = np.random.default_rng(21)
    cfg = scenes.manhattan_config(2)
    rx = np.column_stack([rng.uniform(-20.0, 340.0, 48), rng.uniform(-20.0, 340.0, 48),
                          np.concatenate([rng.uniform(0.0, 2.0, 16), rng.uniform(2.0, 70.0, 24),
                                          rng.uniform(70.0, 200.0, 8)])])
    cfg = dict(cfg, rx=rx)
    prm = dict(cfg["params"], division_n=80, max_order=4)
    base = gpu.tuning()
    try:
        gpu.set_tuning(**dict(base, rx_tree_min=1 if tree else 1 << 30))
        g = _compare_candidates(gpu, orc, cfg, **prm)
    finally:
        gpu.set_tuning(**base)
    assert len(g) > 50 and len(np.unique(g["rx"])) > 20


# ------------------------------------------------------------ full paths --
def _run_both(gpu, orc, cfg, **prm):
    sc = gpu.scene(cfg["scene"])
    try:
        g, st = sc.trace(cfg["tx"], cfg["rx"], **prm)
    finally:
        sc.close()
    o = orc.run(cfg["scene"], cfg["tx"], cfg["rx"], **prm)["paths"]
    return g, o, st


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_paths_shoebox(gpu, orc, seed):
    cfg = scenes.shoebox_config(seed)
    g, o, st = _run_both(gpu, orc, cfg, **cfg["params"])
    _compare_paths(g, o)
    assert st["n_rays"] == 4002 and st["n_paths"] == len(g) > 20


@pytest.mark.parametrize("S", [6, 7])
def test_paths_shoebox_target_and_invalid(gpu, orc, S):
    cfg = scenes.shoebox_config(5)
    prm = dict(max_order=3, division_n=21, iterations=30, subrays=S, target_err_deg=0.01,
               keep_invalid=True)
    g, o, _ = _run_both(gpu, orc, cfg, **prm)
    _compare_paths(g, o)
    assert (g["flags"] & 2).any()  # some paths fail path test 2 and are kept
    assert (g["flags"] & 4).any()  # the target stop is taken


@pytest.mark.parametrize("K,iters", [(0, 3), (0, 0), (8, 3), (8, 0)])
def test_paths_order_extremes(gpu, orc, K, iters):
    """No reflections (direct paths only) and the most the records hold
    (SBR_MAX_ORDER = 8), with and without refinement, in the closed shoebox
    and the Manhattan scene: every record field against the oracle."""
    for cfg, n in ((scenes.shoebox_config(4), 20), (scenes.manhattan_config(3, n_rx=8), 30)):
        prm = dict(cfg["params"], max_order=K, division_n=n, iterations=iters)
        g, o, st = _run_both(gpu, orc, cfg, **prm)
        _compare_paths(g, o)
        assert len(g) > 0 and (g["order"] <= K).all()
        if K == 0:
            assert (g["order"] == 0).all()
        assert st["n_rays"] == 10 * n * n + 2


def test_paths_coplanar_split_ground(gpu, orc):
    """Two coplanar ground faces meeting at x = 0: the paths of the face
    that does not hold the specular point (kept invalid) refine toward the
    shared edge only; every record equals the oracle's."""
    b = scenes.SceneBuilder()
    b.quad((-20, -20, 0), (0, -20, 0), (0, 20, 0), (-20, 20, 0), 0)
    b.quad((0, -20, 0), (20, -20, 0), (20, 20, 0), (0, 20, 0), 0)
    cfg = {"scene": b.scene([5.0 + 0j]), "tx": np.array([-0.3, 0.0, 3.0]),
           "rx": np.array([[1.0, 0.2, 3.0], [0.5, -0.4, 2.0], [-2.0, 1.0, 1.0]])}
    for n in (2, 3, 4, 6):
        prm = dict(max_order=1, division_n=n, iterations=8, subrays=6, keep_invalid=True)
        g, o, _ = _run_both(gpu, orc, cfg, **prm)
        _compare_paths(g, o)
        assert len(g) > 0


def test_degenerate_receivers(gpu, orc):
    """Receivers at the transmitter, 1e-9 m from it, on a wall, in a room
    corner, and a repeated receiver: the same records as the oracle, and the
    repeated receiver gets the same paths as its twin."""
    cfg = scenes.shoebox_config(1)
    tx = cfg["tx"]
    rx = np.array([tx, tx + np.array([1e-9, 0.0, 0.0]), [0.0, 4.0, 1.5], [10.0, 8.0, 3.0],
                   [6.5, 2.25, 0.75], [6.5, 2.25, 0.75], [5.0, 4.0, 0.0]])
    cfg = dict(cfg, rx=rx)
    prm = dict(cfg["params"], max_order=3, division_n=30, iterations=3)
    g, o, _ = _run_both(gpu, orc, cfg, **prm)
    _compare_paths(g, o)
    a, b = g[g["rx"] == 4], g[g["rx"] == 5]
    assert len(a) > 0 and len(a) == len(b)
    for f in a.dtype.names:
        if f != "rx":
            assert a[f].tobytes() == b[f].tobytes(), f


def test_paths_traditional_sbr(gpu, orc):
    cfg = scenes.shoebox_config(2)
    prm = dict(cfg["params"], iterations=0)
    g, o, _ = _run_both(gpu, orc, cfg, **prm)
    _compare_paths(g, o)
    assert (g["iters_used"] == 0).all()


def test_paths_manhattan_full_config(gpu, orc):
    """The benchmark workload at full size: 770 triangles, 64 Rx, n = 200
    (400,002 rays), 6 reflections, 5 iterations of 7 sub-rays."""
    cfg = scenes.manhattan_config(0)
    g, o, st = _run_both(gpu, orc, cfg, **cfg["params"])
    _compare_paths(g, o)
    assert st["n_rays"] == 400002


def test_paths_manhattan_other_seed_small(gpu, orc):
    cfg = scenes.manhattan_config(4, n_rx=16)
    prm = dict(cfg["params"], division_n=67, max_order=5)
    g, o, _ = _run_both(gpu, orc, cfg, **prm)
    _compare_paths(g, o)


def test_no_receivers(gpu):
    cfg = scenes.shoebox_config(0)
    sc = gpu.scene(cfg["scene"])
    try:
        p, st = sc.trace(cfg["tx"], np.zeros((0, 3)), **cfg["params"])
    finally:
        sc.close()
    assert len(p) == 0 and st["n_candidates"] == 0


def test_capacity_two_call_sizing(gpu):
    from paper_2208_10009_amd import sbr
    cfg = scenes.shoebox_config(0)
    sc = gpu.scene(cfg["scene"])
    try:
        with pytest.raises(sbr.SbrError) as e:
            sc.trace(cfg["tx"], cfg["rx"], capacity=3, **cfg["params"])
        assert e.value.status == sbr.E_CAPACITY
        p, _ = sc.trace(cfg["tx"], cfg["rx"], **cfg["params"])
        assert len(p) > 3
    finally:
        sc.close()


def test_invalid_arguments(gpu):
    from paper_2208_10009_amd import sbr
    cfg = scenes.shoebox_config(0)
    sc = gpu.scene(cfg["scene"])
    try:
        for bad in (dict(max_order=9), dict(division_n=0), dict(subrays=5),
                    dict(iterations=-1), dict(freq_hz=0.0)):
            prm = dict(cfg["params"], **bad)
            with pytest.raises(sbr.SbrError) as e:
                sc.trace(cfg["tx"], cfg["rx"], **prm)
            assert e.value.status == sbr.E_INVALID_ARG
        with pytest.raises(sbr.SbrError):
            sc.trace([math.nan, 0, 0], cfg["rx"], **cfg["params"])
    finally:
        sc.close()
    bad_scene = dict(cfg["scene"])
    bad_scene["mat_id"] = np.full(12, 3, np.int32)
    with pytest.raises(sbr.SbrError):
        gpu.scene(bad_scene)
    # a face whose second triangle leaves the first one's plane
    off = scenes.SceneBuilder()
    off.add(np.array([[0, 0, 0], [4, 0, 0], [4, 4, 0], [0, 4, 0.01]], float),
            [(0, 1, 2), (0, 2, 3)], [0, 0], 0)
    with pytest.raises(sbr.SbrError, match="not in the plane") as e:
        gpu.scene(off.scene([5.0 + 0j]))
    assert e.value.status == sbr.E_INVALID_ARG
    # the same quad within the tolerance is accepted
    flat = scenes.SceneBuilder()
    flat.add(np.array([[0, 0, 0], [4, 0, 0], [4, 4, 0], [0, 4, 1e-12]], float),
             [(0, 1, 2), (0, 2, 3)], [0, 0], 0)
    gpu.scene(flat.scene([5.0 + 0j])).close()
    # a face whose lowest-index triangle is degenerate (no plane); a later
    # degenerate triangle of a face is accepted
    deg = scenes.SceneBuilder()
    deg.add(np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 4, 0]], float),
            [(0, 1, 2), (0, 1, 3)], [0, 0], 0)
    with pytest.raises(sbr.SbrError, match="degenerate") as e:
        gpu.scene(deg.scene([5.0 + 0j]))
    assert e.value.status == sbr.E_INVALID_ARG
    ok = scenes.SceneBuilder()
    ok.add(np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 4, 0]], float),
           [(0, 1, 3), (0, 1, 2)], [0, 0], 0)
    gpu.scene(ok.scene([5.0 + 0j])).close()


def test_deterministic_reruns(gpu):
    cfg = scenes.manhattan_config(1)
    sc = gpu.scene(cfg["scene"])
    try:
        a, _ = sc.trace(cfg["tx"], cfg["rx"], **cfg["params"])
        b, _ = sc.trace(cfg["tx"], cfg["rx"], fresh_grid=True, **cfg["params"])
    finally:
        sc.close()
    assert a.tobytes() == b.tobytes()


def _context_with_env(env):
    """A library context created with the environment overrides `env` (the
    context reads its SBR_* settings when it is created)."""
    import os
    from paper_2208_10009_amd import sbr
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return sbr.Context(0)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("n", [3, 4, 5, 6, 7, 20, 200])
def test_streamed_grid(orc, n):
    """A fresh equiangular grid whose ray orders exist is streamed (here
    whenever possible): its ring setup runs on a second stream beside the
    trace, which forms each packet's directions itself once the setup has
    published the layers they need.  The directions it leaves are the
    oracle's bit for bit (n = 3..7 cover the innermost layer cases), and the
    paths equal those of the first call, whose grid was formed before its
    trace, through both entry points."""
    import torch
    ctx = _context_with_env({"SBR_GRID_STREAM": "2"})
    cfg = scenes.manhattan_config(1, n_rx=16)
    prm = dict(cfg["params"], division_n=n)
    sc = ctx.scene(cfg["scene"])
    try:
        a, sa = sc.trace(cfg["tx"], cfg["rx"], fresh_grid=True, **prm)
        b, sb = sc.trace(cfg["tx"], cfg["rx"], fresh_grid=True, **prm)
        rx = torch.as_tensor(cfg["rx"], device="cuda")
        c, sc_ = sc.trace_device(cfg["tx"], rx, fresh_grid=True, **prm)
        d = ctx.launch_grid(n)
    finally:
        sc.close()
        ctx.close()
    # the first call formed the grid (and the orders); the others streamed it
    assert sa["ms_launch"] > 0 and sb["ms_launch"] == 0 and sc_["ms_launch"] == 0
    assert a.tobytes() == b.tobytes() == c.cpu().numpy().tobytes()
    assert np.array_equal(bits(d), bits(orc.launch_dirs(n)))


@pytest.mark.parametrize("device_api", [False, True])
def test_streamed_grid_fallback(orc, device_api):
    """A streamed grid whose setup does not publish in time (forced from the
    host: the trace and the start wait expect an epoch the setup never
    writes, and give up after a few polls) switches streaming off for the
    context; the call runs again with its grid formed first and returns the
    same paths."""
    import torch
    ctx = _context_with_env({"SBR_GRID_STREAM": "2", "SBR_GRID_STREAM_MISS": "1"})
    cfg = scenes.manhattan_config(1, n_rx=16)
    prm = dict(cfg["params"], division_n=20)
    sc = ctx.scene(cfg["scene"])
    rx = torch.as_tensor(cfg["rx"], device="cuda")
    try:
        runs = []
        for _ in range(3):
            if device_api:
                p, st = sc.trace_device(cfg["tx"], rx, fresh_grid=True, **prm)
                runs.append((p.cpu().numpy().tobytes(), st))
            else:
                p, st = sc.trace(cfg["tx"], cfg["rx"], fresh_grid=True, **prm)
                runs.append((p.tobytes(), st))
        d = ctx.launch_grid(20)
    finally:
        sc.close()
        ctx.close()
    assert all(b == runs[0][0] for b, _ in runs)
    # every call formed its grid before its trace: the first by rule, the
    # second on its retry, the third with streaming switched off
    assert all(st["ms_launch"] > 0 for _, st in runs)
    assert np.array_equal(bits(d), bits(orc.launch_dirs(20)))


def test_streamed_grid_automatic_choice(gpu):
    """By default a grid is streamed only once a fresh call of it has shown
    a trace at least three times as long as its grid: never for a 12-triangle
    room at n = 60 (the trace is short), the same paths either way."""
    cfg = scenes.shoebox_config(2)
    prm = dict(cfg["params"], division_n=60)
    sc = gpu.scene(cfg["scene"])
    try:
        runs = [sc.trace(cfg["tx"], cfg["rx"], fresh_grid=True, **prm) for _ in range(4)]
    finally:
        sc.close()
    assert all(st["ms_launch"] > 0 for _, st in runs)
    assert all(p.tobytes() == runs[0][0].tobytes() for p, _ in runs)


def _trace_with_env(env, cfg, **prm):
    import os
    from paper_2208_10009_amd import sbr
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        ctx = sbr.Context(0)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    try:
        sc = ctx.scene(cfg["scene"])
        p, _ = sc.trace(cfg["tx"], cfg["rx"], **prm)
        sc.close()
    finally:
        ctx.close()
    return p


@pytest.mark.parametrize("prm", [dict(iterations=5, subrays=7), dict(iterations=4, subrays=6),
                                 dict(iterations=9, subrays=7, target_err_deg=0.01),
                                 dict(iterations=7, subrays=6, target_err_deg=0.003),
                                 dict(iterations=1, subrays=7), dict(iterations=2, subrays=6),
                                 dict(iterations=0, subrays=7),
                                 dict(iterations=0, subrays=6, target_err_deg=0.5),
                                 dict(iterations=20, subrays=7, target_err_deg=0.0002),
                                 dict(iterations=13, subrays=6)])
def test_refine_lookahead_matches_single_step(gpu, orc, prm):
    """The three-iteration (512 lanes per path) and two-iteration (64 lanes)
    lookahead kernels, the one-iteration kernel (8 lanes per path), the
    segment-parallel kernels (a lane per sub-ray segment: a wave per path, a
    512-lane workgroup per path, and the hand-over from the first to the
    second) and the persistent work-queue refinement (depth 0) give
    byte-identical paths, and all match the oracle."""
    cfg = scenes.manhattan_config(2, n_rx=24)
    full = dict(cfg["params"], division_n=80, **prm)
    a = _trace_with_env({"SBR_LOOKAHEAD_PATHS": "0", "SBR_LOOKAHEAD_DEPTH": "1"}, cfg, **full)
    b = _trace_with_env({"SBR_LOOKAHEAD_PATHS": "100000", "SBR_LOOKAHEAD_DEPTH": "2",
                         "SBR_REFINE_SEGMENTS": "0"}, cfg, **full)
    c = _trace_with_env({"SBR_LOOKAHEAD_PATHS": "100000", "SBR_LOOKAHEAD_DEPTH": "3",
                         "SBR_LOOKAHEAD3_PATHS": "100000", "SBR_REFINE_SEGMENTS": "0"}, cfg,
                        **full)
    q = _trace_with_env({"SBR_LOOKAHEAD_DEPTH": "0"}, cfg, **full)
    assert a.tobytes() == b.tobytes() == c.tobytes() == q.tobytes()
    # segments in parallel lanes: one wave per path only; 512 lanes per path
    # (two iterations per step) from the start; one wave per path handing the
    # paths still running to 512-lane workgroups after 1 and after 2
    # iterations (odd and even splits)
    for env in ({"SBR_LOOKAHEAD3_PATHS": "0", "SBR_SEG_TAIL": "0"},
                {"SBR_LOOKAHEAD3_PATHS": "100000"},
                {"SBR_LOOKAHEAD3_PATHS": "0", "SBR_SEG_TAIL": "1"},
                {"SBR_LOOKAHEAD3_PATHS": "0", "SBR_SEG_TAIL": "2"}):
        g = _trace_with_env(dict(env, SBR_LOOKAHEAD_PATHS="100000", SBR_REFINE_SEGMENTS="1"), cfg,
                            **full)
        assert g.tobytes() == a.tobytes(), env
    o = orc.run(cfg["scene"], cfg["tx"], cfg["rx"], **full)["paths"]
    _compare_paths(a, o)


@pytest.mark.parametrize("seed,order", [(2, 6), (5, 3)])
def test_refine_three_level_lds_matches_global(gpu, orc, seed, order):
    """The three-level refinement with the scene staged in LDS and reading
    global memory give byte-identical paths, equal to the oracle's."""
    cfg = scenes.manhattan_config(seed, n_rx=20)
    full = dict(cfg["params"], division_n=70, max_order=order, iterations=7)
    env = {"SBR_LOOKAHEAD_PATHS": "100000", "SBR_LOOKAHEAD_DEPTH": "3",
           "SBR_LOOKAHEAD3_PATHS": "100000", "SBR_REFINE_SEGMENTS": "0"}
    a = _trace_with_env(dict(env, SBR_LA3_LDS="1"), cfg, **full)
    b = _trace_with_env(dict(env, SBR_LA3_LDS="0"), cfg, **full)
    assert a.tobytes() == b.tobytes() and len(a) > 20
    _compare_paths(a, orc.run(cfg["scene"], cfg["tx"], cfg["rx"], **full)["paths"])


def test_bvh_options_do_not_change_paths(gpu, orc):
    """The hierarchy (leaf size, SAH bins, split references with clipped
    boxes) only decides which nodes a ray visits: paths and per-ray traces are
    byte-identical across builds, and match the oracle."""
    cfg = scenes.manhattan_config(4, n_rx=24)
    prm = dict(cfg["params"], division_n=90)
    ref_p = ref_t = None
    for opt in (dict(), dict(max_leaf_size=1, sah_bins=16), dict(sah_bins=32, split_pct=100),
                dict(max_leaf_size=8, split_pct=400), dict(split_pct=50),
                dict(max_leaf_size=3, sah_bins=48)):
        sc = gpu.scene(cfg["scene"], **opt)
        try:
            p, _ = sc.trace(cfg["tx"], cfg["rx"], **prm)
            tri, t = sc.trace_rays(cfg["tx"], prm["division_n"], prm["max_order"], 0, 20000)
        finally:
            sc.close()
        if ref_p is None:
            ref_p, ref_t = p, (tri, t)
            _compare_paths(p, orc.run(cfg["scene"], cfg["tx"], cfg["rx"], **prm)["paths"])
        else:
            assert p.tobytes() == ref_p.tobytes(), opt
            assert np.array_equal(tri, ref_t[0]) and np.array_equal(t, ref_t[1]), opt


def test_trace_counters_are_consistent(gpu):
    """The instrumented trace kernel's counts: a wave pass serves 1 to 64
    lanes, every segment traces at least the root node, and the counts do not
    depend on the launch tuning that leaves packets whole."""
    cfg = scenes.manhattan_config(1, n_rx=32)
    prm = dict(cfg["params"], division_n=120)
    sc = gpu.scene(cfg["scene"])
    try:
        c = sc.trace_counters(cfg["tx"], cfg["rx"], **prm)
        base = gpu.tuning()
        gpu.set_tuning(**dict(base, persist_blocks=37))
        c2 = sc.trace_counters(cfg["tx"], cfg["rx"], **prm)
        gpu.set_tuning(**base)
    finally:
        sc.close()
    n_rays = 10 * prm["division_n"] ** 2 + 2
    assert n_rays <= c["segments"] <= n_rays * (prm["max_order"] + 1)
    assert c["nodes"] >= c["segments"]
    for lanes, steps in (("nodes", "wave_node_steps"), ("tris", "wave_tri_steps"),
                         ("segments", "wave_seg_steps")):
        assert c[steps] <= c[lanes] <= 64 * c[steps], (lanes, c)
    assert c["tris_run"] <= c["tris"] and c["wave_rx_steps"] > 0
    rx_lanes = c["rx_nodes"] + c["rx_tests"]
    assert c["wave_rx_steps"] <= rx_lanes <= 64 * c["wave_rx_steps"], c
    assert c["rx_nodes"] == 0 and c["rx_tests"] > 0  # 32 receivers: tested one by one
    for k in ("segments", "nodes", "tris", "events", "tris_run", "rx_nodes", "rx_tests"):
        assert c2[k] == c[k], k


def test_trace_counters_receiver_tree(gpu):
    """Through the receiver box tree: boxes and receivers tested, each wave
    pass of the receiver walk serving 1 to 64 lanes, and the same events as
    testing every receiver."""
    cfg = scenes.manhattan_config(2, n_rx=256)
    prm = dict(cfg["params"], division_n=100)
    sc = gpu.scene(cfg["scene"])
    base = gpu.tuning()
    try:
        gpu.set_tuning(**dict(base, rx_tree_min=16))
        t = sc.trace_counters(cfg["tx"], cfg["rx"], **prm)
        gpu.set_tuning(**dict(base, rx_tree_min=1 << 30))
        lin = sc.trace_counters(cfg["tx"], cfg["rx"], **prm)
    finally:
        gpu.set_tuning(**base)
        sc.close()
    assert t["rx_nodes"] > 0 and 0 < t["rx_tests"] < lin["rx_tests"]
    assert t["wave_rx_steps"] <= t["rx_nodes"] + t["rx_tests"] <= 64 * t["wave_rx_steps"]
    assert t["events"] == lin["events"] and t["segments"] == lin["segments"]


def test_receiver_tree_kept_across_calls(gpu):
    """The context keeps the last single-job call's receiver tree for the next
    call over the same receivers: calls that alternate between two receiver
    sets of the same size, a two-job batch over a third (which replaces the
    tree on the device), and host-array calls all give the bytes of testing
    every receiver."""
    import torch
    from paper_2208_10009_amd import sbr
    cfg = scenes.manhattan_config(5, n_rx=128)
    prm = dict(cfg["params"], division_n=60)
    rng = np.random.default_rng(3)
    rx_a = np.asarray(cfg["rx"], np.float64)
    rx_b = rx_a + rng.uniform(-3.0, 3.0, size=rx_a.shape) * np.array([1.0, 1.0, 0.0])
    base = gpu.tuning()
    sc = gpu.scene(cfg["scene"])
    try:
        gpu.set_tuning(**dict(base, rx_tree_min=1 << 30))
        ref = {k: sc.trace(cfg["tx"], r, **prm)[0].tobytes() for k, r in (("a", rx_a), ("b", rx_b))}
        gpu.set_tuning(**dict(base, rx_tree_min=16))
        jobs = [dict(prm, scene=0, tx=cfg["tx"], rx_first=0, n_rx=64),
                dict(prm, scene=0, tx=cfg["tx"], rx_first=64, n_rx=64)]
        for k, use in (("a", "dev"), ("a", "dev"), ("b", "dev"), ("a", "dev"), ("a", "batch"),
                       ("a", "dev"), ("b", "host"), ("b", "dev"), ("a", "host")):
            r = rx_a if k == "a" else rx_b
            if use == "batch":
                gpu.trace_batch([sc], jobs, rx_b)
                continue
            if use == "dev":
                got, _ = sc.trace_device(cfg["tx"], torch.as_tensor(r, device="cuda"), **prm)
                got = got.cpu().numpy().reshape(-1).view(sbr.PATH_DTYPE)
            else:
                got, _ = sc.trace(cfg["tx"], r, **prm)
            assert got.tobytes() == ref[k], (k, use)
    finally:
        gpu.set_tuning(**base)
        sc.close()


def test_lds_staged_traversal_matches(gpu, orc):
    """LDS-staged traversal (node prefix, triangles and stack in LDS, or the
    stack alone) gives the same paths as global-memory traversal."""
    cfg = scenes.manhattan_config(3, n_rx=16)
    prm = dict(cfg["params"], division_n=80)
    a = _trace_with_env({"SBR_LDS_BUDGET": "0"}, cfg, **prm)
    b = _trace_with_env({"SBR_LDS_BUDGET": "65536", "SBR_STACK_DEPTH": "4"}, cfg, **prm)
    c = _trace_with_env({"SBR_LDS_BUDGET": "163840", "SBR_TRACE_BLOCK": "128"}, cfg, **prm)
    d = _trace_with_env({"SBR_LDS_BUDGET": "24576", "SBR_STACK_DEPTH": "24"}, cfg, **prm)
    assert a.tobytes() == b.tobytes() == c.tobytes() == d.tobytes()
    _compare_paths(a, orc.run(cfg["scene"], cfg["tx"], cfg["rx"], **prm)["paths"])


def test_many_events_multikernel_path(gpu, orc):
    """More than 4096 reception events: path test 1 and the final compaction
    take the multi-kernel sort/scan route; results still match the oracle."""
    cfg = scenes.shoebox_config(7)
    rng = np.random.default_rng(11)
    rx = rng.uniform(0.2, 0.8, size=(160, 3)) * np.array([10.0, 8.0, 3.0])
    prm = dict(cfg["params"], iterations=2)
    sc = gpu.scene(cfg["scene"])
    try:
        g, st = sc.trace(cfg["tx"], rx, **prm)
        cands = sc.candidates(cfg["tx"], rx, **prm)
    finally:
        sc.close()
    assert st["n_candidates"] > 4096
    r = orc.run(cfg["scene"], cfg["tx"], rx, **prm)
    _compare_paths(g, r["paths"])
    o = _sorted_oracle_cands(r["candidates"])
    assert len(cands) == len(o) and np.array_equal(cands["ray"], o["ray"])


# ---------------------------------------------------------------- batched --
def _small_batch(seed=3):
    return scenes.batch_config(seed, n_scenes=4, n_pairs=10, tri_min=100, tri_max=2000,
                               n_range=(15, 45), order_range=(1, 5), iterations=4)


def _individual(gpu, b):
    """Each job traced alone with sbr_trace, receivers renumbered to the
    batch's array."""
    scs = [gpu.scene(s) for s in b["scenes"]]
    parts = []
    try:
        for j in b["jobs"]:
            prm = {k: v for k, v in j.items() if k not in ("scene", "tx", "rx_first", "n_rx")}
            rx = b["rx"][j["rx_first"]:j["rx_first"] + j["n_rx"]]
            p, _ = scs[j["scene"]].trace(j["tx"], rx, **prm)
            p["rx"] += j["rx_first"]
            parts.append(p)
    finally:
        for s in scs:
            s.close()
    allp = np.concatenate(parts) if parts else np.zeros(0, parts[0].dtype)
    order = np.lexsort((*[allp["face"][:, j] for j in range(7, -1, -1)], allp["order"],
                        allp["rx"]))
    return allp[order]


def test_batch_equals_individual_traces(gpu):
    """sbr_trace_batch (one persistent trace launch over all jobs and scenes)
    returns byte for byte the paths of the jobs traced one by one."""
    b = _small_batch()
    ref = _individual(gpu, b)
    scs = [gpu.scene(s) for s in b["scenes"]]
    try:
        got, st = gpu.trace_batch(scs, b["jobs"], b["rx"])
    finally:
        for s in scs:
            s.close()
    assert len(ref) > 10
    assert st["n_rays"] == sum(10 * j["division_n"] ** 2 + 2 for j in b["jobs"])
    assert got.tobytes() == ref.tobytes()


def _mixed_batch(seed):
    """A batch whose jobs differ in iteration count, sub-rays and target, so
    that paths leave the refinement queue at different iterations."""
    b = scenes.batch_config(seed, n_scenes=3, n_pairs=40, tri_min=100, tri_max=3000,
                            n_range=(40, 90), order_range=(2, 6), iterations=4)
    rng = np.random.default_rng(seed + 77)
    for j in b["jobs"]:
        j["iterations"] = int(rng.integers(0, 12))
        j["subrays"] = int(rng.choice([6, 7]))
        j["target_err_deg"] = float(rng.choice([0.0, 0.0, 0.05, 0.005]))
    return b


@pytest.mark.parametrize("seed", [11, 12])
def test_batch_queue_mixed_iterations(gpu, seed):
    """Jobs of one batch with their own iteration counts (0 to 11), sub-ray
    counts and targets share the persistent refinement queue (depth 0): every
    job's paths are byte for byte those of its own single call with the
    segment-parallel kernel (the default), and of the batch and the single
    calls refined the other ways (queue, lookahead kernels)."""
    b = _mixed_batch(seed)
    ref = _individual(gpu, b)
    scs = [gpu.scene(s) for s in b["scenes"]]
    base = gpu.tuning()
    try:
        got_seg, _ = gpu.trace_batch(scs, b["jobs"], b["rx"])
        gpu.set_tuning(**dict(base, refine_segments=0))
        got_la, _ = gpu.trace_batch(scs, b["jobs"], b["rx"])
        gpu.set_tuning(**dict(base, lookahead_depth=0))
        got, _ = gpu.trace_batch(scs, b["jobs"], b["rx"])
        ref_q = _individual(gpu, b)
    finally:
        gpu.set_tuning(**base)
        for s in scs:
            s.close()
    assert len(ref) > 15
    assert got.tobytes() == ref.tobytes() == ref_q.tobytes() == got_la.tobytes() == \
        got_seg.tobytes()
    assert len(np.unique(got["iters_used"])) > 2


def test_batch_graph_replay_matches_eager(gpu):
    """SBR_FLAG_GRAPH on every job of a batch: the first call captures a HIP
    graph, later calls with other transmitters and receiver positions replay
    it.  Every replay, with eager batches and synchronizations between the
    replays, gives the same bytes as the batch without the graph; a replay
    that outgrows the captured sizes is redone as a normal call, and a batch
    of another shape is not replayed."""
    import torch
    b = _small_batch(7)
    scs = [gpu.scene(s) for s in b["scenes"]]
    rng = np.random.default_rng(4)
    try:
        replays = 0
        for i in range(6):
            jobs = [dict(j, tx=np.asarray(j["tx"]) + (rng.uniform(-2, 2, 3) if i else 0.0))
                    for j in b["jobs"]]
            rx = b["rx"] + (np.array([1.0, -1.0, 0.0]) if i >= 3 else 0.0)
            got, st = gpu.trace_batch(scs, [dict(j, graph=True) for j in jobs], rx)
            replays += i > 0 and st["ms_trace"] == 0.0  # a replay reports no stage times
            ref, _ = gpu.trace_batch(scs, jobs, rx)  # eager work between replays
            torch.cuda.synchronize()
            assert got.tobytes() == ref.tobytes(), i
            assert st["n_paths"] == len(got)
        assert replays >= 3, replays
        # captured with few paths (transmitters 400 m up), replayed with many
        high = [dict(j, tx=np.asarray(j["tx"]) + np.array([0.0, 0.0, 400.0]), graph=True)
                for j in b["jobs"]]
        gpu.trace_batch(scs, high, b["rx"])
        got, _ = gpu.trace_batch(scs, [dict(j, graph=True) for j in b["jobs"]], b["rx"])
        ref, _ = gpu.trace_batch(scs, b["jobs"], b["rx"])
        assert got.tobytes() == ref.tobytes()
        # another shape (one job fewer) after a capture: a normal call
        got, _ = gpu.trace_batch(scs, [dict(j, graph=True) for j in b["jobs"][1:]], b["rx"])
        ref, _ = gpu.trace_batch(scs, b["jobs"][1:], b["rx"])
        assert got.tobytes() == ref.tobytes()
    finally:
        for s in scs:
            s.close()


def test_batch_job_matches_oracle(gpu, orc):
    b = _small_batch(5)
    scs = [gpu.scene(s) for s in b["scenes"]]
    try:
        got, _ = gpu.trace_batch(scs, b["jobs"], b["rx"])
    finally:
        for s in scs:
            s.close()
    for j in b["jobs"][:4]:
        prm = {k: v for k, v in j.items() if k not in ("scene", "tx", "rx_first", "n_rx")}
        rx = b["rx"][j["rx_first"]:j["rx_first"] + j["n_rx"]]
        o = orc.run(b["scenes"][j["scene"]], j["tx"], rx, **prm)["paths"]
        g = got[(got["rx"] >= j["rx_first"]) & (got["rx"] < j["rx_first"] + j["n_rx"])].copy()
        g["rx"] -= j["rx_first"]
        _compare_paths(g, o)


def test_batch_argument_errors(gpu):
    from paper_2208_10009_amd import sbr
    b = _small_batch()
    scs = [gpu.scene(s) for s in b["scenes"][:2]]
    try:
        bad = [dict(b["jobs"][0], scene=5)]
        with pytest.raises(sbr.SbrError) as e:
            gpu.trace_batch(scs, bad, b["rx"])
        assert e.value.status == sbr.E_INVALID_ARG
        bad = [dict(b["jobs"][0], scene=0, rx_first=0, n_rx=2),
               dict(b["jobs"][1], scene=1, rx_first=1, n_rx=1)]
        with pytest.raises(sbr.SbrError):
            gpu.trace_batch(scs, bad, b["rx"])  # receiver 1 in two jobs
        p, st = gpu.trace_batch(scs, [], b["rx"])
        assert len(p) == 0 and st["n_rays"] == 0
    finally:
        for s in scs:
            s.close()


def test_tuning_roundtrip_and_invariance(gpu):
    """Launch tuning (packet size, persistent workgroups, LDS staging, the
    refinement lookahead) changes scheduling only: results are byte-identical."""
    from paper_2208_10009_amd import sbr
    cfg = scenes.manhattan_config(6, n_rx=12)
    prm = dict(cfg["params"], division_n=70)
    base = gpu.tuning()
    sc = gpu.scene(cfg["scene"])
    try:
        ref, _ = sc.trace(cfg["tx"], cfg["rx"], **prm)
        for t in (dict(trace_chunk=3, persist_blocks=7), dict(persist_blocks=1),
                  dict(lds_budget=65536, stack_depth=8, trace_block=128),
                  dict(lds_budget=24 * 4 * 256, stack_depth=24),
                  dict(lookahead_max_paths=0, trace_chunk=64), dict(rx_tree_min=1),
                  dict(lookahead_depth=2, refine_segments=0), dict(lookahead_depth=1),
                  dict(lookahead_depth=0), dict(lookahead_depth=3, refine_segments=0),
                  dict(ray_order=0), dict(refine_segments=0),
                  dict(refine_segments=1, lds_budget=65536, stack_depth=8),
                  dict(ray_order=0, trace_chunk=2, lds_budget=24 * 4 * 256)):
            gpu.set_tuning(**dict(base, **t))
            assert gpu.tuning()["trace_chunk"] == dict(base, **t)["trace_chunk"]
            got, _ = sc.trace(cfg["tx"], cfg["rx"], **prm)
            assert got.tobytes() == ref.tobytes(), t
        with pytest.raises(sbr.SbrError):
            gpu.set_tuning(trace_block=100)
        with pytest.raises(sbr.SbrError):
            gpu.set_tuning(rx_tree_min=0)
        with pytest.raises(sbr.SbrError):
            gpu.set_tuning(lookahead_depth=4)
        with pytest.raises(sbr.SbrError):
            gpu.set_tuning(lookahead_depth=-1)
        with pytest.raises(sbr.SbrError):
            gpu.set_tuning(ray_order=2)
        with pytest.raises(sbr.SbrError):
            gpu.set_tuning(refine_segments=2)
    finally:
        gpu.set_tuning(**base)
        sc.close()


def test_ray_order_full_size(gpu, orc):
    """Whole-grid jobs hand their rays out sorted by direction cell
    (ray_order = 1, the default) or by index (0): at the benchmark's full size
    (n = 200, 6 reflections, 64 Rx) and at n = 1000 the path records and the
    per-ray traces are byte-identical, and match the oracle."""
    base = gpu.tuning()
    assert base["ray_order"] == 1
    cfg = scenes.manhattan_config(0)
    sc = gpu.scene(cfg["scene"])
    try:
        got = {}
        for o in (1, 0):
            gpu.set_tuning(**dict(base, ray_order=o))
            g, st = sc.trace(cfg["tx"], cfg["rx"], **cfg["params"])
            t, T = sc.trace_rays(cfg["tx"], 200, 6)
            g2, _ = sc.trace(cfg["tx"], cfg["rx"][:8], **dict(cfg["params"], division_n=1000,
                                                                 max_order=2, iterations=1))
            got[o] = (g, t, T, g2)
    finally:
        gpu.set_tuning(**base)
        sc.close()
    for a, b in zip(got[0], got[1]):
        assert a.tobytes() == b.tobytes()
    g, t, T, g2 = got[1]
    assert len(g) > 100 and len(g2) > 0 and t.shape == (400002, 7)
    o = orc.run(cfg["scene"], cfg["tx"], cfg["rx"], **cfg["params"])["paths"]
    _compare_paths(g, o)
    ids = np.unique(np.random.default_rng(12).integers(0, 400002, 3000))
    ot, _, oT = orc.trace_rays(cfg["scene"], cfg["tx"], 200, 6, ids=ids)
    assert np.array_equal(t[ids], ot) and np.array_equal(bits(T[ids]), bits(oT))


# --------------------------------------------------- device-memory variant --
def test_trace_device_matches_host_api(gpu):
    """sbr_trace_device (receivers and paths in device memory) returns the
    same records as sbr_trace: small and large receiver sets (the latter
    through the receiver tree), a too-small output buffer (two-call sizing
    inside the binding) and no receivers."""
    import torch
    from paper_2208_10009_amd import sbr
    base = gpu.tuning()
    for cfg, prm, tree in ((scenes.manhattan_config(0), {}, None),
                           (scenes.manhattan_config(5, n_rx=300), dict(division_n=80), 16)):
        p = dict(cfg["params"], **prm)
        sc = gpu.scene(cfg["scene"])
        try:
            if tree:
                gpu.set_tuning(rx_tree_min=tree)
            ref, st = sc.trace(cfg["tx"], cfg["rx"], **p)
            rx = torch.as_tensor(cfg["rx"], device="cuda")
            got, st2 = sc.trace_device(cfg["tx"], rx, **p)
            small = torch.empty((3, sbr.PATH_DTYPE.itemsize), dtype=torch.uint8, device="cuda")
            got2, _ = sc.trace_device(cfg["tx"], rx, out=small, **p)
            none, _ = sc.trace_device(cfg["tx"], rx[:0], **p)
        finally:
            gpu.set_tuning(**base)
            sc.close()
        g = got.cpu().numpy().reshape(-1).view(sbr.PATH_DTYPE)
        assert len(ref) > 3 and g.tobytes() == ref.tobytes()
        assert got2.cpu().numpy().tobytes() == ref.tobytes()
        assert none.shape[0] == 0 and st2["n_paths"] == st["n_paths"]


def test_trace_device_event_prediction(gpu):
    """Device-memory calls predict their event count from the previous call
    (and skip reading it back after the trace); a call with more events than
    predicted runs again and still returns sbr_trace's records: few events,
    then a few hundred, then more than 4096, then few again."""
    import torch
    from paper_2208_10009_amd import sbr
    cfg = scenes.shoebox_config(7)
    rng = np.random.default_rng(11)
    rx_many = rng.uniform(0.2, 0.8, size=(160, 3)) * np.array([10.0, 8.0, 3.0])
    prm = dict(cfg["params"], iterations=2)
    sc = gpu.scene(cfg["scene"])
    seen = []
    try:
        # a receiver subset with a few hundred events (above the first call's bound)
        mid = next(rx_many[:k] for k in (4, 8, 16, 32, 64)
                   if sc.trace(cfg["tx"], rx_many[:k], **prm)[1]["n_candidates"] > 300)
        for rx_np in (cfg["rx"][:1], mid, rx_many, cfg["rx"][:1], cfg["rx"][:1]):
            ref, st = sc.trace(cfg["tx"], rx_np, **prm)
            got, st2 = sc.trace_device(cfg["tx"], torch.as_tensor(rx_np, device="cuda"), **prm)
            g = got.cpu().numpy().reshape(-1).view(sbr.PATH_DTYPE)
            assert g.tobytes() == ref.tobytes()
            assert st2["n_candidates"] == st["n_candidates"] and st2["n_paths"] == st["n_paths"]
            seen.append(st["n_candidates"])
    finally:
        sc.close()
    assert seen[0] < 128 and 300 < seen[1] <= 4096 and seen[2] > 4096, seen


@pytest.mark.parametrize("fresh", [False, True])
def test_graph_replay_matches_eager(gpu, fresh):
    """SBR_FLAG_GRAPH: the first call captures a HIP graph, later calls with
    other transmitters and receiver positions replay it.  Every replay, with
    eager calls and synchronizations between the replays, gives the same
    bytes as a call without the graph; a replay that outgrows the captured
    sizes is redone as a normal call."""
    import torch
    from paper_2208_10009_amd import sbr
    cfg = scenes.manhattan_config(1, n_rx=32)
    prm = dict(cfg["params"], division_n=90, fresh_grid=fresh)
    sc = gpu.scene(cfg["scene"])
    rec = sbr.PATH_DTYPE.itemsize
    try:
        rx = torch.as_tensor(cfg["rx"], device="cuda")
        out = torch.zeros((2048, rec), dtype=torch.uint8, device="cuda")
        rng = np.random.default_rng(3)
        txs = [cfg["tx"]] + [cfg["tx"] + np.array([rng.uniform(-30, 30), rng.uniform(-30, 30),
                                                   rng.uniform(-10, 10)]) for _ in range(5)]
        replays = 0
        for i, tx in enumerate(txs):
            if i == 3:  # move the receivers in place
                rx.copy_(torch.as_tensor(cfg["rx"] + np.array([3.0, -2.0, 0.0]), device="cuda"))
            got, st = sc.trace_device(tx, rx, out=out, graph=True, **prm)
            got = got.cpu().numpy().tobytes()
            replays += i > 0 and st["ms_trace"] == 0.0  # a replay reports no stage times
            ref, _ = sc.trace_device(tx, rx, **prm)  # eager work between replays
            torch.cuda.synchronize()
            assert got == ref.cpu().numpy().tobytes(), i
            assert st["n_paths"] * rec == len(got)
        assert replays >= 3, replays
        # a transmitter far from the captured one: more paths than captured
        far = np.array([40.0, 40.0, 60.0])
        got, _ = sc.trace_device(far, rx, out=out, graph=True, **prm)
        ref, _ = sc.trace_device(far, rx, **prm)
        assert got.cpu().numpy().tobytes() == ref.cpu().numpy().tobytes()
    finally:
        sc.close()
