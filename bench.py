"""Benchmark of the SBR hot path on one MI355X.

One step = one sbr_trace_device call over the whole path: equiangular launch
(recomputed every step), BVH traversal with specular bounces and cone
reception, path test 1, the precise algorithm, image solve / path test 2 /
power, and the canonical emit.  The scene (BVH) is uploaded once before the
timed region and the receivers are a device tensor, so the inputs are
resident in HBM; the paths are written to a device buffer.

Headline workload: the large procedural city (2000 extruded polygon
buildings on a terrain mesh, 498,614 triangles), one Tx 30 m above the
terrain, 1024 Rx on a 32 x 32 grid at 1.5 m, n = 1000 (10,000,002 rays),
up to 8 reflections, 5 iterations of 6 sub-rays, 28 GHz -- the largest
single-GPU configuration, seeded synthetic stand-in for the paper's scenes.
The Manhattan grid (770 triangles, 400,002 rays, 64 Rx), the batched
workload (256 Tx/Rx pairs on 16 scenes, one call against one call per pair)
and the launch-grid comparison are reported beside it.

Prints ONE JSON line: value = launched rays per second of whole-step time for
the headline configuration as stated (I = 5); refined paths per second counts
the paths whose refined AOD and AOA are within 0.01 deg of the exact solve, in
a second timed run that iterates each path to that target; the roofline of
the trace kernel; the CPU oracle baseline on a seeded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rays/s + refined paths/s at ≤0.01° AOA/AOD error; batched vs plain, 1 GPU"
HBM_PEAK_GBS = 8000.0
NODE_BYTES = 128    # BVH4 node: four FP32 child boxes + child references
TRI_BYTES = 80      # FP64 triangle record (v0, e1, e2, face, index)
RAY_BYTES = 24      # FP64 launch direction read per ray
EVENT_BYTES = 56    # reception event record written
# The trace kernel is bound by vector-ALU issue.  Its algorithmic work in
# VALU lane operations (one FP32 or FP64 add, multiply, FMA, min, max or
# compare on one lane): a BVH4 node visit is four slab tests of 15 (six slab
# parameters, three entry and three exit minima/maxima, the two three-way
# combines, the overlap compare); a ray-triangle test is the FP64
# Moller-Trumbore of 50 (two cross products of 9, four dot products of 5,
# o - v0, three divisions, six compares and the u + v add); a segment is the
# specular reflection and the move to the hit point (19).  Reception (eq. (3),
# fused into the same kernel): a receiver-tree box tested against a segment's
# reception cone is 39 (c - o; the largest foot parameter over the box, a dot
# product and three |d_i| h_i terms; its minimum with t; the cone radius
# there; per axis the widened half-extent, the two slab bounds, their two
# products with 1/d_i and the running maximum and minimum; the final
# compare); a receiver tested on a segment is 25 (rx - o, t* = (rx - o).d,
# 0 < t* <= t, the perpendicular f, D + t*, |f|^2 against
# (theta_launch (D + t*))^2).
NODE_OPS = 60
TRI_OPS = 50
SEG_OPS = 19
RX_NODE_OPS = 39
RX_TEST_OPS = 25
RX_NODE_BYTES = 64  # receiver-tree node: box centre and half-extents, first/count/skip
RX_BYTES = 16       # FP32 receiver copy read by the pre-test
# Peak VALU lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (one wave64 instruction per SIMD every 4 cycles, FP32 and FP64 alike; twice
# this in flops is the published 78.6 TFLOP/s FP64 vector peak).
VALU_PEAK_GOPS = 256 * 4 * 16 * 2.4
LARGE = "large_city_498614tri_rx1024_n1000_k8_i5_s6"
MANHATTAN = "manhattan_8x8_770tri_n200_k6_i5_s7_rx64"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRACE_SOURCES = ("trace.hip", "traverse.h", "layout.h", "geom.h")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_trace_counters.txt")


def trace_source_hash():
    """SHA-256 over the sources the trace kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for f in TRACE_SOURCES:
        with open(os.path.join(ROOT, "paper_2208_10009_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_counters(workload):
    """Counter values of the trace kernel for `workload` from the committed
    rocprofv3 summary (HBM bytes per launch from FETCH_SIZE + WRITE_SIZE,
    calibrated; VALU busy and lane utilization), or {} when the summary is
    missing or was taken from other kernel sources."""
    try:
        lines = open(COUNTERS_FILE).read().split("\n")
    except OSError:
        return {}
    kv = {}
    for ln in lines:
        ln = ln.strip()
        if ln and not ln.startswith("#") and "=" in ln:
            k, v = ln.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != trace_source_hash():
        return {}
    pre = workload + "."
    return {k[len(pre):]: float(v) for k, v in kv.items() if k.startswith(pre)}


def trace_roofline(counts, n_rays, kernel_ms, workload):
    """Roofline of the trace kernel: algorithmic VALU lane operations per
    launch over its mean HIP-event time, against the VALU peak; beside it the
    measured HBM traffic and its fraction of 8 TB/s, the bytes the traversal
    touches (served from LDS, L1 and L2, not HBM) and the VALU counters."""
    ops = (counts["nodes"] * NODE_OPS + counts["tris"] * TRI_OPS + counts["segments"] * SEG_OPS
           + counts.get("rx_nodes", 0) * RX_NODE_OPS + counts.get("rx_tests", 0) * RX_TEST_OPS)
    touched = (counts["nodes"] * NODE_BYTES + counts["tris"] * TRI_BYTES + n_rays * RAY_BYTES
               + counts["events"] * EVENT_BYTES + counts.get("rx_nodes", 0) * RX_NODE_BYTES
               + counts.get("rx_tests", 0) * RX_BYTES)
    sec = kernel_ms * 1e-3
    ach = ops / sec / 1e9
    mc = measured_counters(workload)
    traffic = int(mc["hbm_bytes"]) if "hbm_bytes" in mc else None
    return {
        "kernel": "k_trace", "bound": "alu", "achieved": round(ach, 1),
        "peak": VALU_PEAK_GOPS, "unit": "Gop/s", "frac": round(ach / VALU_PEAK_GOPS, 5),
        "traffic": traffic,
        "ops_per_launch": int(ops),
        "ops_per_unit": {"node_visit": NODE_OPS, "triangle_test": TRI_OPS, "segment": SEG_OPS,
                         "rx_node_test": RX_NODE_OPS, "rx_test": RX_TEST_OPS},
        "kernel_ms": round(kernel_ms, 5),
        "hbm": {"achieved_gbs": round(traffic / sec / 1e9, 1) if traffic else None,
                "frac": round(traffic / sec / 1e9 / HBM_PEAK_GBS, 5) if traffic else None},
        "bytes_touched_on_chip_gbs": round(touched / sec / 1e9, 1),
        "valu_busy": mc.get("valu_busy"), "valu_lane_util": mc.get("valu_util"),
        # share of the wave's lanes busy in the traversal's node and triangle
        # loops and the segment loop (instrumented copy of the kernel)
        "node_loop_lanes": round(counts["nodes"] / (64 * counts["wave_node_steps"]), 4)
        if counts.get("wave_node_steps") else None,
        "tri_loop_lanes": round(counts["tris"] / (64 * counts["wave_tri_steps"]), 4)
        if counts.get("wave_tri_steps") else None,
        "segment_loop_lanes": round(counts["segments"] / (64 * counts["wave_seg_steps"]), 4)
        if counts.get("wave_seg_steps") else None,
        "rx_loop_lanes": round((counts.get("rx_nodes", 0) + counts.get("rx_tests", 0)) /
                               (64 * counts["wave_rx_steps"]), 4)
        if counts.get("wave_rx_steps") else None,
        "wave_steps": {k: counts.get(k) for k in ("wave_node_steps", "wave_tri_steps",
                                                   "wave_seg_steps", "wave_rx_steps")},
    }


def angle_deg(a, b):
    c = np.cross(a, b)
    return np.degrees(np.arctan2(np.linalg.norm(c, axis=-1), np.sum(a * b, axis=-1)))


def accurate_mask(p, tol_deg=0.01):
    return (angle_deg(p["aod"], p["exact_aod"]) <= tol_deg) & \
        (angle_deg(p["aoa"], p["exact_aoa"]) <= tol_deg) & ((p["flags"] & 2) == 0)


def cpu_info():
    """Host threads available to this process and the CPU model."""
    try:
        cores = int(os.environ["OMP_NUM_THREADS"])
    except (KeyError, ValueError):
        cores = len(os.sched_getaffinity(0))
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return cores, model


def cpu_baseline_manhattan(cfg, budget_s=8.0, max_runs=20):
    """The FP64 CPU oracle, as it stands, on the Manhattan workload: whole
    runs of the configuration as stated, repeated until about budget_s of
    wall time (rays/s), plus one run in the 0.01 deg target mode (refined
    paths/s)."""
    from oracle import oracle as orc
    orc.build()
    n_rays = 10 * cfg["params"]["division_n"] ** 2 + 2
    runs, t0 = 0, time.perf_counter()
    while runs < max_runs and (runs == 0 or time.perf_counter() - t0 < budget_s):
        orc.run(cfg["scene"], cfg["tx"], cfg["rx"], **cfg["params"])
        runs += 1
    dt = time.perf_counter() - t0
    tprm = dict(cfg["params"], iterations=30, target_err_deg=0.01)
    t1 = time.perf_counter()
    tpaths = orc.run(cfg["scene"], cfg["tx"], cfg["rx"], **tprm)["paths"]
    tdt = time.perf_counter() - t1
    cores, model = cpu_info()
    return {
        "value": n_rays * runs / dt, "unit": "rays/s", "cores": cores, "cpu_model": model,
        "kind": "oracle",
        "sample": "%d full run(s) of the Manhattan workload (%d rays, %d Rx), %.1f s; refined "
                  "paths from one 0.01 deg target run, %.2f s" % (runs, n_rays, len(cfg["rx"]), dt,
                                                                 tdt),
        "refined_paths_per_s": float(accurate_mask(tpaths).sum()) / tdt,
    }


def cpu_baseline_large(cfg, stride=1000, n_rx_sample=32, window_deg=0.4):
    """The FP64 CPU oracle, as it stands, on seeded samples of the headline
    workload.  Rays/s: every stride-th launch ray of the large city (brute
    force over all 498,614 triangles, all 1024 receivers, up to 8
    reflections), timed and scaled (the whole 10,000,002-ray run would take
    stride times as long).  Such a sample holds about one reception event,
    so refined paths/s comes from a second sample: the launch rays within
    window_deg of the direct and the ground-image directions from the Tx to
    n_rx_sample seeded receivers (image about the terrain height under the
    receiver), traced with capture at all receivers, path test 1 over their
    events, then the precise algorithm, solve and power of the winners in
    the 0.01 deg target mode, timed."""
    from oracle import oracle as orc
    orc.build()
    prm = cfg["params"]
    n, K = prm["division_n"], prm["max_order"]
    N = 10 * n * n + 2
    ids = np.arange(0, N, stride, dtype=np.int64)
    t0 = time.perf_counter()
    orc.ray_events(cfg["scene"], cfg["tx"], cfg["rx"], n, K, ids)
    dt = time.perf_counter() - t0
    # refinement sample: window rays around the direct and ground-image
    # directions (sampling only: which rays, not what they hit)
    tx, rx = np.asarray(cfg["tx"], float), np.asarray(cfg["rx"], float)
    pick = np.random.default_rng(2208).choice(len(rx), n_rx_sample, replace=False)
    dirs = orc.launch_dirs(n)
    cosw = np.cos(np.radians(window_deg))
    sel = []
    for j in pick:
        img = rx[j].copy()
        img[2] = 2.0 * (rx[j, 2] - 1.5) - rx[j, 2]
        for q in (rx[j], img):
            c = (q - tx) / np.linalg.norm(q - tx)
            sel.append(np.flatnonzero(dirs @ c > cosw))
    del dirs
    wids = np.unique(np.concatenate(sel)).astype(np.int64)
    t1 = time.perf_counter()
    ev = orc.ray_events(cfg["scene"], cfg["tx"], cfg["rx"], n, K, wids)
    win = orc.path_test1(ev)
    edt = time.perf_counter() - t1
    tprm = dict(prm, iterations=30, target_err_deg=0.01)
    t2 = time.perf_counter()
    rec = orc.path_records(cfg["scene"], cfg["tx"], cfg["rx"], win, **tprm) if len(win) else []
    tdt = time.perf_counter() - t2
    good = int(accurate_mask(rec).sum()) if len(win) else 0
    orders = sorted(collections.Counter(int(o) for o in rec["order"]).items()) if len(win) else []
    cores, model = cpu_info()
    return {
        "value": len(ids) / dt, "unit": "rays/s", "cores": cores, "cpu_model": model,
        "kind": "oracle",
        "sample": "rays/s: every %dth launch ray of the large city (%d of %d rays, seeded ray "
                  "indices 0, %d, ...), all 1024 Rx, K = 8: %.1f s, extrapolated (a whole run "
                  "is %d times longer); refined paths/s: the %d launch rays within %.1f deg of "
                  "the direct and ground-image directions to %d seeded Rx (traced and path test "
                  "1 in %.1f s, untimed for the rate), their %d path-test-1 winners (orders %s) "
                  "iterated to 0.01 deg, %.2f s"
                  % (stride, len(ids), N, stride, dt, stride, len(wids), window_deg,
                     n_rx_sample, edt, len(win), dict(orders), tdt),
        "refined_paths_per_s": good / tdt if len(win) and tdt > 0 else None,
        "sample_events": int(len(ev)), "sample_paths_within_0.01deg": good,
    }


def miss_breakdown(p):
    """Why paths end outside 0.01 deg: counts by outcome, with the largest
    AOD and AOA errors of each."""
    ea = angle_deg(p["aod"], p["exact_aod"])
    eo = angle_deg(p["aoa"], p["exact_aoa"])
    ok = accurate_mask(p)
    st = (p["flags"] & 1) != 0
    inv = (p["flags"] & 2) != 0
    met = (p["flags"] & 4) != 0
    out = {}
    for name, m in (("stalled", st & ~inv), ("invalid", inv),
                    ("target_met_aoa_over", met & ~st & ~inv & ~ok),
                    ("iteration_cap", ~met & ~st & ~inv & ~ok)):
        m = m & ~ok
        out[name] = {"paths": int(m.sum()),
                     "max_aod_err_deg": float(ea[m].max()) if m.any() else None,
                     "max_aoa_err_deg": float(eo[m].max()) if m.any() else None,
                     "orders": sorted(set(int(x) for x in p["order"][m]))}
    return out


def error_histogram(p):
    """Refined against exact (image-method) quantities of the valid paths,
    per reflection order: counts of AOD and AOA errors per decade of degrees
    (bins [0, 1e-6), [1e-6, 1e-5), ..., [1, inf)), the median and largest
    angle errors, the largest relative length error and the largest power
    error in dB."""
    edges = [0.0] + [10.0 ** e for e in range(-6, 1)] + [np.inf]
    labels = ["<1e-6"] + ["%g-%g" % (edges[i], edges[i + 1]) for i in range(1, len(edges) - 2)] \
        + [">=1"]
    v = p[(p["flags"] & 2) == 0]
    ea = angle_deg(v["aod"], v["exact_aod"])
    eo = angle_deg(v["aoa"], v["exact_aoa"])
    el = np.abs(v["length_m"] - v["exact_length_m"]) / v["exact_length_m"]
    ep = np.abs(v["power_dbm"] - v["exact_power_dbm"])
    out = {"bins_deg": labels}
    for k in sorted(set(int(x) for x in v["order"])):
        m = v["order"] == k
        out[str(k)] = {
            "paths": int(m.sum()),
            "aod_hist": np.histogram(ea[m], edges)[0].tolist(),
            "aoa_hist": np.histogram(eo[m], edges)[0].tolist(),
            "aod_median_deg": float(np.median(ea[m])), "aod_max_deg": float(ea[m].max()),
            "aoa_median_deg": float(np.median(eo[m])), "aoa_max_deg": float(eo[m].max()),
            "length_max_rel": float(el[m].max()), "power_max_db": float(ep[m].max())}
    return out


def batch_vs_plain(ctx, scenes, torch, seed=0, steps=2):
    """The batched workload (16 box-building cities of 200-50k triangles,
    256 Tx/Rx pairs spread unevenly over them, n in 50-400, K in 3-8), each
    pair refined to 0.01 deg: one sbr_trace_batch call (persistent trace
    over all jobs) against one sbr_trace call per pair, each side autotuned
    over the same space.  Launch grids are cached (both sides), the scenes'
    BVHs are built beforehand.  The per-pair results, renumbered to the
    batch's receivers, must equal the batch's byte for byte."""
    from paper_2208_10009_amd import autotune
    b = scenes.batch_config(seed)
    jobs = [dict(j, iterations=30, target_err_deg=0.01) for j in b["jobs"]]
    n_rays = sum(10 * j["division_n"] ** 2 + 2 for j in jobs)
    t0 = time.perf_counter()
    scs = [ctx.scene(s) for s in b["scenes"]]
    build_s = time.perf_counter() - t0
    ctx.trace_batch(scs, jobs, b["rx"])  # warm-up: launch grids of every n
    base = ctx.tuning()
    # depth 0: the refinement's persistent work queue; 3: the lookahead
    # kernels, or with refine_segments the segment-parallel kernel
    space = {"trace_chunk": [1, 2, 4], "persist_blocks": [1024, 2048, 4096],
             "lookahead_max_paths": [0, 4096], "lookahead_depth": [0, 3],
             "refine_segments": [1, 0]}
    best, trials = autotune.autotune(ctx, lambda: ctx.trace_batch(scs, jobs, b["rx"]),
                                     space=space, warmup=0, steps=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pb, stb = ctx.trace_batch(scs, jobs, b["rx"])
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / steps
    # the same batch captured as a HIP graph (first call) and replayed
    gjobs = [dict(j, graph=True) for j in jobs]
    ctx.trace_batch(scs, gjobs, b["rx"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pg, stg = ctx.trace_batch(scs, gjobs, b["rx"])
    torch.cuda.synchronize()
    tg = (time.perf_counter() - t0) / steps
    assert pg.tobytes() == pb.tobytes(), "graph replay differs from the batch"

    def plain_pass():
        got = []
        for j in jobs:
            prm = {k: v for k, v in j.items() if k not in ("scene", "tx", "rx_first", "n_rx")}
            rx = b["rx"][j["rx_first"]:j["rx_first"] + j["n_rx"]]
            p, _ = scs[j["scene"]].trace(j["tx"], rx, **prm)
            p["rx"] += j["rx_first"]
            got.append(p)
        return np.concatenate(got)

    ctx.set_tuning(**base)
    best_p, _ = autotune.autotune(ctx, plain_pass, space=space, warmup=0, steps=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pp = plain_pass()
    torch.cuda.synchronize()
    tp = (time.perf_counter() - t0) / steps
    for sc in scs:
        sc.close()
    ctx.set_tuning(**base)
    pp = pp[np.argsort(pp["rx"], kind="stable")]
    assert pp.tobytes() == pb.tobytes(), "batched paths differ from one call per pair"
    gb, gp = int(accurate_mask(pb).sum()), int(accurate_mask(pp).sum())
    return {
        "workload": "batch_16scenes_200-50k_tri_256pairs_n50-400_k3-8_target0.01deg",
        "triangles": [int(len(s["tri"])) for s in b["scenes"]], "pairs": len(jobs),
        "rays": int(n_rays), "bvh_build_s": round(build_s, 3),
        "same_bytes_as_one_call_per_pair": True,
        "batched": {"ms": round(1e3 * tb, 3), "rays_per_s": n_rays / tb,
                    "paths": int(len(pb)), "within_0.01deg": gb,
                    "refined_paths_per_s": gb / tb, "tuning": best,
                    "tuning_trials": len(trials),
                    "stage_ms": {k: round(float(stb[k]), 4) for k in
                                 ("ms_launch", "ms_trace", "ms_dedup", "ms_refine", "ms_solve",
                                  "ms_emit", "ms_total")}},
        "graph_replay": {"ms": round(1e3 * tg, 3), "rays_per_s": n_rays / tg,
                         "replayed": bool(stg["ms_trace"] == 0.0),
                         "same_bytes_as_batch": True},
        "plain": {"ms": round(1e3 * tp, 3), "rays_per_s": n_rays / tp, "paths": int(len(pp)),
                  "tuning": best_p, "within_0.01deg": gp, "refined_paths_per_s": gp / tp},
        "speedup": tp / tb,
    }


STAGES = ("ms_launch", "ms_trace", "ms_dedup", "ms_refine", "ms_solve", "ms_emit", "ms_total")


def timed_device(sc, cfg, torch, steps, warmup, out_buf, **kw):
    """steps timed sbr_trace_device calls (after warmup ones): paths of the
    last call, wall seconds, mean stage milliseconds (HIP events)."""
    from paper_2208_10009_amd import sbr
    rx_dev = torch.as_tensor(cfg["rx"], device="cuda")
    for _ in range(warmup):
        sc.trace_device(cfg["tx"], rx_dev, out=out_buf, **kw)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        got, st = sc.trace_device(cfg["tx"], rx_dev, out=out_buf, **kw)
        stats.append(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    paths = got.cpu().numpy().reshape(-1).view(sbr.PATH_DTYPE)
    stage = {k: float(np.mean([x[k] for x in stats])) for k in STAGES}
    return paths, wall, stage, stats


def large_city_leg(ctx, scenes, torch, steps, warmup, tuning=None):
    """The headline: the large procedural city (498,614 triangles, 1024 Rx on
    a 32 x 32 grid, n = 1000: 10,000,002 rays, K = 8, I = 5, S = 6), one
    sbr_trace_device call per step with the launch grid recomputed: rays/s,
    stage times, the trace kernel's roofline, refined paths/s in the 0.01 deg
    target mode and why paths miss it."""
    from paper_2208_10009_amd import autotune, sbr
    cfg = scenes.large_city_config(0)
    prm = cfg["params"]
    n_rays = 10 * prm["division_n"] ** 2 + 2
    t0 = time.perf_counter()
    sc = ctx.scene(cfg["scene"])
    build_s = time.perf_counter() - t0
    rx_tune = torch.as_tensor(cfg["rx"], device="cuda")
    if tuning:
        ctx.set_tuning(**dict(ctx.tuning(), **tuning))
        best = tuning
    else:
        best, _ = autotune.autotune(
            ctx, lambda: sc.trace_device(cfg["tx"], rx_tune, **prm),
            space={"trace_chunk": [1, 2], "persist_blocks": [1024, 2048, 640, 768],
                   "rx_tree_min": [16, 1 << 30], "lds_budget": [65536, 0, 24 * 4 * 256],
                   "stack_depth": [24]}, warmup=1, steps=2)
    log("large city tuning", best)
    # work counts in the timed tuning (the receiver tree depends on it)
    counts = sc.trace_counters(cfg["tx"], cfg["rx"], **prm)
    log("large city counts", counts)
    out_buf = torch.empty((8192, sbr.PATH_DTYPE.itemsize), dtype=torch.uint8, device="cuda")
    paths, wall, stage, stats = timed_device(sc, cfg, torch, steps, warmup, out_buf,
                                             fresh_grid=True, **prm)
    ms = 1e3 * wall / steps
    log("large city stages (mean ms):", json.dumps(stage))
    tpaths, twall, tstage, _ = timed_device(sc, cfg, torch, steps, 1, out_buf, fresh_grid=True,
                                            **dict(prm, iterations=30, target_err_deg=0.01))
    tms = 1e3 * twall / steps
    sc.close()
    tgood = int(accurate_mask(tpaths).sum())
    t_paths_ms = tstage["ms_dedup"] + tstage["ms_refine"] + tstage["ms_solve"] + tstage["ms_emit"]
    return cfg, {
        "value": n_rays * steps / wall, "ms_per_step": ms,
        "triangles": int(len(cfg["scene"]["tri"])), "rx": int(len(cfg["rx"])), "rays": n_rays,
        "bvh_build_s": round(build_s, 3),
        "trace_rays_per_s": n_rays / (stage["ms_trace"] * 1e-3),
        "paths": int(len(paths)), "stage_ms": {k: round(v, 4) for k, v in stage.items()},
        "counts": counts, "tuning": ctx.tuning(),
        "lds": {k: int(stats[-1][k]) for k in ("lds_bytes", "lds_nodes", "lds_tris", "lds_max")},
        "roofline": trace_roofline(counts, n_rays, stage["ms_trace"], LARGE),
        "refined_paths_per_s": tgood / (tms * 1e-3),
        "refined_paths": {
            "mode": "target 0.01 deg (AOD, AOA via L_last/L_total), at most 30 iterations",
            "paths": int(len(tpaths)), "within_0.01deg": tgood, "ms_per_step": round(tms, 4),
            "per_s_paths_stages": tgood / (t_paths_ms * 1e-3),
            "mean_iterations": float(np.mean(tpaths["iters_used"])) if len(tpaths) else 0.0,
            "stage_ms": {k: round(v, 4) for k, v in tstage.items()},
            "misses": miss_breakdown(tpaths), "errors_by_order": error_histogram(tpaths)},
        "fixed_i5": {"paths": int(len(paths)), "within_0.01deg": int(accurate_mask(paths).sum()),
                     "errors_by_order": error_histogram(paths)},
    }


def manhattan_leg(ctx, scenes, torch, args):
    """The Manhattan grid (8 x 8 box buildings plus ground, 770 triangles),
    Tx at 25 m, 64 Rx at 1.5 m on street centrelines, n = 200 (400,002
    rays), K = 6, I = 5, S = 7: rays/s as stated, with cached launch
    directions, through the host-array entry point and replayed from a
    captured HIP graph; refined paths/s; the trace kernel's roofline."""
    from paper_2208_10009_amd import autotune, sbr
    cfg = scenes.manhattan_config(args.seed)
    prm = cfg["params"]
    sc = ctx.scene(cfg["scene"])
    n_rays = 10 * prm["division_n"] ** 2 + 2
    rx_tune = torch.as_tensor(cfg["rx"], device="cuda")
    entry = ctx.tuning()
    if args.tuning:
        ctx.set_tuning(**dict(entry, **args.tuning))
        best = args.tuning
    else:
        best, _ = autotune.autotune(
            ctx, lambda: sc.trace_device(cfg["tx"], rx_tune, **prm),
            space={"trace_chunk": [1, 2], "persist_blocks": [640, 704, 768, 1024, 2048],
                   "lds_budget": [65536, 0, 24 * 4 * 256], "stack_depth": [24],
                   "lookahead_max_paths": [4096], "rx_tree_min": [16, 1 << 30]}, warmup=1,
            steps=5)
    log("manhattan tuning", best)
    counts = sc.trace_counters(cfg["tx"], cfg["rx"], **prm)
    out_buf = torch.empty((4096, sbr.PATH_DTYPE.itemsize), dtype=torch.uint8, device="cuda")
    steps, warmup = args.steps, args.warmup
    paths, wall, stage, stats = timed_device(sc, cfg, torch, steps, warmup, out_buf,
                                             fresh_grid=True, **prm)
    # launch directions cached in the context (a tracer serving many calls at one n)
    _, wall_c, _, _ = timed_device(sc, cfg, torch, steps, 1, out_buf, **prm)
    # the host-array entry point: receivers and paths cross PCIe every call
    for _ in range(1):
        sc.trace(cfg["tx"], cfg["rx"], fresh_grid=True, **prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sc.trace(cfg["tx"], cfg["rx"], fresh_grid=True, **prm)
    torch.cuda.synchronize()
    wall_h = time.perf_counter() - t0
    # replayed from a captured HIP graph
    gpaths, wall_g, _, gstats = timed_device(sc, cfg, torch, steps, 2, out_buf, fresh_grid=True,
                                             graph=True, **prm)
    graph_replays = sum(1 for st in gstats if st["ms_trace"] == 0.0)
    assert gpaths.tobytes() == paths.tobytes(), "graph replay differs from the eager call"
    tpaths, twall, tstage, _ = timed_device(sc, cfg, torch, steps, 1, out_buf, fresh_grid=True,
                                            **dict(prm, iterations=30, target_err_deg=0.01))
    tms = 1e3 * twall / steps
    tgood = int(accurate_mask(tpaths).sum())
    sc.close()
    tuning = ctx.tuning()
    ctx.set_tuning(**entry)
    return cfg, {
        "workload": MANHATTAN, "triangles": len(cfg["scene"]["tri"]), "rays": n_rays,
        "rx": len(cfg["rx"]), "value": n_rays * steps / wall, "ms_per_step": 1e3 * wall / steps,
        "value_cached_grid": n_rays * steps / wall_c,
        "value_host_arrays_pcie": n_rays * steps / wall_h,
        "value_graph_replay": n_rays * steps / wall_g, "graph_replays": graph_replays,
        "trace_rays_per_s": n_rays / (stage["ms_trace"] * 1e-3),
        "stage_ms": {k: round(v, 5) for k, v in stage.items()}, "counts": counts,
        "lds": {k: int(stats[-1][k]) for k in ("lds_bytes", "lds_nodes", "lds_tris", "lds_max")},
        "tuning": tuning,
        "roofline": trace_roofline(counts, n_rays, stage["ms_trace"], MANHATTAN),
        "refined_paths_per_s": tgood / (tms * 1e-3),
        "refined_paths": {"paths": int(len(tpaths)), "within_0.01deg": tgood,
                          "ms_per_step": round(tms, 4),
                          "mean_iterations": float(np.mean(tpaths["iters_used"])),
                          "stage_ms": {k: round(v, 5) for k, v in tstage.items()},
                          "misses": miss_breakdown(tpaths), "errors_by_order": error_histogram(tpaths)},
        "fixed_i5": {"paths": int(len(paths)), "within_0.01deg": int(accurate_mask(paths).sum()),
                     "errors_by_order": error_histogram(paths)},
    }


def launch_variants(ctx, scenes, torch, steps=3):
    """Sec. II / Sec. IV comparison on the Manhattan workload at about 400k
    rays per grid: the paper's equiangular icosahedral grid and the
    equidistant icosahedral and octahedral grids it is compared with, each
    traced as traditional SBR (no iterations) and with the precise algorithm
    to 0.01 deg: time, paths, and AOD/AOA error against the exact solve."""
    cfg = scenes.manhattan_config(0)
    sc = ctx.scene(cfg["scene"])
    out = []
    for name, launch, n in (("equiangular_icosa", 0, 200), ("equidistant_icosa", 1, 200),
                            ("equidistant_octa", 2, 316)):
        for mode, kw in (("traditional", dict(iterations=0)),
                         ("precise_0.01deg", dict(iterations=30, target_err_deg=0.01))):
            prm = dict(cfg["params"], division_n=n, launch=launch, **kw)
            sc.trace(cfg["tx"], cfg["rx"], **prm)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                p, _ = sc.trace(cfg["tx"], cfg["rx"], **prm)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / steps
            ea = angle_deg(p["aod"], p["exact_aod"]) if len(p) else np.zeros(0)
            eo = angle_deg(p["aoa"], p["exact_aoa"]) if len(p) else np.zeros(0)
            out.append({"grid": name, "n": n, "rays": 10 * n * n + 2 if launch < 2 else 4 * n * n + 2,
                        "mode": mode, "ms": round(ms, 4), "paths": int(len(p)),
                        "aod_err_deg_mean": float(ea.mean()) if len(p) else None,
                        "aod_err_deg_max": float(ea.max()) if len(p) else None,
                        "aoa_err_deg_mean": float(eo.mean()) if len(p) else None,
                        "within_0.01deg": int(accurate_mask(p).sum())})
    sc.close()
    return out


def diffraction_leg(ctx, scenes, torch, steps=5):
    """Order-1 diffraction (the paper's second workload, Sec. IV) on the
    Manhattan grid: 768 wedges, Tx at 25 m, 64 Rx, n = 200 (400,002 rays),
    10 iterations of 6 sub-rays as in the paper, then the 0.01 deg target
    mode: one sbr_diffract call per step, rays/s, paths, the AOD and AOA
    errors against the exact (Keller) paths before and after refinement."""
    cfg = scenes.manhattan_config(0)
    prm = dict(division_n=200, iterations=10, subrays=6)
    sc = ctx.scene(cfg["scene"])
    n_w = len(sc.wedges())
    N = 10 * 200 * 200 + 2

    def timed(**kw):
        sc.diffract(cfg["tx"], cfg["rx"], **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            p, st = sc.diffract(cfg["tx"], cfg["rx"], **kw)
        torch.cuda.synchronize()
        return p, st, (time.perf_counter() - t0) / steps

    p0, _, _ = timed(**dict(prm, iterations=0))
    p10, st10, t10 = timed(**prm)
    pt, stt, tt = timed(**dict(prm, iterations=30, target_err_deg=0.01))
    sc.close()

    def errs(p):
        return (float(angle_deg(p["aod"], p["exact_aod"]).mean()) if len(p) else None,
                float(angle_deg(p["aoa"], p["exact_aoa"]).mean()) if len(p) else None)

    e0, e10, et = errs(p0), errs(p10), errs(pt)
    good = int(accurate_mask(pt).sum())
    return {
        "workload": "manhattan_8x8_770tri_768wedges_n200_rx64_order1_diffraction",
        "wedges": n_w, "rays": N, "paths": int(len(p10)),
        "ms_per_call_i10": round(1e3 * t10, 4), "rays_per_s": N / t10,
        "stage_ms_i10": {k: round(float(st10[k]), 4) for k in STAGES},
        "mean_err_deg": {"traditional": {"aod": e0[0], "aoa": e0[1]},
                         "i10": {"aod": e10[0], "aoa": e10[1]},
                         "target_0.01deg": {"aod": et[0], "aoa": et[1]}},
        "refined_paths_per_s": good / tt, "within_0.01deg": good, "target_paths": int(len(pt)),
        "ms_per_call_target": round(1e3 * tt, 4),
        "stage_ms_target": {k: round(float(stt[k]), 4) for k in STAGES},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-vs-plain comparison on the 256-pair workload")
    ap.add_argument("--no-manhattan", action="store_true",
                    help="skip the Manhattan (770 triangles, 400k rays, 64 Rx) leg")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the launch-grid / traditional-vs-precise comparison")
    ap.add_argument("--no-diffraction", action="store_true",
                    help="skip the order-1 diffraction leg")
    ap.add_argument("--large-only", action="store_true",
                    help="run only the headline large-city leg and print its JSON object "
                         "(profiling)")
    ap.add_argument("--manhattan-only", action="store_true",
                    help="run only the Manhattan leg and print its JSON object (profiling)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched-vs-plain comparison and print its JSON object")
    ap.add_argument("--tuning", type=json.loads, default=None, metavar="JSON",
                    help="tuning fields for the Manhattan leg instead of autotuning "
                         "(profiling runs pin what an earlier run chose)")
    ap.add_argument("--large-tuning", type=json.loads, default=None, metavar="JSON",
                    help="the same for the large-city leg")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes 5 times (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2208_10009_amd import sbr, scenes

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.copy_probe:
        x = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copy probe: 5 x %d bytes" % (x.numel() * 4))
        return
    ctx = sbr.Context(0)
    if args.manhattan_only:
        print(json.dumps(manhattan_leg(ctx, scenes, torch, args)[1]), flush=True)
        ctx.close()
        return
    if args.batch_only:
        print(json.dumps(batch_vs_plain(ctx, scenes, torch)), flush=True)
        ctx.close()
        return
    lcfg, lc = large_city_leg(ctx, scenes, torch, args.steps, args.warmup,
                              tuning=args.large_tuning)
    if args.large_only:
        print(json.dumps(lc), flush=True)
        ctx.close()
        return
    prm = lcfg["params"]
    out = {
        "metric": METRIC,
        "value": lc.pop("value"),
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": lc.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": LARGE, "triangles": lc["triangles"], "rays": lc["rays"], "rx": lc["rx"],
            "max_order": prm["max_order"], "iterations": prm["iterations"],
            "subrays": prm["subrays"], "freq_hz": prm["freq_hz"], "mode": "plain",
        },
        "refined_paths_per_s": lc.pop("refined_paths_per_s"),
        "roofline": lc.pop("roofline"),
    }
    out.update(lc)
    mcfg = None
    if not args.no_manhattan:
        mcfg, out["manhattan"] = manhattan_leg(ctx, scenes, torch, args)
        log("manhattan", json.dumps(out["manhattan"]))
    if not args.no_variants:
        out["launch_variants"] = launch_variants(ctx, scenes, torch)
    if not args.no_diffraction:
        out["diffraction"] = diffraction_leg(ctx, scenes, torch)
        log("diffraction", json.dumps(out["diffraction"]))
    if not args.no_batch:
        out["batched"] = batch_vs_plain(ctx, scenes, torch)
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_large(lcfg)
        log("cpu baseline", json.dumps(out["cpu_baseline"]))
        if mcfg is not None:
            out["manhattan"]["cpu_baseline"] = cpu_baseline_manhattan(mcfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
