"""Seeded synthetic scene and receiver generators.

This module only builds inputs (triangle meshes, transmitter and receiver
positions, materials and run parameters); it holds none of the tracing
method's arithmetic.  Both the HIP path and the CPU oracle are fed from it.

A scene is a dict:
    xyz      float64 [V, 3]   vertex positions in metres
    tri      int32   [T, 3]   vertex indices per triangle
    face_id  int32   [T]      planar polygon ("face") each triangle belongs to
    mat_id   int32   [T]      material index
    eps_r    complex128 [M]   relative permittivity per material (e' - j e'')

The paper's own scenes (an office with 1573 faces and an outdoor scene) are
not available; the generators below stand in for them with the shapes and
sizes of the benchmark configurations: a shoebox room, a Manhattan grid of
box buildings, and a large procedural city of extruded polygons on terrain.
"""
from __future__ import annotations

import numpy as np

CONCRETE = 5.31 + 0.0j
GROUND = 15.0 - 1.0j


def _box(x0, y0, z0, x1, y1, z1):
    """8 vertices and 12 triangles of an axis-aligned box; 6 faces."""
    v = np.array(
        [[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
         [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], np.float64)
    quads = [
        (0, 3, 2, 1),  # z = z0
        (4, 5, 6, 7),  # z = z1
        (0, 1, 5, 4),  # y = y0
        (3, 7, 6, 2),  # y = y1
        (0, 4, 7, 3),  # x = x0
        (1, 2, 6, 5),  # x = x1
    ]
    tris, faces = [], []
    for f, (a, b, c, d) in enumerate(quads):
        tris += [(a, b, c), (a, c, d)]
        faces += [f, f]
    return v, np.array(tris, np.int32), np.array(faces, np.int32)


class SceneBuilder:
    def __init__(self):
        self.xyz, self.tri, self.face, self.mat = [], [], [], []
        self.nv = 0
        self.nf = 0

    def add(self, v, t, f, mat):
        self.xyz.append(np.asarray(v, np.float64))
        self.tri.append(np.asarray(t, np.int32) + self.nv)
        self.face.append(np.asarray(f, np.int32) + self.nf)
        self.mat.append(np.full(len(t), mat, np.int32))
        self.nv += len(v)
        self.nf += int(np.max(f)) + 1 if len(f) else 0

    def quad(self, p0, p1, p2, p3, mat):
        self.add(np.array([p0, p1, p2, p3], np.float64), [(0, 1, 2), (0, 2, 3)], [0, 0], mat)

    def box(self, lo, hi, mat):
        v, t, f = _box(*lo, *hi)
        self.add(v, t, f, mat)

    def scene(self, eps):
        return {
            "xyz": np.concatenate(self.xyz) if self.xyz else np.zeros((0, 3)),
            "tri": np.concatenate(self.tri) if self.tri else np.zeros((0, 3), np.int32),
            "face_id": np.concatenate(self.face) if self.face else np.zeros(0, np.int32),
            "mat_id": np.concatenate(self.mat) if self.mat else np.zeros(0, np.int32),
            "eps_r": np.asarray(eps, np.complex128),
        }


def shoebox(dims=(10.0, 8.0, 3.0), eps=CONCRETE):
    b = SceneBuilder()
    b.box((0.0, 0.0, 0.0), dims, 0)
    return b.scene([eps])


def shoebox_config(seed=0):
    """Shoebox room 10 x 8 x 3 m, 12 triangles, er = 5.31, 28 GHz, Tx at
    (2, 3, 1.5), one Rx uniform in the room, n = 20, up to 3 reflections,
    3 iterations of the precise algorithm with 6 sub-rays."""
    rng = np.random.default_rng(seed)
    dims = np.array([10.0, 8.0, 3.0])
    rx = rng.uniform(0.0, 1.0, size=(1, 3)) * dims
    return {
        "name": "shoebox_10x8x3_n20_k3",
        "scene": shoebox(tuple(dims)),
        "tx": np.array([2.0, 3.0, 1.5]),
        "rx": rx,
        "params": dict(max_order=3, division_n=20, iterations=3, subrays=6, freq_hz=28e9),
    }


def two_ray(size=2000.0, eps=GROUND):
    """A single square ground face at z = 0 (two triangles)."""
    b = SceneBuilder()
    h = size / 2
    b.quad((-h, -h, 0.0), (h, -h, 0.0), (h, h, 0.0), (-h, h, 0.0), 0)
    return b.scene([eps])


def manhattan(seed=0, nx=8, ny=8, pitch=40.0):
    """8 x 8 box buildings on a 40 m pitch (centres 40 i + 20), footprints
    U(20, 30) m, heights U(10, 60) m, closed boxes (12 triangles, 6 faces
    each, material 0 concrete) plus a ground quad over [-40, 360]^2
    (material 1): 770 triangles."""
    rng = np.random.default_rng(seed)
    b = SceneBuilder()
    for i in range(nx):
        for j in range(ny):
            cx, cy = pitch * i + pitch / 2, pitch * j + pitch / 2
            w, d = rng.uniform(20.0, 30.0, size=2)
            h = rng.uniform(10.0, 60.0)
            b.box((cx - w / 2, cy - d / 2, 0.0), (cx + w / 2, cy + d / 2, h), 0)
    lo, hi = -pitch, pitch * nx + pitch
    b.quad((lo, lo, 0.0), (hi, lo, 0.0), (hi, hi, 0.0), (lo, hi, 0.0), 1)
    return b.scene([CONCRETE, GROUND])


def manhattan_config(seed=0, n_rx=64):
    """Manhattan grid, Tx at a street intersection (160, 160, 25), n_rx
    receivers at 1.5 m on random street centrelines, n = 200 (400,002
    rays), up to 6 reflections, 5 iterations with 7 sub-rays."""
    rng = np.random.default_rng(seed + 1000)
    scene = manhattan(seed)
    along = rng.uniform(0.0, 320.0, size=n_rx)
    line = rng.integers(0, 9, size=n_rx) * 40.0
    horiz = rng.integers(0, 2, size=n_rx).astype(bool)
    rx = np.stack([np.where(horiz, along, line), np.where(horiz, line, along),
                   np.full(n_rx, 1.5)], axis=1)
    return {
        "name": "manhattan_8x8_n200_k6_rx64",
        "scene": scene,
        "tx": np.array([160.0, 160.0, 25.0]),
        "rx": rx,
        "params": dict(max_order=6, division_n=200, iterations=5, subrays=7, freq_hz=28e9),
    }


def box_city(seed, n_buildings, pitch=40.0):
    """A square grid of closed box buildings (12 triangles, 6 faces each) on
    `pitch` m centres (footprints U(20, 30) m, heights U(10, 60) m, concrete)
    plus a ground quad one pitch beyond the grid (15 - 1j): 12 n + 2
    triangles.  Streets run along x = pitch i and y = pitch j."""
    rng = np.random.default_rng(seed)
    side = int(np.ceil(np.sqrt(max(n_buildings, 1))))
    b = SceneBuilder()
    placed = 0
    for i in range(side):
        for j in range(side):
            if placed == n_buildings:
                break
            cx, cy = pitch * i + pitch / 2, pitch * j + pitch / 2
            w, d = rng.uniform(20.0, 30.0, size=2)
            h = rng.uniform(10.0, 60.0)
            b.box((cx - w / 2, cy - d / 2, 0.0), (cx + w / 2, cy + d / 2, h), 0)
            placed += 1
    lo, hi = -pitch, pitch * side + pitch
    b.quad((lo, lo, 0.0), (hi, lo, 0.0), (hi, hi, 0.0), (lo, hi, 0.0), 1)
    return b.scene([CONCRETE, GROUND]), side * pitch


def _street_point(rng, extent, pitch, z):
    along = rng.uniform(0.0, extent)
    line = rng.integers(0, int(extent // pitch) + 1) * pitch
    return np.array([along, line, z]) if rng.integers(0, 2) else np.array([line, along, z])


def batch_config(seed=0, n_scenes=16, n_pairs=256, tri_min=200, tri_max=50000, n_range=(50, 400),
                 order_range=(3, 8), iterations=5, subrays=7):
    """Batched workload: n_scenes seeded box-building cities whose triangle
    counts are log-uniform in [tri_min, tri_max], and n_pairs Tx/Rx pairs
    spread unevenly over them (Dirichlet(0.5) shares), each with its own
    division n (uniform in n_range, 10 n^2 + 2 rays) and maximum order
    (uniform in order_range); Tx 5-30 m and Rx 1.5 m above street centrelines,
    28 GHz."""
    rng = np.random.default_rng(seed + 5000)
    tris = np.exp(rng.uniform(np.log(tri_min), np.log(tri_max), size=n_scenes))
    scenes, extents = [], []
    for s in range(n_scenes):
        sc, ext = box_city(seed * 100 + s, max(1, int(round((tris[s] - 2) / 12))))
        scenes.append(sc)
        extents.append(ext)
    share = rng.dirichlet(np.full(n_scenes, 0.5))
    counts = rng.multinomial(n_pairs, share)
    jobs, rx = [], []
    for s in range(n_scenes):
        for _ in range(counts[s]):
            tx = _street_point(rng, extents[s], 40.0, rng.uniform(5.0, 30.0))
            rx.append(_street_point(rng, extents[s], 40.0, 1.5))
            jobs.append(dict(scene=s, tx=tx, rx_first=len(rx) - 1, n_rx=1,
                             max_order=int(rng.integers(order_range[0], order_range[1] + 1)),
                             division_n=int(rng.integers(n_range[0], n_range[1] + 1)),
                             iterations=iterations, subrays=subrays, freq_hz=28e9))
    return {"name": "batch_%dscenes_%dpairs" % (n_scenes, n_pairs), "scenes": scenes,
            "jobs": jobs, "rx": np.array(rx, np.float64).reshape(-1, 3)}


NOMINAL_EPS = (5.3 - 0.4j, 3.8 - 0.1j, 6.3 - 0.05j, 15.0 - 1.0j)


def materials_city(seed=0, n_rx=1024, eps=None):
    """The Manhattan grid with four materials: every building is concrete,
    brick or glass (seeded choice) and the ground is soil; the hidden
    permittivities are the nominal ones perturbed by a seeded factor
    (real part x U(0.9, 1.1), imaginary part x U(0.8, 1.2)) unless eps is
    given.  n_rx receivers at 1.5 m on street centrelines."""
    rng = np.random.default_rng(seed + 7000)
    cfg = manhattan_config(seed, n_rx=n_rx)
    scene = dict(cfg["scene"])
    mat = scene["mat_id"].copy()
    n_build = (len(mat) - 2) // 12
    kinds = rng.integers(0, 3, size=n_build)
    mat[:12 * n_build] = np.repeat(kinds, 12)
    mat[12 * n_build:] = 3
    scene["mat_id"] = mat.astype(np.int32)
    if eps is None:
        nom = np.array(NOMINAL_EPS)
        eps = (nom.real * rng.uniform(0.9, 1.1, 4)) + 1j * (nom.imag * rng.uniform(0.8, 1.2, 4))
    scene["eps_r"] = np.asarray(eps, np.complex128)
    return {"name": "materials_city_4mat_rx%d" % n_rx, "scene": scene, "tx": cfg["tx"],
            "rx": cfg["rx"], "params": dict(cfg["params"], iterations=10,
                                             target_err_deg=0.01)}


def _terrain_height(x, y, coef):
    """Smooth seeded terrain: a sum of a few planar sinusoids (metres)."""
    z = np.zeros(np.broadcast(x, y).shape)
    for a, kx, ky, ph in coef:
        z = z + a * np.sin(kx * x + ky * y + ph)
    return z


def large_city(seed=0, n_buildings=2000, quads=477, extent=1700.0, margin=50.0, plaza=40.0):
    """Procedural city: n_buildings extruded convex polygons (4-12 vertices at
    jittered angles on a circle of radius U(5, 15) m, so every polygon is
    convex; centres rejected when the circles, widened by 2 m each, overlap
    or reach into the central plaza), heights lognormal (median 25 m,
    sigma 0.5), on a heightfield terrain of quads x quads cells over
    [-margin, extent + margin]^2 (two triangles per cell, each its own face,
    since terrain cells are not planar).  Walls are one face per polygon
    edge and run from 2 m below the lowest terrain point under the footprint
    to the roof; roofs are one fan-triangulated face.  Concrete buildings
    (material 0), ground 15 - 1j (material 1).  Returns (scene, info) with
    the terrain coefficients for placing Tx/Rx on it."""
    rng = np.random.default_rng(seed + 9000)
    coef = [(rng.uniform(1.0, 4.0), *(rng.normal(size=2) * 2 * np.pi / rng.uniform(300, 900)),
             rng.uniform(0, 2 * np.pi)) for _ in range(4)]
    # building footprints by rejection on a hash grid of 40 m cells
    cell = 40.0
    grid = {}
    placed = []
    c0 = extent / 2
    attempts = 0
    while len(placed) < n_buildings:
        attempts += 1
        if attempts > 200 * n_buildings:
            raise RuntimeError("could not place %d buildings" % n_buildings)
        r = rng.uniform(5.0, 15.0)
        cx, cy = rng.uniform(r, extent - r, size=2)
        if np.hypot(cx - c0, cy - c0) < plaza + r + 2.0:
            continue
        gx, gy = int(cx // cell), int(cy // cell)
        ok = True
        for i in range(gx - 1, gx + 2):
            for j in range(gy - 1, gy + 2):
                for (px, py, pr) in grid.get((i, j), ()):
                    if np.hypot(cx - px, cy - py) < r + pr + 4.0:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        grid.setdefault((gx, gy), []).append((cx, cy, r))
        placed.append((cx, cy, r))
    b = SceneBuilder()
    for (cx, cy, r) in placed:
        m = int(rng.integers(4, 13))
        step = 2 * np.pi / m
        ang = rng.uniform(0, 2 * np.pi) + step * np.arange(m) + rng.uniform(-0.3, 0.3, m) * step
        px, py = cx + r * np.cos(ang), cy + r * np.sin(ang)
        ground = _terrain_height(np.append(px, cx), np.append(py, cy), coef)
        z0 = ground.min() - 2.0
        z1 = ground[-1] + rng.lognormal(np.log(25.0), 0.5)
        # walls: one quad face per edge
        for e in range(m):
            a, q = e, (e + 1) % m
            b.quad((px[a], py[a], z0), (px[q], py[q], z0), (px[q], py[q], z1),
                   (px[a], py[a], z1), 0)
        # roof: one fan-triangulated face
        v = np.stack([px, py, np.full(m, z1)], 1)
        t = [(0, i, i + 1) for i in range(1, m - 1)]
        b.add(v, t, [0] * len(t), 0)
    # terrain
    xs = np.linspace(-margin, extent + margin, quads + 1)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    Z = _terrain_height(X, Y, coef)
    verts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    i, j = np.meshgrid(np.arange(quads), np.arange(quads), indexing="ij")
    v00 = (i * (quads + 1) + j).ravel()
    v10, v01, v11 = v00 + (quads + 1), v00 + 1, v00 + quads + 2
    tris = np.empty((2 * len(v00), 3), np.int64)
    tris[0::2] = np.stack([v00, v10, v11], 1)
    tris[1::2] = np.stack([v00, v11, v01], 1)
    b.add(verts, tris, np.arange(len(tris)), 1)
    return b.scene([CONCRETE, GROUND]), {"coef": coef, "extent": extent, "buildings": placed}


def large_city_config(seed=0, n_buildings=2000, quads=477, grid=32):
    """Large procedural city (about 500k triangles): Tx 30 m above the
    terrain at the plaza in the centre, grid x grid receivers 1.5 m above the
    terrain on a regular grid over the city (some fall inside buildings and
    receive nothing), n = 1000 (10,000,002 rays), up to 8 reflections,
    5 iterations with 6 sub-rays."""
    scene, info = large_city(seed, n_buildings=n_buildings, quads=quads)
    ext, coef = info["extent"], info["coef"]
    c = ext / 2
    tx = np.array([c, c, float(_terrain_height(c, c, coef)) + 30.0])
    g = (np.arange(grid) + 0.5) * (ext / grid)
    X, Y = np.meshgrid(g, g, indexing="ij")
    rx = np.stack([X.ravel(), Y.ravel(), _terrain_height(X.ravel(), Y.ravel(), coef) + 1.5], 1)
    return {
        "name": "large_city_%dtri_rx%d_n1000_k8" % (len(scene["tri"]), len(rx)),
        "scene": scene, "tx": tx, "rx": rx,
        "params": dict(max_order=8, division_n=1000, iterations=5, subrays=6, freq_hz=28e9),
    }
