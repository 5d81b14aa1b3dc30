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
