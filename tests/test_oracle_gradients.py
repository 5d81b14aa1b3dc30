"""Pins of the oracle's analytic Jacobian of the image-method path quantities
(delay, AOD, AOA, power; Sec. IV's quantities at a fixed face sequence)
against FP64 central differences of the oracle's own image-method solve by
back-projection (orc_exact_path), an independent computation of the same
values: in the shoebox room (orders 0-3, one material) and on the
four-material Manhattan grid (lossy permittivities, orders 0-3)."""
import numpy as np
import pytest

from paper_2208_10009_amd import scenes

C0 = 299792458.0
H = 1e-6


def _unit(v):
    return v / np.linalg.norm(v)


def exact_values(orc, scene, tx, rx, faces):
    pts, L, P, valid = orc.exact_path(scene, tx, rx, faces)
    k = len(faces)
    first = pts[0] if k else rx
    last = pts[k - 1] if k else tx
    return np.concatenate([[L / C0], _unit(first - tx), _unit(last - rx), [P]]), valid


def central_differences(orc, scene, tx, rx, faces):
    n_mat = len(scene["eps_r"])
    J = np.zeros((8, 6 + 2 * n_mat))
    for a in range(3):
        e = np.zeros(3)
        e[a] = H
        J[:, a] = (exact_values(orc, scene, tx + e, rx, faces)[0] -
                   exact_values(orc, scene, tx - e, rx, faces)[0]) / (2 * H)
        J[:, 3 + a] = (exact_values(orc, scene, tx, rx + e, faces)[0] -
                       exact_values(orc, scene, tx, rx - e, faces)[0]) / (2 * H)
    for m in range(n_mat):
        for part, dz in ((0, H), (1, 1j * H)):
            sp, sm = dict(scene), dict(scene)
            sp["eps_r"] = scene["eps_r"].copy()
            sm["eps_r"] = scene["eps_r"].copy()
            sp["eps_r"][m] += dz
            sm["eps_r"][m] -= dz
            J[:, 6 + 2 * m + part] = (exact_values(orc, sp, tx, rx, faces)[0] -
                                      exact_values(orc, sm, tx, rx, faces)[0]) / (2 * H)
    return J


def _valid_paths(orc, cfg, rx, max_order, n, per_order):
    p = orc.run(cfg["scene"], cfg["tx"], rx, max_order=max_order, division_n=n, iterations=0,
                subrays=6)["paths"]
    out = []
    for k in range(max_order + 1):
        for q in p[p["order"] == k][:per_order]:
            out.append((int(q["rx"]), list(q["face"][:k])))
    return out


def _check(orc, scene, tx, rx, faces):
    v, J = orc.path_jacobian(scene, tx, rx, faces)
    ev, valid = exact_values(orc, scene, tx, rx, faces)
    assert valid
    assert abs(v[0] - ev[0]) <= 1e-12 * ev[0]
    assert np.abs(v[1:7] - ev[1:7]).max() <= 1e-12
    assert abs(v[7] - ev[7]) <= 1e-9
    N = central_differences(orc, scene, tx, rx, faces)
    # rows scaled to O(1): delay in units of 1 m / c0
    scale = np.array([C0, 1, 1, 1, 1, 1, 1, 1.0])[:, None]
    d = np.abs((J - N) * scale)
    assert d.max() <= 1e-6 * max(1.0, np.abs(J * scale).max()), (faces, d.max())
    return J


@pytest.mark.parametrize("seed", [0, 3])
def test_jacobian_shoebox(orc, seed):
    cfg = scenes.shoebox_config(seed)
    paths = _valid_paths(orc, cfg, cfg["rx"], 3, 20, 4)
    assert {len(f) for _, f in paths} == {0, 1, 2, 3}
    for x, faces in paths:
        _check(orc, cfg["scene"], cfg["tx"], cfg["rx"][x], faces)


def test_jacobian_four_materials(orc):
    cfg = scenes.materials_city(1, n_rx=12)
    paths = _valid_paths(orc, cfg, cfg["rx"], 3, 40, 4)
    assert {len(f) for _, f in paths} >= {0, 1, 2}
    used = set()
    for x, faces in paths:
        J = _check(orc, cfg["scene"], cfg["tx"], cfg["rx"][x], faces)
        used |= {m for m in range(len(cfg["scene"]["eps_r"])) if np.abs(J[7, 6 + 2 * m:]).max() > 0}
    assert len(used) >= 2  # the permittivity columns of several materials are exercised


def test_jacobian_line_of_sight_closed_form(orc):
    """Free space: d delay / d Rx = (Rx - Tx) / (L c0), d power / d Rx =
    -20 / (L ln 10) (Rx - Tx) / L, d AOA / d Tx = (I - u u^T) / L."""
    sc = scenes.two_ray()
    tx, rx = np.array([0.0, 0.0, 30.0]), np.array([200.0, 10.0, 1.5])
    v, J = orc.path_jacobian(sc, tx, rx, [])
    L = np.linalg.norm(rx - tx)
    u = (tx - rx) / L
    assert np.allclose(J[0, 3:6], (rx - tx) / L / C0, rtol=1e-14, atol=0)
    assert np.allclose(J[7, 3:6], -20.0 / (L * np.log(10.0)) * (rx - tx) / L, rtol=1e-13)
    assert np.allclose(J[4:7, 0:3], (np.eye(3) - np.outer(u, u)) / L, atol=1e-16)
    assert np.all(J[:, 6:] == 0)


def _skew_room():
    """Four large planar faces whose normals are pairwise not orthogonal (a
    tilted floor, two walls 70 degrees apart, a tilted ceiling), so that the
    products of the reflections depend on their order and are not symmetric
    (with axis-aligned walls every mirror product is diagonal)."""
    def quad(b, n, c, size=60.0):
        n = _unit(np.asarray(n, float))
        p0 = c * n
        a = _unit(np.cross(n, [0.3, 0.5, 0.8]))
        bb = np.cross(n, a)
        pts = [p0 + size * (sx * a + sy * bb) for sx, sy in ((-1, -1), (1, -1), (1, 1), (-1, 1))]
        b.quad(*pts, len(b.tri) % 2)
    b = scenes.SceneBuilder()
    quad(b, (0.05, 0.1, 1.0), -1.0)                                   # floor
    quad(b, (1.0, 0.0, 0.15), -12.0)                                  # wall 1
    quad(b, (np.cos(np.radians(110)), np.sin(np.radians(110)), -0.1), -12.0)  # wall 2
    quad(b, (-0.1, 0.05, -1.0), -9.0)                                 # ceiling
    return b.scene([5.3 - 0.4j, 3.9 - 0.1j])


def test_jacobian_non_orthogonal_faces(orc):
    sc = _skew_room()
    cfg = {"scene": sc, "tx": np.array([1.0, 2.0, 2.0])}
    rx = np.array([[4.0, -3.0, 1.5], [-2.0, 5.0, 3.0]])
    paths = _valid_paths(orc, cfg, rx, 3, 30, 6)
    assert {len(f) for _, f in paths} == {0, 1, 2, 3}
    asym = False
    for x, faces in paths:
        _check(orc, sc, cfg["tx"], rx[x], faces)
        if len(faces) >= 2:
            J = orc.path_jacobian(sc, cfg["tx"], rx[x], faces)[1]
            asym = asym or not np.allclose(J[4:7, 0:3], J[4:7, 0:3].T, atol=1e-9)
    assert asym  # the AOA's Tx block involves a non-symmetric mirror product
