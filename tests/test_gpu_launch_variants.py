"""GPU launch variants: the equidistant icosahedral and octahedral grids of
Sec. II.A (the paper's comparison methods) as launch modes of the HIP path,
bit-exact against the oracle's grids, traced and refined to the same parity
bar as the equiangular grid; plus the Fig. 2 uniformity ordering and the
traditional-SBR (no iterations) against precise comparison, computed from
the GPU's own output."""
import numpy as np
import pytest

from paper_2208_10009_amd import scenes
from parity_util import angle_deg, bits, compare_paths

pytestmark = pytest.mark.gpu
ICOSA, OCTA = 1, 2


@pytest.mark.parametrize("launch", [ICOSA, OCTA])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 20, 33, 200])
def test_equidistant_grid_bitexact(gpu, orc, launch, n):
    g = gpu.launch_grid(n, launch=launch)
    o = orc.launch_dirs(n, launch=launch)
    assert g.shape == o.shape == (orc.num_rays(n, launch), 3)
    assert np.array_equal(bits(g), bits(o))


@pytest.mark.parametrize("launch", [ICOSA, OCTA])
def test_equidistant_grid_large_n_sampled(gpu, orc, launch):
    n = 1000
    N = orc.num_rays(n, launch)
    rng = np.random.default_rng(3)
    ids = np.unique(np.concatenate([np.arange(64), N - 64 + np.arange(64),
                                    rng.integers(0, N, 4000)]))
    g = gpu.launch_grid(n, launch=launch)
    assert np.array_equal(bits(g[ids]), bits(orc.launch_dirs(n, ids, launch=launch)))


@pytest.mark.parametrize("launch", [ICOSA, OCTA])
def test_equidistant_trace_rays(gpu, orc, launch):
    cfg = scenes.manhattan_config(0)
    n = 50
    sc = gpu.scene(cfg["scene"])
    try:
        gt, gT = sc.trace_rays(cfg["tx"], n, 6, launch=launch)
    finally:
        sc.close()
    ot, _, oT = orc.trace_rays(cfg["scene"], cfg["tx"], n, 6, launch=launch)
    assert np.array_equal(gt, ot) and np.array_equal(bits(gT), bits(oT))


@pytest.mark.parametrize("launch,n", [(ICOSA, 21), (OCTA, 33)])
@pytest.mark.parametrize("iterations", [0, 4])
def test_equidistant_paths_shoebox(gpu, orc, launch, n, iterations):
    cfg = scenes.shoebox_config(2)
    prm = dict(cfg["params"], division_n=n, iterations=iterations, launch=launch,
               keep_invalid=True)
    sc = gpu.scene(cfg["scene"])
    try:
        g, st = sc.trace(cfg["tx"], cfg["rx"], **prm)
    finally:
        sc.close()
    o = orc.run(cfg["scene"], cfg["tx"], cfg["rx"], **prm)["paths"]
    compare_paths(g, o)
    assert st["n_rays"] == orc.num_rays(n, launch) and len(g) > 20


def test_equidistant_paths_manhattan(gpu, orc):
    cfg = scenes.manhattan_config(4, n_rx=16)
    prm = dict(cfg["params"], division_n=60, launch=OCTA, iterations=3)
    sc = gpu.scene(cfg["scene"])
    try:
        g, _ = sc.trace(cfg["tx"], cfg["rx"], **prm)
    finally:
        sc.close()
    compare_paths(g, orc.run(cfg["scene"], cfg["tx"], cfg["rx"], **prm)["paths"])


def _nearest_angles(P):
    G = P @ P.T
    np.fill_diagonal(G, -2.0)
    c = np.clip(G.max(axis=1), -1.0, 1.0)
    return 2.0 * np.arcsin(np.sqrt(np.maximum(0.0, 2.0 - 2.0 * c)) / 2.0)


def test_fig2_uniformity_from_gpu_grids(gpu):
    """Fig. 2: at about 4400 rays, equiangular division on the icosahedron
    spreads rays more evenly than equidistant division on the icosahedron,
    and that more evenly than on the octahedron (nearest-neighbour angle
    spread)."""
    grids = [gpu.launch_grid(21), gpu.launch_grid(21, launch=ICOSA),
             gpu.launch_grid(33, launch=OCTA)]
    cv = [a.std() / a.mean() for a in map(_nearest_angles, grids)]
    ratio = [a.max() / a.min() for a in map(_nearest_angles, grids)]
    assert cv[0] < cv[1] < cv[2] and ratio[0] < ratio[1] < ratio[2]


def test_traditional_vs_precise_accuracy(gpu):
    """Sec. IV: plain (traditional) SBR leaves degree-level AOD errors; the
    precise algorithm brings every path to within 0.01 deg of the exact
    solve."""
    cfg = scenes.shoebox_config(3)
    sc = gpu.scene(cfg["scene"])
    try:
        trad, _ = sc.trace(cfg["tx"], cfg["rx"], max_order=2, division_n=21, iterations=0,
                           launch=ICOSA)
        prec, _ = sc.trace(cfg["tx"], cfg["rx"], max_order=2, division_n=21, iterations=30,
                           target_err_deg=0.01)
    finally:
        sc.close()
    e_trad = angle_deg(trad["aod"], trad["exact_aod"])
    e_prec = angle_deg(prec["aod"], prec["exact_aod"])
    assert e_trad.mean() > 0.2 and e_prec.max() <= 0.01
    assert angle_deg(prec["aoa"], prec["exact_aoa"]).max() <= 0.01
