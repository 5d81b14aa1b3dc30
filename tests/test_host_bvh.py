"""The BVH builder's split references keep every triangle reachable: a host
build of the builder over the benchmark's scenes, with and without split
references, walks from the root through the FP32 child boxes that contain a
point (exact comparisons) for vertices, edge midpoints and random points of
every split triangle (and a sample of the others), and must reach a leaf that
references the point's triangle."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2208_10009_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2208_10009_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("bvh")
    exe = d / "h"
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-ffp-contract=off", "--cuda-host-only",
                           "-x", "hip", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                           os.path.join(ROOT, "tests", "host", "bvh_cover_harness.cpp"),
                           os.path.join(CSRC, "bvh_build.cpp"), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)
    return str(exe), d


def _write(d, name, sc):
    v = np.ascontiguousarray(sc["xyz"][sc["tri"]].reshape(-1, 9), np.float64)
    p = d / name
    with open(p, "wb") as f:
        f.write(np.int64(len(v)).tobytes())
        f.write(v.tobytes())
    return str(p)


@pytest.mark.parametrize("name,split,bfs", [("manhattan", 50, False), ("manhattan", 400, True),
                                            ("manhattan", 0, False), ("terrain", 100, False),
                                            ("batch", 200, True)])
def test_split_references_cover_their_triangles(harness, name, split, bfs):
    exe, d = harness
    if name == "manhattan":
        sc = scenes.manhattan_config(0)["scene"]
    elif name == "terrain":
        sc = scenes.large_city_config(0, n_buildings=300, quads=80)["scene"]
    else:
        sc = scenes.batch_config(0, n_scenes=2, n_pairs=2, tri_min=20000, tri_max=30000)["scenes"][1]
    f = _write(d, name + ".bin", sc)
    r = subprocess.run([exe, f, str(split), "24"] + (["bfs"] if bfs else []), capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stdout
    fields = dict(kv.split("=") for kv in r.stdout.split())
    assert int(fields["bad"]) == 0
    if split > 0:
        assert int(fields["split_tris"]) > 0 and int(fields["refs"]) > int(fields["T"])
    else:
        assert int(fields["refs"]) == int(fields["T"])
