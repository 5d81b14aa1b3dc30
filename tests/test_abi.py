"""Host-side checks of the C ABI that need no GPU: the library builds for
gfx950, loads, and exports every function include/sbr.h declares; the Python
binding's record layouts match the header's structs; the product path has no
CPU fallback."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sbr.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\*?\s+\*?(sbr_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def built_lib():
    from paper_2208_10009_amd import sbr
    if not os.path.exists(sbr.LIB_PATH):
        from paper_2208_10009_amd import build
        build.build()
    return sbr


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["sbr_context_create", "sbr_context_destroy", "sbr_scene_upload", "sbr_bvh_build",
              "sbr_trace", "sbr_scene_destroy", "sbr_status_string", "sbr_last_error",
              "sbr_candidates", "sbr_launch_grid", "sbr_trace_rays"]:
        assert n in names


def test_library_exports_every_declared_symbol(built_lib):
    lib = C.CDLL(built_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(built_lib.EXPORTS) == declared_functions()


def test_exported_symbols_are_c_linkage(built_lib):
    out = subprocess.run(["nm", "-D", "--defined-only", built_lib.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in declared_functions():
        assert name in syms


def test_status_strings_without_device(built_lib):
    lib = C.CDLL(built_lib.LIB_PATH)
    lib.sbr_status_string.restype = C.c_char_p
    assert lib.sbr_status_string(0) == b"ok"
    assert lib.sbr_status_string(-4) == b"output capacity too small"


def _struct_layout_probe():
    """Compile a tiny C program against the header and print struct sizes and
    offsets, so the binding's numpy dtypes are checked against the compiler."""
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "sbr.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(sbr_path), sizeof(sbr_candidate),
         sizeof(sbr_trace_params), sizeof(sbr_trace_stats), sizeof(sbr_complex),
         sizeof(sbr_diff_path), sizeof(sbr_wedge), offsetof(sbr_diff_path, exact_point),
         offsetof(sbr_diff_path, init_tan_err));
  printf("%zu %zu %zu %zu %zu %zu\n", offsetof(sbr_path, launch_ray), offsetof(sbr_path, tan_err),
         offsetof(sbr_path, delay_s), offsetof(sbr_path, exact_delay_s),
         offsetof(sbr_path, init_tan_err), offsetof(sbr_candidate, tan_err));
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(sbr_tuning),
         offsetof(sbr_tuning, lookahead_max_paths), offsetof(sbr_tuning, ray_order),
         offsetof(sbr_tuning, refine_segments), sizeof(sbr_bvh_params),
         offsetof(sbr_bvh_params, split_pct), sizeof(sbr_job));
  return 0;
}
"""
    import tempfile
    d = tempfile.mkdtemp()
    c = os.path.join(d, "probe.c")
    open(c, "w").write(src)
    exe = os.path.join(d, "probe")
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
    lines = subprocess.check_output([exe], text=True).split("\n")
    return ([int(x) for x in lines[0].split()], [int(x) for x in lines[1].split()],
            [int(x) for x in lines[2].split()])


def test_binding_layouts_match_header():
    from paper_2208_10009_amd import sbr
    sizes, offs, more = _struct_layout_probe()
    assert sizes[0] == sbr.PATH_DTYPE.itemsize
    assert sizes[1] == sbr.CAND_DTYPE.itemsize
    assert sizes[2] == C.sizeof(sbr.TraceParams)
    assert sizes[3] == C.sizeof(sbr.TraceStats)
    assert sizes[4] == C.sizeof(sbr.Complex)
    assert sizes[5] == sbr.DPATH_DTYPE.itemsize and sizes[6] == sbr.WEDGE_DTYPE.itemsize
    assert sizes[7] == sbr.DPATH_DTYPE.fields["exact_point"][1]
    assert sizes[8] == sbr.DPATH_DTYPE.fields["init_tan_err"][1]
    P, K = sbr.PATH_DTYPE, sbr.CAND_DTYPE
    assert offs == [P.fields["launch_ray"][1], P.fields["tan_err"][1], P.fields["delay_s"][1],
                    P.fields["exact_delay_s"][1], P.fields["init_tan_err"][1],
                    K.fields["tan_err"][1]]
    assert more == [C.sizeof(sbr.Tuning), sbr.Tuning.lookahead_max_paths.offset,
                    sbr.Tuning.ray_order.offset, sbr.Tuning.refine_segments.offset,
                    C.sizeof(sbr.BvhParams), sbr.BvhParams.split_pct.offset, C.sizeof(sbr.Job)]


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2208_10009_amd import sbr
    monkeypatch.setattr(sbr, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(sbr, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        sbr.lib(load_torch=False)


def test_product_package_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2208_10009_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", txt).lower() or f == "scenes.py", f


def test_scene_generators_are_seeded():
    from paper_2208_10009_amd import scenes
    a = scenes.manhattan_config(3)
    b = scenes.manhattan_config(3)
    assert np.array_equal(a["scene"]["xyz"], b["scene"]["xyz"])
    assert np.array_equal(a["rx"], b["rx"])
    assert len(a["scene"]["tri"]) == 770
    assert len(scenes.shoebox_config(0)["scene"]["tri"]) == 12


def test_factorial_table_is_exact_double_double():
    """The library's 1/k! literals (used by its correctly rounded sin/acos) are
    the double-double split of the exact rationals: hi = 1/k! rounded to
    nearest, lo = (1/k! - hi) rounded to nearest."""
    import math
    from fractions import Fraction
    src = open(os.path.join(ROOT, "paper_2208_10009_amd", "csrc", "geom.h")).read()
    body = src[src.index("kInvFact[kFactN] = {"):]
    body = body[:body.index("};")]
    pairs = re.findall(r"\{([^,{}]+),\s*([^,{}]+)\}", body)
    assert len(pairs) == 36
    for k, (hi_s, lo_s) in enumerate(pairs):
        hi = float.fromhex(hi_s.strip()) if "0x" in hi_s else float(hi_s)
        lo = float.fromhex(lo_s.strip()) if "0x" in lo_s else float(lo_s)
        x = Fraction(1, math.factorial(k))
        assert hi == float(x), k
        assert lo == float(x - Fraction(hi)), k
