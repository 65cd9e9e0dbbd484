"""C ABI checks that need no GPU: exported symbols, struct layout, host-only
argument validation and workspace arithmetic."""

import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sacx.h")
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))


@pytest.fixture(scope="module")
def sx():
    from paper_1710_06423_amd import sacx
    if not os.path.exists(sacx.LIB_PATH):
        from paper_1710_06423_amd import build
        build.build()
    sacx.load_library()
    return sacx


def declared_functions():
    """Every function declared in any header under include/."""
    names = set()
    for h in HEADERS:
        names |= set(re.findall(r"^\s*(?:int|const char \*)\s*(sacx3?_\w+)\s*\(", open(h).read(), re.M))
    return sorted(names)


def test_every_declared_symbol_is_exported(sx):
    from paper_1710_06423_amd import sacx3
    lib = sx.load_library()
    names = declared_functions()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(sx.EXPORTED) | set(sacx3.EXPORTED3)


def test_abi_version_matches_header(sx):
    m = re.search(r"#define SACX_ABI_VERSION (\d+)", open(HEADER).read())
    assert sx.load_library().sacx_abi_version() == int(m.group(1))


def test_struct_layout_matches_header(sx, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "sacx.h"
int main(void) {
  printf("%zu %zu %zu %zu\\n", sizeof(sacx_grid), sizeof(sacx_params), sizeof(sacx_diag), sizeof(sacx_profile));
  printf("%zu %zu %zu\\n", offsetof(sacx_grid, precision), offsetof(sacx_params, c2), offsetof(sacx_diag, steps));
  printf("%zu %zu\\n", offsetof(sacx_profile, n_stage), offsetof(sacx_diag, nonphys));
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(sacx_surrogate), offsetof(sacx_surrogate, refresh_every),
         offsetof(sacx_surrogate, bound), sizeof(sacx_hd_stats), sizeof(sacx_cnn_sizes),
         offsetof(sacx_profile, ms_surrogate));
  printf("%d %d\\n", SACX_CNN_NPARAM, SACX_CNN_PACKED_BYTES);
  printf("%zu\\n", offsetof(sacx_params, g));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), "-o", str(exe), str(src)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals[:4] == [ctypes.sizeof(sx.Grid), ctypes.sizeof(sx.Params), ctypes.sizeof(sx.Diag),
                        ctypes.sizeof(sx.Profile)]
    assert vals[4] == sx.Grid.precision.offset
    assert vals[5] == sx.Params.c2.offset
    assert vals[6] == sx.Diag.steps.offset
    assert vals[7] == sx.Profile.n_stage.offset
    assert vals[8] == sx.Diag.nonphys.offset
    assert vals[9:15] == [ctypes.sizeof(sx.Surrogate), sx.Surrogate.refresh_every.offset, sx.Surrogate.bound.offset,
                          ctypes.sizeof(sx.HdStats), ctypes.sizeof(sx.CnnSizes), sx.Profile.ms_surrogate.offset]
    assert vals[15:17] == [sx.CNN_NPARAM, sx.CNN_PACKED_BYTES]
    assert vals[17] == sx.Params.g.offset


def test_strerror_and_codes(sx):
    lib = sx.load_library()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.sacx_strerror(code)
    assert b"unknown" in lib.sacx_strerror(-99)


def test_workspace_size_arithmetic(sx):
    p = sx.make_params(5 / 3)
    a = sx.workspace_size(sx.make_grid(1000, 1000, 0, 1, 0, 1), p)
    b = sx.workspace_size(sx.make_grid(2000, 2000, 0, 1, 0, 1), p)
    c = sx.workspace_size(sx.make_grid(1000, 1000, 0, 1, 0, 1, precision=sx.FP32), p)
    d = sx.workspace_size(sx.make_grid(1000, 1000, 0, 1, 0, 1, background_on=True), p)
    assert a % 256 == 0 and b > 3.9 * a * 0.9 and c < a and d > a
    # 4 state copies x 6 fields x (ny + 6) rows x pitch x 8 bytes dominate
    assert a >= 4 * 6 * 1006 * 1035 * 8


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=-3), dict(nx=1, ny=1), dict(x1=0.0), dict(precision=7), dict(background_on=2),
    dict(nx=(1 << 24) + 1, ny=2), dict(nx=2, ny=(1 << 24) + 1), dict(nx=1 << 17, ny=(1 << 17) + 1),
])
def test_invalid_grids_rejected(sx, bad):
    kw = dict(nx=16, ny=16, x0=0.0, x1=1.0, y0=0.0, y1=1.0, precision=0, background_on=0)
    kw.update(bad)
    g = sx.Grid(kw["nx"], kw["ny"], kw["x0"], kw["x1"], kw["y0"], kw["y1"], kw["precision"], kw["background_on"])
    with pytest.raises(sx.SacxError) as e:
        sx.workspace_size(g, sx.make_params(5 / 3))
    assert e.value.code == sx.EINVAL


@pytest.mark.parametrize("nx, ny", [(1 << 24, 2), (2, 1 << 24), (1 << 17, 1 << 17)])
def test_largest_grids_accepted(sx, nx, ny):
    """The size limits themselves (a side of 2^24 cells, 2^34 cells in all)
    are accepted, and the workspace size is computed without overflow."""
    g = sx.make_grid(nx, ny, 0, 1, 0, 1)
    b = sx.workspace_size(g, sx.make_params(5 / 3))
    assert b >= 4 * 6 * (nx + 6) * (ny + 6) * 8


@pytest.mark.parametrize("bad", [dict(gamma=1.0), dict(cfl=0.0), dict(c2=(-1, 0, 0, 0)), dict(cshk=(0, float("nan"), 0, 0)),
                                 dict(g=(float("inf"), 0.0)), dict(g=(0.0, float("nan")))])
def test_invalid_params_rejected(sx, bad):
    kw = dict(gamma=5 / 3, cfl=0.3, c2=sx.DEFAULT_C2, cshk=sx.DEFAULT_CSHK, g=(0.0, 0.0))
    kw.update(bad)
    p = sx.make_params(kw["gamma"], kw["cfl"], True, True, kw["c2"], kw["cshk"], kw["g"])
    with pytest.raises(sx.SacxError) as e:
        sx.workspace_size(sx.make_grid(8, 8, 0, 1, 0, 1), p)
    assert e.value.code == sx.EINVAL


def test_create_rejects_bad_workspace_without_touching_the_device(sx):
    lib = sx.load_library()
    g, p = sx.make_grid(8, 8, 0, 1, 0, 1), sx.make_params(5 / 3)
    out = ctypes.c_void_p()
    assert lib.sacx_create(ctypes.byref(g), ctypes.byref(p), None, 1 << 20, None, ctypes.byref(out)) == sx.EINVAL
    assert b"NULL" in lib.sacx_last_error()
    assert lib.sacx_create(ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(256 * 7 + 8), 1 << 20, None,
                           ctypes.byref(out)) == sx.EINVAL
    assert lib.sacx_create(ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(1 << 20), 1024, None,
                           ctypes.byref(out)) == sx.ENOSPC
    assert lib.sacx_destroy(None) == 0


def test_product_path_does_not_reference_the_oracle():
    """The HIP library and its binding share no code with the oracle."""
    pkg = os.path.join(ROOT, "paper_1710_06423_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "sacx_oracle" not in text, fn


def test_stage_code_hash_ignores_comments_and_layout():
    """The hash that ties recorded traffic counters to the stage kernel's code
    changes with the code, not with its comments or layout."""
    from paper_1710_06423_amd.profiling import code_text
    a = 'x = a * b; // one\n/* two\n three */ y  =\n  "// kept" ;'
    b = 'x = a * b;\ny = "// kept";'
    assert code_text(a) == 'x = a * b; y = "// kept" ;'
    assert code_text(a).replace(" ", "") == code_text(b).replace(" ", "")
    assert code_text("x = a * b;") != code_text("x = a + b;")
    assert code_text("s = 'a'; // c") == "s = 'a';"


def test_setters_reject_null_context(sx):
    """Host-side argument checks of the launch and tile-kind setters (no
    device work): a NULL context is EINVAL."""
    lib = sx.load_library()
    assert lib.sacx_set_column_split(None, 1) == sx.EINVAL
    assert lib.sacx_set_launch(None, 128, 64) == sx.EINVAL
    assert lib.sacx_set_boundaries(None, None) == sx.EINVAL


def test_stage_calls_reject_null_context(sx):
    """Host-side argument checks of the decomposed-stepping calls."""
    lib = sx.load_library()
    c = (ctypes.c_double * 2)(1.0, 1.0)
    assert lib.sacx_fill_boundaries(None, 0) == sx.EINVAL
    assert lib.sacx_stage(None, c, 0, None) == sx.EINVAL
    assert lib.sacx_wave_speeds(None, c) == sx.EINVAL
    assert lib.sacx_wave_speeds_max(None, c) == sx.EINVAL
    assert lib.sacx_set_spacing(None, 0.1, 0.1) == sx.EINVAL
    assert lib.sacx_init_problem(None, 0, None, 0, 0.0) == sx.EINVAL
    n = ctypes.c_size_t(0)
    assert lib.sacx_domain_buffer_size(0, 1, None, ctypes.byref(n)) == sx.EINVAL
    assert lib.sacx_domain_buffer_size(1, 1, None, ctypes.byref(n)) == sx.EINVAL
    assert lib.sacx_domain_advance(None, 1) == sx.EINVAL
    assert lib.sacx_domain_destroy(None) == 0


def test_missing_library_fails_loudly(tmp_path):
    """Without the built HIP library the binding raises; nothing falls back
    to another implementation."""
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_1710_06423_amd.sacx as sx\n"
        "sx.LIB_PATH = %r\n"
        "sx._lib = None\n"
        "try:\n"
        "    sx.load_library()\n"
        "except RuntimeError as e:\n"
        "    print('raised:', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(1)\n"
    ) % (ROOT, str(tmp_path / "libsacx.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (r.stdout, r.stderr)
    assert "missing" in r.stdout


# ------------------------------------------------------------ 3-D contexts

def test_3d_struct_layout_matches_header(sx, tmp_path):
    from paper_1710_06423_amd import sacx3
    src = tmp_path / "layout3.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "sacx3.h"
int main(void) {
  printf("%zu %zu %zu\\n", sizeof(sacx3_grid), sizeof(sacx3_params), sizeof(sacx3_diag));
  printf("%zu %zu %zu %zu\\n", offsetof(sacx3_grid, x0), offsetof(sacx3_params, c2), offsetof(sacx3_diag, sums),
         offsetof(sacx3_diag, nonphys));
  return 0;
}
""")
    exe = tmp_path / "layout3"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), "-o", str(exe), str(src)], check=True)
    got = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    want = [ctypes.sizeof(sacx3.Grid3), ctypes.sizeof(sacx3.Params3), ctypes.sizeof(sacx3.Diag3),
            sacx3.Grid3.x0.offset, sacx3.Params3.c2.offset, sacx3.Diag3.sums.offset, sacx3.Diag3.nonphys.offset]
    assert [int(v) for v in got] == want


def test_3d_workspace_size_arithmetic(sx):
    """Four state arrays of 8 fields, and with hyper-diffusion 21 face arrays,
    each (nz + 6) planes of (ny + 6) rows of a 256-byte-rounded pitch."""
    from paper_1710_06423_amd import sacx3
    g = sacx3.make_grid3(37, 21, 19, (0, 1, 0, 1, 0, 1))
    on = sacx3.workspace_size3(g, sacx3.make_params3(5 / 3))
    off = sacx3.workspace_size3(g, sacx3.make_params3(5 / 3, hd_on=False))
    pitch = ((32 + 37 + 3 + 31) // 32) * 32
    field = ((pitch * 27 * 25 + 31) // 32) * 32 * 8
    assert on - off == 21 * field
    assert off >= 32 * field and off < 32 * field + (1 << 17)


@pytest.mark.parametrize("bad", [dict(nx=0), dict(nz=-1), dict(nx=1, ny=1, nz=1), dict(x1=0.0),
                                 dict(nx=1200, ny=1200, nz=1200)])
def test_3d_invalid_grids_rejected(sx, bad):
    from paper_1710_06423_amd import sacx3
    kw = dict(nx=8, ny=8, nz=8, x1=1.0)
    kw.update(bad)
    g = sacx3.make_grid3(kw["nx"], kw["ny"], kw["nz"], (0.0, kw["x1"], 0.0, 1.0, 0.0, 1.0))
    with pytest.raises(sx.SacxError) as e:
        sacx3.workspace_size3(g, sacx3.make_params3(5 / 3))
    assert e.value.code in (sx.EINVAL, sx.EUNSUP)


def test_3d_calls_reject_null_context(sx):
    from paper_1710_06423_amd import sacx3
    lib = sacx3.load_library()
    bc = (ctypes.c_int32 * 6)(*([0] * 6))
    assert lib.sacx3_set_boundaries(None, bc) == sx.EINVAL
    assert lib.sacx3_advance(None, 1, 0.0, None, None) == sx.EINVAL
    assert lib.sacx3_read_fields(None, None, 1, 1, 1) == sx.EINVAL
    assert lib.sacx3_diagnostics(None, None) == sx.EINVAL
    assert lib.sacx3_set_launch(None, 4) == sx.EINVAL
    assert lib.sacx3_destroy(None) == sx.OK


def test_3d_create_rejects_bad_workspace_without_touching_the_device(sx):
    from paper_1710_06423_amd import sacx3
    lib = sacx3.load_library()
    g = sacx3.make_grid3(8, 8, 8, (0, 1, 0, 1, 0, 1))
    p = sacx3.make_params3(5 / 3)
    need = sacx3.workspace_size3(g, p)
    out = ctypes.c_void_p(None)
    assert lib.sacx3_create(ctypes.byref(g), ctypes.byref(p), None, need, None, ctypes.byref(out)) == sx.EINVAL
    assert lib.sacx3_create(ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(256 * 7 + 8), need, None,
                            ctypes.byref(out)) == sx.EINVAL
    assert lib.sacx3_create(ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(256 * 7), need - 1, None,
                            ctypes.byref(out)) == sx.ENOSPC
    assert not out.value
