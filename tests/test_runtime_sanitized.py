"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only).  The runtime translation unit is rebuilt with its host side
instrumented and linked with the other (unchanged) objects of the library; a
C driver then runs every path that needs no GPU: version and error strings,
workspace arithmetic for many grids (valid and invalid), creation with bad
workspaces, batch and network buffer sizes, and every entry point with a
NULL context."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"

DRIVER = r"""
#include <stdio.h>
#include <string.h>
#include "sacx.h"

#define EXPECT(cond) do { if (!(cond)) { printf("FAILED line %d: %s\n", __LINE__, #cond); return 1; } } while (0)

int main(void) {
    EXPECT(sacx_abi_version() == SACX_ABI_VERSION);
    for (int c = -8; c <= 1; ++c) EXPECT(sacx_strerror(c) != NULL && strlen(sacx_strerror(c)) > 0);
    EXPECT(sacx_last_error() != NULL);

    sacx_params p;
    memset(&p, 0, sizeof(p));
    p.gamma = 5.0 / 3.0; p.cfl = 0.3; p.hd_on = 1; p.hd_cross_on = 1;
    for (int m = 0; m < 4; ++m) { p.c2[m] = 0.02; p.cshk[m] = 0.5; }
    const int dims[][2] = {{1, 1}, {1, 7}, {2, 2}, {3, 5}, {7, 1}, {129, 65}, {1000, 1}, {1, 1000}, {8000, 8000}};
    size_t prev = 0;
    for (unsigned k = 0; k < sizeof(dims) / sizeof(dims[0]); ++k)
        for (int prec = 0; prec < 2; ++prec)
            for (int bg = 0; bg < 2; ++bg) {
                sacx_grid g = {dims[k][0], dims[k][1], 0.0, 1.0, 0.0, 1.0, prec, bg};
                size_t bytes = 0;
                int rc = sacx_workspace_size(&g, &p, &bytes);
                if (dims[k][0] == 1 && dims[k][1] == 1) { EXPECT(rc == SACX_EINVAL); continue; }
                EXPECT(rc == SACX_OK && bytes > 0 && bytes % 256 == 0);
                prev = bytes;
            }
    EXPECT(prev > 0);
    /* invalid grids and parameters */
    sacx_grid bad = {16, 16, 0.0, 0.0, 0.0, 1.0, SACX_FP64, 0};
    size_t b = 0;
    EXPECT(sacx_workspace_size(&bad, &p, &b) == SACX_EINVAL);
    EXPECT(sacx_workspace_size(NULL, &p, &b) == SACX_EINVAL);
    sacx_grid good = {16, 16, 0.0, 1.0, 0.0, 1.0, SACX_FP64, 0};
    sacx_params q = p;
    q.gamma = 1.0;
    EXPECT(sacx_workspace_size(&good, &q, &b) == SACX_EINVAL);
    q = p;
    q.g[1] = 1.0 / 0.0;
    EXPECT(sacx_workspace_size(&good, &q, &b) == SACX_EINVAL);
    /* creation that fails before touching the device */
    sacx_ctx *ctx = NULL;
    EXPECT(sacx_create(&good, &p, NULL, 1 << 20, NULL, &ctx) == SACX_EINVAL);
    EXPECT(sacx_create(&good, &p, (void *)(uintptr_t)(256 * 7 + 8), 1 << 20, NULL, &ctx) == SACX_EINVAL);
    EXPECT(sacx_create(&good, &p, (void *)(uintptr_t)(1 << 20), 1024, NULL, &ctx) == SACX_ENOSPC);
    EXPECT(sacx_destroy(NULL) == SACX_OK);
    /* batch and network sizes */
    sacx_grid gs[3] = {{96, 64, 0, 1, 0, 1, SACX_FP32, 0}, {400, 1, 0, 1, 0, 0.0025, SACX_FP32, 0},
                       {80, 80, 0, 1, 0, 1, SACX_FP32, 0}};
    sacx_params ps[3] = {p, p, p};
    EXPECT(sacx_batch_workspace_size(3, gs, ps, &b) == SACX_OK && b > 0);
    EXPECT(sacx_batch_workspace_size(0, gs, ps, &b) == SACX_EINVAL);
    sacx_cnn_sizes cs;
    EXPECT(sacx_cnn_buffer_sizes(2, 48, 64, &cs) == SACX_OK && cs.input_bytes > 0 && cs.work_bytes > 0);
    EXPECT(sacx_cnn_buffer_sizes(2, 64, 48, &cs) != SACX_OK);   /* width not a multiple of 32 */
    EXPECT(sacx_cnn_buffer_sizes(0, 64, 64, &cs) != SACX_OK);
    /* every context entry point with a NULL context */
    int32_t bc[4] = {0, 0, 0, 0};
    double c[2] = {1.0, 1.0};
    int32_t t = 0, r = 0, st = 0;
    EXPECT(sacx_set_boundaries(NULL, bc) == SACX_EINVAL);
    EXPECT(sacx_set_launch(NULL, 128, 64) == SACX_EINVAL);
    EXPECT(sacx_get_launch(NULL, &t, &r) == SACX_EINVAL);
    EXPECT(sacx_set_column_split(NULL, 1) == SACX_EINVAL);
    EXPECT(sacx_advance(NULL, 1, 0.0, NULL, NULL) == SACX_EINVAL);
    EXPECT(sacx_read_fields(NULL, NULL, 16, 0x3f, SACX_FP64) == SACX_EINVAL);
    EXPECT(sacx_init_state(NULL, NULL, NULL, 16, SACX_FP64, 0.0) == SACX_EINVAL);
    EXPECT(sacx_init_problem(NULL, SACX_PROBLEM_ORSZAG_TANG, NULL, 0, 0.0) == SACX_EINVAL);
    EXPECT(sacx_halo_buffer_size(NULL, 0, &b) == SACX_EINVAL);
    EXPECT(sacx_halo_pack(NULL, 0, NULL) == SACX_EINVAL);
    EXPECT(sacx_halo_unpack(NULL, 0, NULL) == SACX_EINVAL);
    EXPECT(sacx_fill_boundaries(NULL, 0) == SACX_EINVAL);
    EXPECT(sacx_stage(NULL, c, 0, &st) == SACX_EINVAL);
    EXPECT(sacx_wave_speeds(NULL, c) == SACX_EINVAL);
    EXPECT(sacx_wave_speeds_max(NULL, c) == SACX_EINVAL);
    EXPECT(sacx_set_spacing(NULL, 0.1, 0.1) == SACX_EINVAL);
    EXPECT(sacx_profile_enable(NULL, 1) == SACX_EINVAL);
    EXPECT(sacx_hd_clear_surrogate(NULL) == SACX_EINVAL);
    EXPECT(sacx_batch_destroy(NULL) == SACX_OK);
    printf("ok\n");
    return 0;
}
"""


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="no ROCm toolchain")
def test_runtime_host_code_under_sanitizers(tmp_path):
    from paper_1710_06423_amd import build
    objs = [os.path.join(build.BUILD, os.path.splitext(s)[0] + ".o") for s in build.SOURCES if s != "sacx_runtime.hip"]
    if not all(os.path.exists(o) for o in objs):
        build.build()
    rt = tmp_path / "sacx_runtime_asan.o"
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={build.ARCH}", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-I", build.INCLUDE, "-I", build.CSRC, "-ffp-contract=off", *san,
           "-c", os.path.join(build.CSRC, "sacx_runtime.hip"), "-o", str(rt)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    lib = tmp_path / "libsacx_asan.so"
    # the sanitizer runtime comes with the driver executable
    r = subprocess.run([HIPCC, "-shared", "-fPIC", f"--offload-arch={build.ARCH}", "-o", str(lib), *objs, str(rt)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    drv = tmp_path / "drv.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "drv"
    r = subprocess.run([CLANG, "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", build.INCLUDE,
                        "-o", str(exe), str(drv), str(lib), f"-Wl,-rpath,{tmp_path}"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:])
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.strip().endswith("ok")
