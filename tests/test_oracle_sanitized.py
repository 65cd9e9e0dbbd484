"""The oracle's C source under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): a small C driver compiled together with the oracle runs every
entry point on grids from smaller than the stencil to a few tiles, with
periodic, open and mixed boundaries, a background with gravity, the cross
terms on and off, in both arithmetic forms.  Any out-of-bounds access, leak, use after free or
undefined operation aborts the driver."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sacx_oracle.c")

DRIVER = r"""
#include <stdio.h>
#include <math.h>
#include "sacx_oracle.c"

static double *mk(size_t n) { double *p = calloc(n, sizeof(double)); if (!p) abort(); return p; }

/* a smooth positive state: rho~ > 0 (no background) or small (background) */
static void fill(int nx, int ny, double *f[NF], double *bg[NB], int background, int seed) {
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t e = (size_t)j * nx + i;
            double x = (i + 0.5) / nx, y = (j + 0.5) / ny, s = 0.1 * seed;
            double r = 1.0 + 0.2 * sin(6.283 * (x + s)) * cos(6.283 * y);
            double vx = 0.3 * sin(6.283 * y + s), vy = 0.2 * cos(6.283 * x);
            double bx = 0.25 * sin(6.283 * (y + x)), by = 0.15 * cos(12.566 * x);
            double p = 1.0 + 0.1 * cos(6.283 * (x - y));
            if (background) {
                bg[B_RHO][e] = 1.0 + 0.5 * y; bg[B_E][e] = 2.0 + 0.5 * y; bg[B_BX][e] = 0.1; bg[B_BY][e] = 0.2;
                f[F_RHO][e] = 0.01 * sin(6.283 * x); f[F_MX][e] = 0.01 * vx; f[F_MY][e] = 0.01 * vy;
                f[F_E][e] = 0.01 * cos(6.283 * y); f[F_BX][e] = 0.001 * bx; f[F_BY][e] = 0.001 * by;
            } else {
                f[F_RHO][e] = r; f[F_MX][e] = r * vx; f[F_MY][e] = r * vy; f[F_BX][e] = bx; f[F_BY][e] = by;
                f[F_E][e] = p / (5.0 / 3.0 - 1.0) + 0.5 * r * (vx * vx + vy * vy) + 0.5 * (bx * bx + by * by);
            }
        }
}

static int run(int nx, int ny, int b0, int b2, int background, int cross, int seed, int form) {
    orc_cfg c;
    memset(&c, 0, sizeof(c));
    c.nx = nx; c.ny = ny; c.x0 = 0; c.x1 = 1; c.y0 = 0; c.y1 = 1;
    c.gamma = 5.0 / 3.0; c.cfl = 0.3; c.hd_on = 1; c.hd_cross_on = cross;
    for (int m = 0; m < 4; ++m) { c.c2[m] = 0.02; c.cshk[m] = 0.5; }
    c.bc[0] = c.bc[1] = b0; c.bc[2] = c.bc[3] = b2;
    c.background_on = background;
    c.form = form;
    if (background) { c.g[0] = 0.1; c.g[1] = -0.5; }
    size_t n = (size_t)nx * ny;
    double *f[NF], *K[NF], *bg[NB];
    for (int k = 0; k < NF; ++k) { f[k] = mk(n); K[k] = mk(n); }
    for (int k = 0; k < NB; ++k) bg[k] = mk(n);
    fill(nx, ny, f, bg, background, seed);
    double info[4], t = 0, ws[4], sums[NF];
    int done = 0, rc;
    if ((rc = orc_wavespeed(&c, f, background ? bg : NULL, ws))) return 100 + rc;
    if ((rc = orc_rhs(&c, f, background ? bg : NULL, ws[2], K))) return 200 + rc;
    if ((rc = orc_advance(&c, f, background ? bg : NULL, 3, 0.0, &t, &done, info)) || done != 3) return 300 + rc;
    if ((rc = orc_sums(&c, f, sums))) return 400 + rc;
    if (nx >= 2 && ny >= 2) {
        double *R = mk(10 * n), *D1 = mk(10 * n);
        if ((rc = orc_hd_face_fields(&c, f, background ? bg : NULL, R, D1))) return 500 + rc;
        if (!background && b0 == 0 && b2 == 0) {
            float *rn = malloc(10 * n * sizeof(float));
            if (!rn) abort();
            for (size_t i = 0; i < 10 * n; ++i) rn[i] = (i % 3) ? (float)R[i] : -1.0f;
            int mask[64 * 64], nfall = 0;
            double eu, ea;
            if ((rc = orc_hd_check(&c, f, rn, 0.05, 8, 1, mask, &nfall, &eu, &ea))) return 600 + rc;
            if ((rc = orc_rhs_ext(&c, f, ws[2], K, rn))) return 700 + rc;
            if ((rc = orc_advance_ext(&c, f, 2, 0.0, &t, &done, info, rn))) return 800 + rc;
            free(rn);
        }
        free(R); free(D1);
    }
    if (nx >= 25 && ny >= 25) {
        double *out[NF];
        for (int k = 0; k < NF; ++k) out[k] = mk((size_t)(nx - 24) * (ny - 24));
        if ((rc = orc_step_patch(&c, nx, ny, f, background ? bg : NULL, 1e-4, ws[2], out))) return 900 + rc;
        for (int k = 0; k < NF; ++k) free(out[k]);
    }
    for (int k = 0; k < NF; ++k) { free(f[k]); free(K[k]); }
    for (int k = 0; k < NB; ++k) free(bg[k]);
    return 0;
}

int main(void) {
    /* (nx, ny, x boundaries, y boundaries, background, cross terms) */
    const int cases[][6] = {
        {2, 2, 0, 0, 0, 1}, {3, 3, 0, 0, 0, 1}, {2, 5, 0, 0, 0, 0}, {7, 4, 0, 0, 0, 1},
        {6, 5, 1, 1, 0, 1}, {40, 1, 1, 0, 0, 1}, {1, 33, 0, 1, 0, 1}, {30, 26, 0, 0, 0, 1},
        {27, 31, 1, 0, 0, 0}, {26, 28, 0, 1, 1, 1}, {29, 25, 1, 1, 1, 1},
    };
    for (int form = ORC_FORM_PAPER; form <= ORC_FORM_LOWSTORE; ++form)
        for (size_t i = 0; i < sizeof(cases) / sizeof(cases[0]); ++i) {
            const int *q = cases[i];
            int rc = run(q[0], q[1], q[2], q[3], q[4], q[5], (int)i, form);
            printf("form %d case %dx%d bc %d/%d bg %d cross %d: %d\n", form, q[0], q[1], q[2], q[3], q[4], q[5], rc);
            if (rc) return 1;
        }
    double line[16], out[16], R[16];
    for (int i = 0; i < 16; ++i) line[i] = sin(0.4 * i);
    if (orc_deriv_line(16, line, 0.1, out) || orc_hd_ratio_line(16, line, R)) return 1;
    if (orc_deriv_line(1, line, 0.1, out) || orc_hd_ratio_line(2, line, R)) return 1;
    printf("ok\n");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_address_and_undefined_behavior_sanitizers(tmp_path):
    drv = tmp_path / "drv.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "drv"
    cmd = ["gcc", "-std=gnu11", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wno-unknown-pragmas",
           "-I", os.path.dirname(SRC), "-o", str(exe), str(drv), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:])
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.strip().endswith("ok")
