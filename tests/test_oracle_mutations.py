"""The oracle's pins catch planted mistakes (CPU only).

Each mutant below is one plausible slip in ``oracle/sacx_oracle.c``: a wrong
stencil coefficient or window, a dropped or sign-flipped flux term, a wrong
Runge-Kutta weight or stage input, a boundary-copy or time-step error, a
conservation-sum slip.  The test writes a copy of the source with the
mistake, compiles it with the oracle's own flags, and runs the oracle pin
suites against that build (through ``SACX_ORACLE_LIB``).  Some pin must fail
for every mutant.

Not planted: halving the compression term's coefficient or its indicator s,
which only rescales an HD constant that no outside value fixes (the
constants are "parity unpinned").
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sacx_oracle.c")
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_forms.py", "tests/test_oracle_gravity.py",
        "tests/test_oracle_surrogate.py"]

# (name, text in the source, replacement); each text occurs exactly once
MUTANTS = [
    ("stencil inner weight 8 -> 7",
     "over(paper, 8.0 * (f[i + st] - f[i - st])", "over(paper, 7.0 * (f[i + st] - f[i - st])"),
    ("stencil outer difference sign",
     "- (f[i + 2 * st] - f[i - 2 * st]), h12, inv12h)", "+ (f[i + 2 * st] - f[i - 2 * st]), h12, inv12h)"),
    ("third difference weight 3 -> 2",
     "- 3.0 * (q[i + st] - q[i]);", "- 2.0 * (q[i + st] - q[i]);"),
    ("third-difference window 3 faces -> 1",
     "for (int k = -1; k <= 1; ++k) n = dmax", "for (int k = 0; k <= 0; ++k) n = dmax"),
    ("first-difference window 5 faces -> 3",
     "for (int k = -2; k <= 2; ++k) m = dmax", "for (int k = -1; k <= 1; ++k) m = dmax"),
    ("momentum flux without total pressure",
     "Fx[F_MX][c] = (ux * mx - (bxt * bxt + 2.0 * bxt * bxb)) + ptt[c];",
     "Fx[F_MX][c] = (ux * mx - (bxt * bxt + 2.0 * bxt * bxb));"),
    ("energy flux B.v term sign",
     "Fx[F_E][c] = ((ux * eflux - bxt * bv_t)", "Fx[F_E][c] = ((ux * eflux + bxt * bv_t)"),
    ("induction y flux with swapped velocity",
     "Fy[F_BX][c] = uy * bxT[c] - byT[c] * ux;", "Fy[F_BX][c] = ux * bxT[c] - byT[c] * uy;"),
    ("cross momentum flux loses B_x B_y",
     "Fy[F_MX][c] = uy * mx - (byt * bxt + byt * bxb + byb * bxt);",
     "Fy[F_MX][c] = uy * mx - (byt * bxb + byb * bxt);"),
    ("kinetic pressure with full v^2",
     "double kin = 0.5 * (mx * ux + my * uy);          /* rho v^2 / 2 */",
     "double kin = (mx * ux + my * uy);          /* rho v^2 / 2 */"),
    ("HD coefficient drops c_max",
     "double nu = P->c2[cls[k]] * dx * cmax * R + P->cshk[cls[k]] * dx * dx * sf;",
     "double nu = P->c2[cls[k]] * dx * R + P->cshk[cls[k]] * dx * dx * sf;"),
    ("HD energy flux loses the e.m.f. term",
     "Hx[F_E][c] = (Gx[Q_EPS][c] + (vxf * txx + vyf * txy)) + byf * ez;",
     "Hx[F_E][c] = (Gx[Q_EPS][c] + (vxf * txx + vyf * txy));"),
    ("hyper-resistive y-face e.m.f. sign",
     "Hy[F_BX][c] = -ez;", "Hy[F_BX][c] = ez;"),
    ("cross stress average over 2 faces",
     "a4_vx = ((Gy[Q_VX][c - nxe] + Gy[Q_VX][c]) + (Gy[Q_VX][c + 1 - nxe] + Gy[Q_VX][c + 1])) / 4.0;",
     "a4_vx = (Gy[Q_VX][c - nxe] + Gy[Q_VX][c]) / 2.0;"),
    ("HD divergence sign",
     "K[k][c] = K[k][c] + hd;", "K[k][c] = K[k][c] - hd;"),
    ("RK4 weight of K2 is 1",
     "u[q] = u[q] + dt6 * (((k1[q] + 2.0 * k2[q]) + 2.0 * k3[q]) + k4[q]);",
     "u[q] = u[q] + dt6 * (((k1[q] + k2[q]) + 2.0 * k3[q]) + k4[q]);"),
    ("RK4 third stage input at dt/2",
     "const double c = stage == 3 ? dt : 0.5 * dt;", "const double c = 0.5 * dt;"),
    ("low-storage combine weight 1/3 -> 1/2",
     "const double dt6 = dt / 6.0, third = 1.0 / 3.0;\n    for (int k = 0; k < NF; ++k) {\n        double *u = d->U.f[k];\n        const double *s = d->S.f[k]",
     "const double dt6 = dt / 6.0, third = 1.0 / 2.0;\n    for (int k = 0; k < NF; ++k) {\n        double *u = d->U.f[k];\n        const double *s = d->S.f[k]"),
    ("low-storage accumulator without dt K2",
     "acc[q] = (u[q] + u[q]) + ((s[q] - u[q]) + dt * kk[q]);", "acc[q] = (u[q] + u[q]) + (s[q] - u[q]);"),
    ("open x- boundary copies the second cell",
     "int s = bc[0] == ORC_PERIODIC ? imod(i, nx) : iclamp(i, nx);",
     "int s = bc[0] == ORC_PERIODIC ? imod(i, nx) : 1;"),
    ("periodic y+ ghosts from the wrong image",
     "int s = bc[3] == ORC_PERIODIC ? imod(j, ny) : iclamp(j, ny);",
     "int s = bc[3] == ORC_PERIODIC ? imod(j - 1, ny) : iclamp(j, ny);"),
    ("CFL step from the larger of the two",
     "if (ax && ay) h = dmin(dx / c[0], dy / c[1]);", "if (ax && ay) h = dmax(dx / c[0], dy / c[1]);"),
    ("fast speed without the field",
     "double cf = sqrt(over(pf, cfg->gamma * pk + (bx * bx + by * by), r, ir));",
     "double cf = sqrt(over(pf, cfg->gamma * pk, r, ir));"),
    ("gravity energy source sign",
     "K[F_E][c] = K[F_E][c] + rt * (P->g[0] * vx[c] + P->g[1] * vy[c]);",
     "K[F_E][c] = K[F_E][c] - rt * (P->g[0] * vx[c] + P->g[1] * vy[c]);"),
    ("background energy term sign",
     "K[F_E][c] = K[F_E][c] + (bb - ptb[c] * (dxvx + dyvy));",
     "K[F_E][c] = K[F_E][c] + (bb + ptb[c] * (dxvx + dyvy));"),
    ("sums use dx dx",
     "sums[k] = psum(f[k], (size_t)cfg->nx * cfg->ny) * (dx * dy);",
     "sums[k] = psum(f[k], (size_t)cfg->nx * cfg->ny) * (dx * dx);"),
    ("sums drop the last row",
     "sums[k] = psum(f[k], (size_t)cfg->nx * cfg->ny)", "sums[k] = psum(f[k], (size_t)cfg->nx * (cfg->ny - 1))"),
    ("compression face value from one cell",
     "double sf = dmax(s[c], s[c + 1]);", "double sf = s[c];"),
]


def _mutant_source(text, new):
    src = open(SRC).read()
    assert src.count(text) == 1, text
    return src.replace(text, new)


@pytest.mark.parametrize("name,text,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_text_is_present(name, text, new):
    """Every planted mistake still names one place in the current source."""
    _mutant_source(text, new)


def _run_pins(workdir, idx, name, text, new):
    d = os.path.join(workdir, f"m{idx}")
    os.makedirs(d, exist_ok=True)
    c = os.path.join(d, "sacx_oracle.c")
    with open(c, "w") as fh:
        fh.write(_mutant_source(text, new))
    lib = os.path.join(d, "liborc.so")
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-o", lib, c, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        return name, "compile", r.stderr[-500:]
    env = dict(os.environ, SACX_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        "-k", "not mutant", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode, r.stdout[-300:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_pins_catch_every_mutant(tmp_path):
    workers = max(1, min(4, (os.cpu_count() or 2) // 2))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda a: _run_pins(str(tmp_path), a[0], *a[1]), enumerate(MUTANTS)))
    survivors = [(n, rc, out) for n, rc, out in results if rc == 0]
    broken = [(n, out) for n, rc, out in results if rc == "compile"]
    assert not broken, broken
    assert not survivors, survivors
