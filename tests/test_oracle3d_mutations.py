"""The 3-D oracle's pins catch planted mistakes (CPU only).

Each mutant is one plausible slip in ``oracle/sacx_oracle3d.c``: a dropped
or sign-flipped term of a z flux or of a cross term, a wrong stride or
component slot, a missing direction in a sum, a boundary-copy, time-step or
conservation-sum error.  The test compiles a copy of the source with the
mistake and runs the 3-D pin suite against that build (through
``SACX_ORACLE3D_LIB``); some pin must fail for every mutant.
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sacx_oracle3d.c")
PINS = ["tests/test_oracle3d_pins.py"]

MUTANTS = [
    ("z momentum flux without total pressure",
     "F[2][F_MZ][c] = (uz * mz - bz * bz) + pt;", "F[2][F_MZ][c] = (uz * mz - bz * bz);"),
    ("z induction flux of B_x sign",
     "F[2][F_BX][c] = uz * bx - bz * ux;", "F[2][F_BX][c] = uz * bx + bz * ux;"),
    ("x flux of m_z loses B_x B_z",
     "F[0][F_MZ][c] = ux * mz - bx * bz;", "F[0][F_MZ][c] = ux * mz;"),
    ("kinetic energy without its z part",
     "double kin = 0.5 * ((mx * ux + my * uy) + mz * uz);\n                double b2 = (bx * bx + by * by) + bz * bz;\n"
     "                double pk = gm1 * ((et - kin) - 0.5 * b2);\n                double pt",
     "double kin = 0.5 * (mx * ux + my * uy);\n                double b2 = (bx * bx + by * by) + bz * bz;\n"
     "                double pk = gm1 * ((et - kin) - 0.5 * b2);\n                double pt"),
    ("z difference with the y stride",
     "double e = d4(pf, F[2][f], c, st[2], h12[2], i12[2]);", "double e = d4(pf, F[2][f], c, st[1], h12[2], i12[2]);"),
    ("ideal right-hand side drops z",
     "K[f][c] = -((a + b) + e);", "K[f][c] = -(a + b);"),
    ("compression without dv_z",
     "+\n                            over(pf, v[2][c + st[2]] - v[2][c - st[2]], h2[2], i2[2]);", "+ 0.0;"),
    ("cross mean with the face's own stride",
     "a4v[k] = ((gv[c - sk] + gv[c]) + (gv[c + sd - sk] + gv[c + sd])) / 4.0;",
     "a4v[k] = ((gv[c - sd] + gv[c]) + (gv[c + sd - sk] + gv[c + sd])) / 4.0;"),
    ("cross e.m.f. from the wrong field slot",
     "*gb = Gf[k][bslot(k, d)];", "*gb = Gf[k][bslot(d, k)];"),
    ("off-diagonal stress from the normal velocity",
     "tau[k] = 0.5 * rf * (Gf[d][Q_V + k][c] + a4v[k]);", "tau[k] = 0.5 * rf * (Gf[d][Q_V + d][c] + a4v[k]);"),
    ("energy flux work misses a component",
     "double work = (vf[d] * tau[d] + vf[o1] * tau[o1]) + vf[o2] * tau[o2];",
     "double work = vf[d] * tau[d] + vf[o1] * tau[o1];"),
    ("magnetic energy flux sign",
     "double mag = bf[o1] * hb[o1] + bf[o2] * hb[o2];", "double mag = bf[o1] * hb[o1] - bf[o2] * hb[o2];"),
    ("hyper-diffusive divergence drops z",
     "K[f][c] = K[f][c] + ((a + b) + e);", "K[f][c] = K[f][c] + (a + b);"),
    ("v_z diffused with the field constant",
     "for (int k = 0; k < 3; ++k) { qs[Q_V + k] = v[k]; cls[Q_V + k] = C_V; }",
     "for (int k = 0; k < 3; ++k) { qs[Q_V + k] = v[k]; cls[Q_V + k] = k == 2 ? C_B : C_V; }"),
    ("periodic z+ ghosts from the wrong image",
     "int s = bc[5] == ORC_PERIODIC ? imod(k, nz) : iclamp(k, nz);",
     "int s = bc[5] == ORC_PERIODIC ? imod(k - 1, nz) : iclamp(k, nz);"),
    ("open z- boundary copies the second cell",
     "int s = bc[4] == ORC_PERIODIC ? imod(k, nz) : iclamp(k, nz);",
     "int s = bc[4] == ORC_PERIODIC ? imod(k, nz) : 1;"),
    ("CFL step from the largest ratio",
     "if (act[d]) m = m < 0.0 ? h[d] / c[d] : dmin(m, h[d] / c[d]);",
     "if (act[d]) m = m < 0.0 ? h[d] / c[d] : dmax(m, h[d] / c[d]);"),
    ("z wave speed without the fast speed",
     "cz = dmax(cz, fabs(uz) + cf);", "cz = dmax(cz, fabs(uz));"),
    ("sums without dz",
     "sums[q] = psum(f[q], n) * ((dx * dy) * dz);", "sums[q] = psum(f[q], n) * (dx * dy);"),
    ("low-storage accumulator without dt K2",
     "aq[c] = (u[c] + u[c]) + ((sq[c] - u[c]) + dt * kq[c]);", "aq[c] = (u[c] + u[c]) + (sq[c] - u[c]);"),
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
    c = os.path.join(d, "sacx_oracle3d.c")
    with open(c, "w") as fh:
        fh.write(_mutant_source(text, new))
    lib = os.path.join(d, "liborc3.so")
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-o", lib, c, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        return name, "compile", r.stderr[-500:]
    env = dict(os.environ, SACX_ORACLE3D_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode, r.stdout[-300:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_3d_pins_catch_every_mutant(tmp_path):
    workers = max(1, min(4, (os.cpu_count() or 2) // 2))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda a: _run_pins(str(tmp_path), a[0], *a[1]), enumerate(MUTANTS)))
    survivors = [(n, rc, out) for n, rc, out in results if rc == 0]
    broken = [(n, out) for n, rc, out in results if rc == "compile"]
    assert not broken, broken
    assert not survivors, survivors
