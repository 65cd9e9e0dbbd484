"""Host logic of the build script (no GPU, no real compiler).

A stand-in compiler records its arguments and fails whenever it is given the
non-default scheduler: the unit built with that scheduler must then be built
again with the default one, and every other unit must see no change.
"""

import os
import stat

import pytest

from paper_1710_06423_amd import build

FAKE = """#!/bin/sh
echo "$@" >> "{log}"
case "$*" in
  *amdgpu-sched-strategy*) echo "scheduler failure" >&2; exit 1 ;;
esac
while [ $# -gt 0 ]; do
  if [ "$1" = "-o" ]; then : > "$2"; fi
  shift
done
exit 0
"""


@pytest.fixture
def fake_hipcc(tmp_path, monkeypatch):
    log = tmp_path / "calls.log"
    exe = tmp_path / "hipcc"
    exe.write_text(FAKE.format(log=log))
    exe.chmod(exe.stat().st_mode | stat.S_IXUSR)
    monkeypatch.setattr(build, "HIPCC", str(exe))
    monkeypatch.setattr(build, "BUILD", str(tmp_path))
    return log


def test_scheduler_failure_falls_back_to_default(fake_hipcc, capsys):
    src = next(iter(build.SCHED))
    obj = build._compile(src)
    assert os.path.exists(obj)
    calls = fake_hipcc.read_text().splitlines()
    assert len(calls) == 2
    assert "amdgpu-sched-strategy" in calls[0] and "amdgpu-sched-strategy" not in calls[1]
    assert "default scheduler" in capsys.readouterr().err


def test_units_without_a_scheduler_choice_compile_once(fake_hipcc):
    src = next(s for s in build.SOURCES if s not in build.SCHED)
    build._compile(src)
    calls = fake_hipcc.read_text().splitlines()
    assert len(calls) == 1 and "amdgpu-sched-strategy" not in calls[0]
    # the packed-FP32 switch and the unit's contraction rule are on every line
    assert "-packed-fp32-ops" in calls[0]
    assert build.CONTRACT.get(src, "-ffp-contract=off") in calls[0]
