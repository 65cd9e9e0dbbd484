"""Summaries of rocprofv3 output for the stage kernel (text for profiles/).

  python -m paper_1710_06423_amd.profiling stats  STATS_CSV BENCH_LOG OUT_MD TITLE COMMAND
  python -m paper_1710_06423_amd.profiling sq     COUNTER_CSV BENCH_LOG OUT_MD COMMAND
  python -m paper_1710_06423_amd.profiling table  STATS_CSV BENCH_LOG OUT_MD TITLE COMMAND [NOTE...]
  python -m paper_1710_06423_amd.profiling select STATS_CSV BENCH_LOG OUT_MD TITLE PATTERN COMMAND [NOTE...]
  python -m paper_1710_06423_amd.profiling traffic FETCH_CSV WRITE_CSV CFETCH_CSV CWRITE_CSV COPY_BYTES
                                                  BENCH_LOG OUT_MD COMMANDS...
  python -m paper_1710_06423_amd.profiling kernels SQ_CSV FETCH_CSV WRITE_CSV CFETCH_CSV CWRITE_CSV COPY_BYTES
                                                  PATTERN BENCH_LOG OUT_MD TITLE COMMANDS...

`stats` turns a --kernel-trace --stats kernel summary into a table and
compares the mean stage-kernel launch with the bench's own HIP-event timing.
`kernels` gives both, per kernel matching PATTERN, for any launch.
`traffic` turns two --pmc passes (FETCH_SIZE, WRITE_SIZE, KiB per dispatch)
over the stage kernel and the same two passes over a device copy of known
size into HBM bytes per stage launch: each counter is divided by what it
reads per byte of the copy.  The traffic file records a hash of the stage
kernel's code (its sources without comments and layout); bench.py reports the
traffic only while the hash matches.
"""

from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys
from typing import Dict, List, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
STAGE_SOURCES = ("csrc/sacx_tile.h", "csrc/sacx_tile_split.h", "csrc/sacx_stage_kernel.h", "csrc/sacx_stage.hip",
                 "csrc/sacx_stage_split.hip", "csrc/sacx_internal.h")
STAGE_UNITS = ("sacx_stage.hip", "sacx_stage_split.hip")


def stage_build_settings() -> str:
    """The compiler settings of the stage kernel's units (target, flags,
    contraction rule, scheduler), without the machine's include paths."""
    from . import build as B
    flags = [f for f in B.FLAGS if not os.path.isabs(f)]
    per_unit = [(u, B.CONTRACT.get(u, "-ffp-contract=off"), list(B.SCHED.get(u, []))) for u in STAGE_UNITS]
    return repr((B.ARCH, flags, per_unit))


def code_text(src: str) -> str:
    """C++ source without its comments and with runs of white space made one
    space (string literals are left alone), so that a change of comments or
    layout leaves the hash of the stage kernel's code unchanged."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c == '"' or c == "'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def stage_source_hash(read=None) -> str:
    """Hash of the stage kernel's code (comments and layout excluded) and of
    the settings its units are compiled with.  `read(rel)` returns a source's
    text (default: the working tree)."""
    h = hashlib.sha256()
    for rel in STAGE_SOURCES:
        if read is None:
            with open(os.path.join(HERE, rel)) as fh:
                text = fh.read()
        else:
            text = read(rel)
        h.update(code_text(text).encode())
    h.update(stage_build_settings().encode())
    return h.hexdigest()[:16]


def _bench_line(path: str) -> Dict:
    for line in reversed(open(path).read().strip().splitlines()):
        line = line.strip()
        if line.startswith("{"):
            return json.loads(line)
    raise ValueError(f"no JSON line in {path}")


def _short(name: str) -> str:
    return name.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]


def stats_summary(stats_csv: str, bench_log: str, title: str, command: str) -> str:
    rows = list(csv.DictReader(open(stats_csv)))
    b = _bench_line(bench_log)
    out = [f"# {title}", "", "Command (repository root on the GPU host):", "", "    " + command, "",
           f"Stage kernel sources hash: {stage_source_hash()}", "",
           "| kernel | calls | avg ms | % of GPU time |", "|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                   f"{float(r['Percentage']):.1f} |")
    st = [r for r in rows if "k_stage" in r["Name"]]
    if st:
        avg = sum(float(r["TotalDurationNs"]) for r in st) / sum(int(r["Calls"]) for r in st) / 1e6
        nl = 4 * b["steps"]
        ev = sum(b["phases_ms"]["stage"]) / nl
        w = 8 if b["dtype"] == "f64" else 4
        cells = b["config"]["nx"] * b["config"]["ny"]
        per_cell = b["config"].get("bytes_per_cell_update", 72 * w) / 4   # per stage launch
        gb = per_cell * cells / 1e9
        out += ["", f"Mean stage-kernel launch: {avg:.3f} ms (rocprofv3, every launch including warm-up) vs "
                    f"{ev:.3f} ms from the bench's HIP events over its timed steps (same run).",
                f"Algorithmic bytes per stage launch: {per_cell:.0f} B x {cells / 1e6:.0f}e6 cells = {gb:.3f} GB -> "
                f"{gb / avg * 1e3:.0f} GB/s = {gb / avg * 1e3 / 8000 * 100:.1f} % of 8 TB/s.",
                f"Bench line of the same run: {b['value']:.0f} Mcell-updates/s, {b['ms_per_step']:.2f} ms/step, "
                f"roofline.achieved {b['roofline']['achieved']} GB/s."]
    return "\n".join(out) + "\n"


def pmc_per_kernel(counter_csv: str, counter: str) -> Dict[str, List[float]]:
    """Counter values per dispatch, grouped by kernel name."""
    res: Dict[str, List[float]] = {}
    for r in csv.DictReader(open(counter_csv)):
        if r.get("Counter_Name", counter) != counter:
            continue
        res.setdefault(_short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return res


def _mean_of(d: Dict[str, List[float]], pattern: str) -> float:
    vals = [v for k, vs in d.items() if re.search(pattern, k) for v in vs]
    if not vals:
        raise ValueError(f"no dispatch of a kernel matching {pattern!r}")
    return sum(vals) / len(vals)


def traffic_summary(fetch_csv: str, write_csv: str, cfetch_csv: str, cwrite_csv: str, copy_bytes: int,
                    bench_log: str, commands: List[str], copy_pattern: str = "copyBuffer") -> str:
    b = _bench_line(bench_log)
    f_st = _mean_of(pmc_per_kernel(fetch_csv, "FETCH_SIZE"), "k_stage")
    w_st = _mean_of(pmc_per_kernel(write_csv, "WRITE_SIZE"), "k_stage")
    f_cp = _mean_of(pmc_per_kernel(cfetch_csv, "FETCH_SIZE"), copy_pattern)
    w_cp = _mean_of(pmc_per_kernel(cwrite_csv, "WRITE_SIZE"), copy_pattern)
    kf = f_cp * 1024.0 / copy_bytes      # counter KiB-units read per byte copied
    kw = w_cp * 1024.0 / copy_bytes
    fetch_b = f_st * 1024.0 / kf
    write_b = w_st * 1024.0 / kw
    w = 8 if b["dtype"] == "f64" else 4
    cells = b["config"]["nx"] * b["config"]["ny"]
    alg = b["config"].get("bytes_per_cell_update", 72 * w) / 4 * cells   # per stage launch
    lines = [f"# HBM traffic of the stage kernel -- {b['config']['workload']}", "",
             "Commands (repository root on the GPU host), one counter per run:", ""]
    lines += ["    " + c for c in commands]
    lines += ["", f"stage_source_hash: {stage_source_hash()}",
              f"copy_calibration: FETCH_SIZE {f_cp:.1f} KiB and WRITE_SIZE {w_cp:.1f} KiB per copy dispatch of "
              f"{copy_bytes} bytes -> factors {kf:.4f} (fetch) and {kw:.4f} (write) counter-KiB per KiB moved",
              f"stage_fetch_kib_per_dispatch: {f_st:.1f}",
              f"stage_write_kib_per_dispatch: {w_st:.1f}",
              f"traffic_bytes_per_launch: {fetch_b + write_b:.6e}",
              f"fetch_bytes_per_launch: {fetch_b:.6e}",
              f"write_bytes_per_launch: {write_b:.6e}",
              f"algorithmic_bytes_per_launch: {alg:.6e}",
              f"traffic_over_algorithmic: {(fetch_b + write_b) / alg:.3f}"]
    return "\n".join(lines) + "\n"


def table_summary(stats_csv: str, bench_log: str, title: str, command: str, notes: List[str],
                  top: int = 16, pattern: Optional[str] = None) -> str:
    """Any kernel trace as a table (the `top` kernels by GPU time, or every
    kernel whose name matches `pattern`), with the bench line of the same
    run."""
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    if pattern is not None:
        rows = [r for r in rows if re.search(pattern, _short(r["Name"]))]
        top = len(rows)
    b = _bench_line(bench_log)
    out = [f"# {title}", "", "Command (repository root on the GPU host):", "", "    " + command, ""]
    out += [n for n in notes] + ([""] if notes else [])
    out += ["| kernel | calls | avg ms | % of GPU time |", "|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                   f"{float(r['Percentage']):.1f} |")
    out += ["", f"Bench line of the same run: workload {b['config']['workload']}, {b['value']} {b['unit']}, "
                f"{b['ms_per_step']} ms/step over {b['steps']} steps."]
    return "\n".join(out) + "\n"


SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_WAVE_CYCLES",
               "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_BUSY_CYCLES")


def sq_summary(counter_csv: str, bench_log: str, command: str) -> str:
    """Per stage kernel: instructions per wave and the share of a wave's
    lifetime with a VALU instruction active (both SQ counters count in the
    same cycle units)."""
    b = _bench_line(bench_log)
    agg: Dict[str, Dict[str, float]] = {}
    for r in csv.DictReader(open(counter_csv)):
        name = _short(r["Kernel_Name"])
        if "k_stage" not in name:
            continue
        agg.setdefault(name, {}).setdefault(r["Counter_Name"], 0.0)
        agg[name][r["Counter_Name"]] += float(r["Counter_Value"])
    lines = [f"# Instruction mix of the stage kernel -- {b['config']['workload']}", "",
             "Command (repository root on the GPU host):", "", "    " + command, "",
             f"Stage kernel sources hash: {stage_source_hash()}", "",
             "| kernel | VALU / wave | LDS / wave | SALU / wave | VALU active / wave cycles | waiting on counters / wave cycles |",
             "|---|---|---|---|---|---|"]
    for name, d in sorted(agg.items()):
        w = d["SQ_WAVES"]
        lines.append(f"| `{name}` | {d['SQ_INSTS_VALU'] / w:.0f} | {d['SQ_INSTS_LDS'] / w:.0f} | "
                     f"{d['SQ_INSTS_SALU'] / w:.0f} | {d['SQ_ACTIVE_INST_VALU'] / d['SQ_WAVE_CYCLES']:.2f} | "
                     f"{d['SQ_WAIT_INST_ANY'] / d['SQ_WAVE_CYCLES']:.2f} |")
    return "\n".join(lines) + "\n"


def kernels_summary(sq_csv: str, fetch_csv: str, write_csv: str, cfetch_csv: str, cwrite_csv: str,
                    copy_bytes: int, pattern: str, bench_log: str, title: str, commands: List[str],
                    copy_pattern: str = "copyBuffer") -> str:
    """Per kernel matching `pattern`: the instruction mix (the SQ counters of
    `sq_summary`) and its HBM bytes per dispatch from FETCH_SIZE and
    WRITE_SIZE, calibrated against a device copy of known size as in
    `traffic_summary`, also per cell of the bench's grid."""
    b = _bench_line(bench_log)
    agg: Dict[str, Dict[str, float]] = {}
    for r in csv.DictReader(open(sq_csv)):
        name = _short(r["Kernel_Name"])
        if not re.search(pattern, name):
            continue
        agg.setdefault(name, {}).setdefault(r["Counter_Name"], 0.0)
        agg[name][r["Counter_Name"]] += float(r["Counter_Value"])
    fetch = pmc_per_kernel(fetch_csv, "FETCH_SIZE")
    write = pmc_per_kernel(write_csv, "WRITE_SIZE")
    kf = _mean_of(pmc_per_kernel(cfetch_csv, "FETCH_SIZE"), copy_pattern) * 1024.0 / copy_bytes
    kw = _mean_of(pmc_per_kernel(cwrite_csv, "WRITE_SIZE"), copy_pattern) * 1024.0 / copy_bytes
    cfg = b["config"]
    cells = cfg.get("nx", 1) * cfg.get("ny", 1) * cfg.get("nz", 1)
    lines = [f"# {title}", "", "Commands (repository root on the GPU host), one counter set per run:", ""]
    lines += ["    " + c for c in commands]
    lines += ["", f"Copy calibration: {kf:.4f} (FETCH_SIZE) and {kw:.4f} (WRITE_SIZE) counter-KiB per KiB moved.",
              f"Bench line of the fetch run: workload {cfg['workload']}, {b['value']} {b['unit']}.", "",
              "| kernel | VALU / wave | LDS / wave | SALU / wave | VALU active / wave cycles | "
              "waiting on counters / wave cycles | HBM read GB / dispatch | HBM written GB / dispatch | "
              "HBM B / cell |", "|---|---|---|---|---|---|---|---|---|"]
    for name, d in sorted(agg.items()):
        w = d["SQ_WAVES"]
        fb = sum(fetch.get(name, [0.0])) / max(len(fetch.get(name, [])), 1) * 1024.0 / kf
        wb = sum(write.get(name, [0.0])) / max(len(write.get(name, [])), 1) * 1024.0 / kw
        lines.append(f"| `{name}` | {d['SQ_INSTS_VALU'] / w:.0f} | {d['SQ_INSTS_LDS'] / w:.0f} | "
                     f"{d['SQ_INSTS_SALU'] / w:.0f} | {d['SQ_ACTIVE_INST_VALU'] / d['SQ_WAVE_CYCLES']:.2f} | "
                     f"{d['SQ_WAIT_INST_ANY'] / d['SQ_WAVE_CYCLES']:.2f} | {fb / 1e9:.3f} | {wb / 1e9:.3f} | "
                     f"{(fb + wb) / cells:.0f} |")
    return "\n".join(lines) + "\n"


def read_traffic(path: str) -> Optional[Dict[str, float]]:
    """The traffic file's figures, or None when it is missing or was taken
    from other stage-kernel sources than the current ones."""
    try:
        text = open(path).read()
    except OSError:
        return None
    kv = dict(re.findall(r"^(\w+): (\S+)", text, re.M))
    if kv.get("stage_source_hash") != stage_source_hash():
        return None
    try:
        return {k: float(kv[k]) for k in ("traffic_bytes_per_launch", "fetch_bytes_per_launch",
                                          "write_bytes_per_launch", "algorithmic_bytes_per_launch")}
    except (KeyError, ValueError):
        return None


def main(argv: List[str]):
    if argv and argv[0] == "stats" and len(argv) == 6:
        text = stats_summary(argv[1], argv[2], argv[4], argv[5])
        open(argv[3], "w").write(text)
        print(text)
    elif argv and argv[0] == "table" and len(argv) >= 6:
        text = table_summary(argv[1], argv[2], argv[4], argv[5], argv[6:])
        open(argv[3], "w").write(text)
        print(text)
    elif argv and argv[0] == "select" and len(argv) >= 7:
        text = table_summary(argv[1], argv[2], argv[4], argv[6], argv[7:], pattern=argv[5])
        open(argv[3], "w").write(text)
        print(text)
    elif argv and argv[0] == "sq" and len(argv) == 5:
        text = sq_summary(argv[1], argv[2], argv[4])
        open(argv[3], "w").write(text)
        print(text)
    elif argv and argv[0] == "kernels" and len(argv) >= 12:
        text = kernels_summary(argv[1], argv[2], argv[3], argv[4], argv[5], int(argv[6]), argv[7], argv[8],
                               argv[10], argv[11:])
        open(argv[9], "w").write(text)
        print(text)
    elif argv and argv[0] == "traffic" and len(argv) >= 9:
        text = traffic_summary(argv[1], argv[2], argv[3], argv[4], int(argv[5]), argv[6], argv[8:])
        open(argv[7], "w").write(text)
        print(text)
    else:
        print(__doc__)
        sys.exit(2)


if __name__ == "__main__":
    main(sys.argv[1:])
