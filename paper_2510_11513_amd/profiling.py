"""Summaries of rocprofv3 output (its rocpd SQLite database).

    python -m paper_2510_11513_amd.profiling stats <run_results.db> <out.md> "<command>"
    python -m paper_2510_11513_amd.profiling pmc <fetch.db> <write.db> <out.md> "<fetch command>" "<write command>"
    python -m paper_2510_11513_amd.profiling sq <sq.db> <out.md> "<command>" <tasks per sweep> <solves per sweep> \
        [<bench JSON line file> ["<the command that wrote it>"]]

`stats` lists every kernel's dispatch count and duration.  `pmc` scales the
FETCH_SIZE and WRITE_SIZE counters (KiB per dispatch) of the sweep kernel by
what the same counters read for a plain 1 GiB device copy recorded in the same
run, giving HBM bytes per sweep launch.  `sq` summarises the shader
sequencer counters of the default sweep kernel (waves, instruction mix, wave
cycles, dependency waits) per task and per 64 solves, and, given the
benchmark's JSON line, the in-kernel phase statistics of the same workload.
"""
from __future__ import annotations

import hashlib
import os
import re
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 2 ** 30


def kernel_hash() -> str:
    path = os.path.join(ROOT, "paper_2510_11513_amd", "csrc", "k_sweep.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def _short(name: str) -> str:
    name = name.replace("snx::(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0][:60]


def kernel_stats(db: str):
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
                       "from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1.0
    return [(_short(r[0]), r[1], r[2] / 1e6, r[3] / 1e3, r[4] / 1e3, r[5] / 1e3, 100.0 * r[2] / total)
            for r in rows]


def stats_summary(db: str, out_path: str, command: str) -> str:
    lines = ["# rocprofv3 kernel statistics", "", f"command: `{command}`", "",
             "| kernel | calls | total ms | average us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for name, calls, tot, avg, mn, mx, pct in kernel_stats(db):
        lines.append(f"| {name} | {calls} | {tot:.3f} | {avg:.2f} | {mn:.2f} | {mx:.2f} | {pct:.2f} |")
    text = "\n".join(lines) + "\n"
    with open(out_path, "w") as fh:
        fh.write(text)
    return text


def _counter(db: str, counter: str):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, value from counters_collection where counter_name=?", (counter,))
    out = {}
    for name, v in rows:
        out.setdefault(name, []).append(float(v))
    return out


def pmc_summary(fetch_db: str, write_db: str, out_path: str, fetch_cmd: str, write_cmd: str) -> str:
    fetch, write = _counter(fetch_db, "FETCH_SIZE"), _counter(write_db, "WRITE_SIZE")

    def copy_value(d):   # the plain 1 GiB copy is the largest dispatch of the runtime's copy kernel (the
        #                   library's own copy kernels do not count)
        return max(max(v) for k, v in d.items() if "rocclr_copyBuffer" in k)

    def sweep_values(d):   # default dependency-driven sweeps that did work (not the per-level comparator
        #                     nor the variant for the optional physics)
        vals = [x for k, v in d.items() if re.search(r"k_sweep<\d+, (true|false), false, false(, 1)?>", k) for x in v]
        top = max(vals)
        return [x for x in vals if x > 0.5 * top]

    f_copy, w_copy = copy_value(fetch), copy_value(write)
    fs, ws = sweep_values(fetch), sweep_values(write)
    kib = COPY_BYTES / 1024.0
    f_scale, w_scale = kib / f_copy, kib / w_copy
    f_sw, w_sw = sum(fs) / len(fs), sum(ws) / len(ws)
    traffic = (f_sw * f_scale + w_sw * w_scale) * 1024.0
    text = "\n".join([
        "# HBM traffic of the sweep kernel (rocprofv3 counters)", "",
        f"fetch command: `{fetch_cmd}`", "", f"write command: `{write_cmd}`", "",
        f"- FETCH_SIZE per sweep dispatch: {f_sw:.1f} KiB (mean of {len(fs)}); the plain 1 GiB copy in the same "
        f"run reads {f_copy:.1f} KiB, scale {f_scale:.4f}",
        f"- WRITE_SIZE per sweep dispatch: {w_sw:.1f} KiB (mean of {len(ws)}); the copy writes {w_copy:.1f} KiB, "
        f"scale {w_scale:.4f}",
        f"- scaled read {f_sw * f_scale * 1024 / 1e9:.3f} GB + write {w_sw * w_scale * 1024 / 1e9:.3f} GB per launch",
        "",
        f"traffic_bytes_per_launch: {traffic:.6e}",
        f"kernel_source_sha256_16: {kernel_hash()}", ""])
    with open(out_path, "w") as fh:
        fh.write(text)
    return text


SQ_COUNTERS = ("SQ_WAVES", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU",
               "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_WAIT_INST_ANY", "GRBM_GUI_ACTIVE")


def sq_summary(db: str, out_path: str, command: str, tasks: int, solves: int, bench_json: str | None = None,
               simds: int = 1024, xcds: int = 8, bench_command: str = "python3 bench.py --gpus 1 --steps 20 --warmup 5") -> str:
    vals = {}
    for c in SQ_COUNTERS:
        d = _counter(db, c)
        v = [x for k, xs in d.items() if re.search(r"k_sweep<\d+, (true|false), false, false(, 1)?>", k) for x in xs]
        vals[c] = sum(v) / len(v) if v else float("nan")
        n = len(v)
    rounds = solves / 64.0
    gui_xcd = vals["GRBM_GUI_ACTIVE"] / xcds
    lines = ["# Shader sequencer counters of the sweep kernel (rocprofv3)", "", f"command: `{command}`", "",
             f"Mean per dispatch of the dependency-driven sweep kernel over {n} dispatches; {tasks} (cell, octant) "
             f"tasks and {solves} solves per dispatch.", "",
             "| counter | per dispatch | per task | per 64 solves |", "|---|---|---|---|"]
    for c in SQ_COUNTERS:
        lines.append(f"| {c} | {vals[c]:.4e} | {vals[c] / tasks:.1f} | {vals[c] / rounds:.2f} |")
    lines += ["", "Derived (formulas stated; GRBM_GUI_ACTIVE is read as the sum over the XCDs):", "",
              f"- resident waves: SQ_WAVES = {vals['SQ_WAVES']:.0f} = {vals['SQ_WAVES'] / (simds // 4):.1f} per CU "
              f"(persistent launch: every wave stays for the whole sweep)",
              f"- VALU issue share: 4 * SQ_ACTIVE_INST_VALU / (SIMDs * GRBM_GUI_ACTIVE / XCDs) = "
              f"{4 * vals['SQ_ACTIVE_INST_VALU'] / (simds * gui_xcd):.2f}",
              f"- share of wave cycles waiting on a dependency (s_waitcnt): SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES = "
              f"{vals['SQ_WAIT_INST_ANY'] / vals['SQ_WAVE_CYCLES']:.3f}",
              f"- instruction mix per 64 solves: VALU {vals['SQ_INSTS_VALU'] / rounds:.0f}, SALU "
              f"{vals['SQ_INSTS_SALU'] / rounds:.0f}, LDS {vals['SQ_INSTS_LDS'] / rounds:.0f}"]
    if bench_json:
        import json
        rec = json.loads(open(bench_json).read().strip().splitlines()[-1])
        lines += ["", "In-kernel phase statistics (`snx_set_sweep_stats`, one sweep, shader-clock cycles summed over "
                  f"workgroups) of the same code, from the `phases` objects of `{bench_command}`:", "",
                  "| workload | tasks | continued by the same workgroup | empty queue polls | cycles per task | "
                  "queue wait | stage | operator build | solve | publish |", "|---|---|---|---|---|---|---|---|---|---|"]
        for name, r in (("headline", rec), ("secondary", rec.get("secondary", {}))):
            ph = r.get("phases")
            if not ph:
                continue
            wl = (r["config"]["workload"] if name == "headline" else r["workload"]).split(":")[0]
            cs = ph["cycle_share"]
            lines.append(f"| {wl} | {ph['tasks']} | {ph['continued']} | {ph['empty_polls']} | "
                         f"{ph['cycles_per_task']:.0f} | {cs['queue_wait']:.3f} | {cs['stage']:.3f} | "
                         f"{cs['build']:.3f} | {cs['solve']:.3f} | {cs['publish']:.3f} |")
    text = "\n".join(lines) + "\n"
    with open(out_path, "w") as fh:
        fh.write(text)
    return text


def counter_table(db: str, out_path: str, command: str, kernel: str, units: float, unit_name: str,
                  title: str) -> str:
    """Totals of every counter in the run over the dispatches of the kernels whose
    names match `kernel`, per dispatch and per unit of work (`units` units over
    all of those dispatches)."""
    con = sqlite3.connect(db)
    names = [r[0] for r in con.execute("select distinct counter_name from counters_collection")]
    lines = [f"# {title} (rocprofv3)", "", f"command: `{command}`", "",
             f"| counter | dispatches | total | per dispatch | per {unit_name} |", "|---|---|---|---|---|"]
    tot = {}
    for c in sorted(names):
        v = [x for k, xs in _counter(db, c).items() if re.search(kernel, k) for x in xs]
        if not v:
            continue
        tot[c] = sum(v)
        lines.append(f"| {c} | {len(v)} | {sum(v):.4e} | {sum(v) / len(v):.4e} | {sum(v) / units:.1f} |")
    if "SQ_WAVE_CYCLES" in tot:
        for c in ("SQ_WAIT_INST_LDS", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_VALU"):
            if c in tot:
                lines.append(f"\n- {c} / SQ_WAVE_CYCLES = {tot[c] / tot['SQ_WAVE_CYCLES']:.3f}")
    text = "\n".join(lines) + "\n"
    with open(out_path, "w") as fh:
        fh.write(text)
    return text


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats_summary(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif sys.argv[1] == "pmc":
        print(pmc_summary(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6]))
    elif sys.argv[1] == "table":
        print(counter_table(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], float(sys.argv[6]), sys.argv[7],
                            sys.argv[8]))
    elif sys.argv[1] == "sq":
        print(sq_summary(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), int(sys.argv[6]),
                         sys.argv[7] if len(sys.argv) > 7 else None,
                         **({"bench_command": sys.argv[8]} if len(sys.argv) > 8 else {})))
