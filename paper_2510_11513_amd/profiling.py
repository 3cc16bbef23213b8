"""Summaries of rocprofv3 output (its rocpd SQLite database).

    python -m paper_2510_11513_amd.profiling stats <run_results.db> <out.md> "<command>"
    python -m paper_2510_11513_amd.profiling pmc <fetch.db> <write.db> <out.md> "<fetch command>" "<write command>"

`stats` lists every kernel's dispatch count and duration.  `pmc` scales the
FETCH_SIZE and WRITE_SIZE counters (KiB per dispatch) of the sweep kernel by
what the same counters read for a plain 1 GiB device copy recorded in the same
run, giving HBM bytes per sweep launch.
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

    def copy_value(d):   # the plain 1 GiB copy is the largest dispatch of the runtime's copy kernel
        return max(max(v) for k, v in d.items() if "copyBuffer" in k or "copy" in k.lower())

    def sweep_values(d):   # default dependency-driven sweeps that did work (not the per-level comparator
        #                     nor the variant for the optional physics)
        vals = [x for k, v in d.items() if re.search(r"k_sweep<\d+, (true|false), false, false>", k) for x in v]
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


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats_summary(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif sys.argv[1] == "pmc":
        print(pmc_summary(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6]))
