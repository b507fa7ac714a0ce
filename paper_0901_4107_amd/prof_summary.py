"""Summaries of rocprofv3 output databases (rocpd SQLite) for the profiles
kept with the library.

    python -m paper_0901_4107_amd.prof_summary trace DIR
        per-kernel calls, average and total duration from a --kernel-trace run

    python -m paper_0901_4107_amd.prof_summary counters DIR [--kernel NAME]
        per-kernel averages of every counter of a --pmc run (dispatches of
        the kernels whose name contains NAME, default every mm:: kernel)

    python -m paper_0901_4107_amd.prof_summary traffic --kernel NAME --workload W \\
        --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR
        HBM bytes per launch of the kernels whose name contains NAME, from a
        FETCH_SIZE run and a WRITE_SIZE run, each counter scaled by what it
        reads for a plain device copy of known size (bench.py
        --calibrate-copy MB, 5 copies of MB MiB); prints the summary and the
        'traffic:' line bench.py reads (tagged with the hash of the kernel
        sources, so a changed kernel reports no traffic).
"""
from __future__ import annotations

import argparse
import glob
import os
import re
import sqlite3
from collections import defaultdict

from .build import source_hash


def _db(path: str) -> sqlite3.Connection:
    files = glob.glob(os.path.join(path, "**", "*.db"), recursive=True)
    if not files:
        raise SystemExit(f"no rocpd database under {path}")
    return sqlite3.connect(files[0])


def _short(name: str) -> str:
    return re.sub(r"\(.*", "", name).replace("void ", "")


def trace(path: str) -> str:
    c = _db(path)
    agg = defaultdict(list)
    for name, start, end in c.execute("select name, start, end from kernels"):
        agg[_short(name)].append(end - start)
    total = sum(sum(v) for v in agg.values())
    lines = [f"{'kernel':56s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>9s} {'pct':>6s}"]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{k[:56]:56s} {len(v):6d} {sum(v) / len(v) / 1e3:10.1f} {sum(v) / 1e6:9.3f} "
                     f"{100 * sum(v) / total:6.1f}")
    return "\n".join(lines)


def counter_kib(path: str, counter: str, kernel: str) -> list[float]:
    c = _db(path)
    rows = c.execute("select kernel_name, value from counters_collection where counter_name = ?", (counter,))
    return [v for name, v in rows if kernel in _short(name)]


def counters(path: str, kernel: str = "mm::") -> str:
    c = _db(path)
    agg = defaultdict(lambda: defaultdict(list))
    for name, counter, v in c.execute("select kernel_name, counter_name, value from counters_collection"):
        if kernel in name:
            agg[_short(name)][counter].append(v)
    lines = []
    for k in sorted(agg):
        vals = " ".join(f"{cn}={sum(v) / len(v):.0f}" for cn, v in sorted(agg[k].items()))
        n = max(len(v) for v in agg[k].values())
        lines.append(f"{k} dispatches={n} {vals}")
    return "\n".join(lines)


def traffic(a) -> str:
    copy_bytes = a.copy_mib * (1 << 20)
    fk = counter_kib(a.copy_fetch, "FETCH_SIZE", a.copy_kernel)
    wk = counter_kib(a.copy_write, "WRITE_SIZE", a.copy_kernel)
    fetch_scale = copy_bytes / (1024 * max(fk))
    write_scale = copy_bytes / (1024 * max(wk))
    f = counter_kib(a.fetch, "FETCH_SIZE", a.kernel)
    w = counter_kib(a.write, "WRITE_SIZE", a.kernel)
    if not f or not w:
        raise SystemExit(f"no dispatch of a kernel named like {a.kernel!r}")
    read = sum(f) / len(f) * 1024 * fetch_scale
    written = sum(w) / len(w) * 1024 * write_scale
    out = [f"copy of {a.copy_mib} MiB: FETCH_SIZE {max(fk):.1f} KiB (scale {fetch_scale:.3f}), "
           f"WRITE_SIZE {max(wk):.1f} KiB (scale {write_scale:.3f})",
           f"{a.kernel}: {len(f)} / {len(w)} dispatches, FETCH_SIZE {sum(f) / len(f):.1f} KiB, "
           f"WRITE_SIZE {sum(w) / len(w):.1f} KiB per dispatch",
           f"per launch: {read / 1e9:.4f} GB read, {written / 1e9:.4f} GB written, "
           f"{(read + written) / 1e9:.4f} GB in all",
           f"traffic: kernel={a.kernel} workload={a.workload} read_bytes={read:.0f} "
           f"written_bytes={written:.0f} source={source_hash()}"]
    return "\n".join(out)


def read_traffic(profile_dir: str, kernel: str, workload: str) -> float | None:
    """HBM bytes per launch recorded for (kernel, workload) under
    profile_dir, if the kernel sources are those the counters were taken
    from; None otherwise."""
    src = source_hash()
    for path in glob.glob(os.path.join(profile_dir, "*.md")) + glob.glob(os.path.join(profile_dir, "*.txt")):
        with open(path) as fh:
            for line in fh:
                m = re.match(r"\s*traffic: kernel=(.+?) workload=(\S+) read_bytes=(\d+) written_bytes=(\d+) "
                             r"source=(\w+)", line)
                if m and m.group(1) == kernel and m.group(2) == workload and m.group(5) == src:
                    return float(m.group(3)) + float(m.group(4))
    return None


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    q = sub.add_parser("counters")
    q.add_argument("dir")
    q.add_argument("--kernel", default="mm::")
    r = sub.add_parser("traffic")
    r.add_argument("--kernel", required=True)
    r.add_argument("--workload", required=True)
    r.add_argument("--fetch", required=True)
    r.add_argument("--write", required=True)
    r.add_argument("--copy-fetch", required=True)
    r.add_argument("--copy-write", required=True)
    r.add_argument("--copy-mib", type=int, default=1024)
    r.add_argument("--copy-kernel", default="copyBuffer")
    a = ap.parse_args()
    if a.cmd == "trace":
        print(trace(a.dir))
    elif a.cmd == "counters":
        print(counters(a.dir, a.kernel))
    else:
        print(traffic(a))


if __name__ == "__main__":
    main()
