"""Summaries of rocprofv3 output for the traversal kernels.

rocprofv3 (ROCm 7) writes its results as an SQLite database (``*_results.db``).
This module turns such databases into short Markdown summaries and, for
hardware-counter runs, into HBM bytes per kernel launch:

  python -m paper_1209_6007_amd.profiling trace DIR --title T --command C
      kernel-trace statistics (calls, total and average duration, resources)

  python -m paper_1209_6007_amd.profiling pmc FETCH_DIR WRITE_DIR --kernel NAME \
      --workload W --kernel-class K --title T --command C [--json PATH]
      FETCH_SIZE / WRITE_SIZE of the kernel per dispatch, scaled by what the
      same counters read for the library's streaming copy kernel of known size
      (sbc_copy_bandwidth run in the same process), and optionally recorded in
      a JSON file keyed by workload and kernel class with the kernel source hash.

FETCH_SIZE and WRITE_SIZE are in KiB per dispatch.  On gfx950 FETCH_SIZE counts
64 bytes per L2-to-fabric read request, so 128-byte requests (a streaming copy)
read as half their size; the copy-kernel factor corrects for that for streaming
traffic, and random 64-byte requests are then over-counted by the same factor,
which makes the scaled figure an upper bound for a random-access kernel.
"""
from __future__ import annotations

import argparse
import glob
import json
import os
import sqlite3
import sys

from . import kernel_source_hash

COPY_KERNEL = "copy_kernel"
COPY_BYTES = 1 << 30  # bytes read and bytes written by one copy launch of the calibration


def _dbs(path: str):
    if path.endswith(".db"):
        return [path]
    out = sorted(glob.glob(os.path.join(path, "**", "*.db"), recursive=True))
    if not out:
        raise FileNotFoundError(f"no rocprofv3 database under {path}")
    return out


def kernel_stats(path: str):
    """[(name, calls, total_us, avg_us, pct, grid, wg, lds, vgpr, agpr, sgpr, scratch)] by total time."""
    rows = {}
    extra = {}
    for db in _dbs(path):
        c = sqlite3.connect(db)
        for name, calls, tot, avg, pct in c.execute(
                "select name, total_calls, total_duration, average, percentage from top_kernels"):
            r = rows.setdefault(name, [0, 0.0])
            r[0] += calls
            r[1] += tot
        for r in c.execute("select name, grid_x, workgroup_x, lds_size, vgpr_count, accum_vgpr_count, sgpr_count, "
                           "scratch_size from kernels"):
            extra.setdefault(r[0], r[1:])
        c.close()
    total = sum(v[1] for v in rows.values()) or 1.0
    out = []
    for name, (calls, tot) in sorted(rows.items(), key=lambda kv: -kv[1][1]):
        # the top_kernels view reports microseconds
        out.append((name, calls, tot, tot / max(calls, 1), 100.0 * tot / total) + tuple(extra.get(name, ("",) * 7)))
    return out


def counter_values(path: str):
    """{kernel name: {counter: [value per dispatch, in dispatch order]}}."""
    out = {}
    for db in _dbs(path):
        c = sqlite3.connect(db)
        for name, counter, value in c.execute(
                "select kernel_name, counter_name, value from counters_collection order by dispatch_id"):
            out.setdefault(name, {}).setdefault(counter, []).append(float(value))
        c.close()
    return out


def _match(values: dict, sub: str):
    names = [k for k in values if sub in k]
    if not names:
        raise KeyError(f"no kernel matching {sub!r}; kernels: {sorted(values)[:8]}")
    return names


def pmc_summary(fetch_dir: str, write_dir: str, kernel: str):
    f = counter_values(fetch_dir)
    w = counter_values(write_dir)
    res = {}
    for tag, vals, counter in (("fetch", f, "FETCH_SIZE"), ("write", w, "WRITE_SIZE")):
        copy = [v for n in _match(vals, COPY_KERNEL) for v in vals[n].get(counter, [])]
        if not copy:
            raise KeyError(f"no {counter} values for the copy kernel")
        copy_kib = sum(copy) / len(copy)
        factor = (COPY_BYTES / 1024.0) / copy_kib
        launches = [v for n in _match(vals, kernel) for v in vals[n].get(counter, [])]
        if not launches:
            raise KeyError(f"no {counter} values for {kernel}")
        kib = sum(launches) / len(launches)
        res[tag] = {"counter": counter, "copy_kib_per_launch": copy_kib, "factor": factor,
                    "kib_per_launch_raw": kib, "bytes_per_launch": kib * 1024.0 * factor,
                    "launches": len(launches)}
    res["bytes_per_launch"] = res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]
    return res


def _cmd_trace(a):
    rows = kernel_stats(a.dir)
    print(f"# {a.title}\n")
    print("Command (run from the repository root on one MI355X):\n")
    print("```\n" + a.command + "\n```\n")
    print("rocprofv3 kernel statistics (durations in microseconds):\n")
    print("| kernel | calls | total us | average us | % | grid | wg | LDS B | VGPR | AGPR | SGPR | scratch |")
    print("|---|---|---|---|---|---|---|---|---|---|---|---|")
    for r in rows:
        name, calls, tot, avg, pct = r[:5]
        g = r[5:]
        print(f"| `{name}` | {calls} | {tot:.1f} | {avg:.1f} | {pct:.2f} | " + " | ".join(str(x) for x in g) + " |")


def _cmd_pmc(a):
    s = pmc_summary(a.fetch_dir, a.write_dir, a.kernel)
    sha = kernel_source_hash()
    print(f"# {a.title}\n")
    print("Commands (run from the repository root on one MI355X, one counter per run):\n")
    print("```\n" + a.command + "\n```\n")
    print(f"Kernel: names containing `{a.kernel}`; kernel source hash `{sha}`.\n")
    print("| counter | copy kernel KiB/launch (1 GiB moved) | scale factor | kernel KiB/launch (raw) | "
          "kernel bytes/launch (scaled) | launches |")
    print("|---|---|---|---|---|---|")
    for tag in ("fetch", "write"):
        r = s[tag]
        print(f"| {r['counter']} | {r['copy_kib_per_launch']:.1f} | {r['factor']:.4f} | {r['kib_per_launch_raw']:.1f} | "
              f"{r['bytes_per_launch']:.4e} | {r['launches']} |")
    print(f"\nHBM traffic per launch (fetch + write, scaled): **{s['bytes_per_launch']:.4e} bytes**.")
    if a.json:
        d = {}
        if os.path.exists(a.json):
            with open(a.json) as fh:
                d = json.load(fh)
        d.setdefault(a.workload, {})[a.kernel_class] = {
            "kernel_sha": sha, "bytes_per_launch": s["bytes_per_launch"],
            "fetch_bytes_per_launch": s["fetch"]["bytes_per_launch"],
            "write_bytes_per_launch": s["write"]["bytes_per_launch"],
            "fetch_factor": s["fetch"]["factor"], "write_factor": s["write"]["factor"], "kernel": a.kernel}
        with open(a.json, "w") as fh:
            json.dump(d, fh, indent=1, sort_keys=True)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1209_6007_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    p = sub.add_parser("pmc")
    p.add_argument("fetch_dir")
    p.add_argument("write_dir")
    p.add_argument("--kernel", required=True)
    p.add_argument("--workload", required=True)
    p.add_argument("--kernel-class", required=True)
    p.add_argument("--title", required=True)
    p.add_argument("--command", required=True)
    p.add_argument("--json")
    a = ap.parse_args(argv)
    (_cmd_trace if a.cmd == "trace" else _cmd_pmc)(a)


if __name__ == "__main__":
    sys.exit(main())
