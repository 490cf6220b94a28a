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

  python -m paper_1209_6007_amd.profiling reqs READ_DIR WRITE_DIR --kernel NAME \
      --workload W --kernel-class K --title T --command C [--json PATH]
      HBM bytes per dispatch from the L2-to-fabric request counters by size:
      reads 32*TCC_EA0_RDREQ_32B + 64*TCC_EA0_RDREQ_64B + 128*TCC_EA0_RDREQ_128B,
      writes 64*TCC_EA0_WRREQ_64B + 32*(TCC_EA0_WRREQ - TCC_EA0_WRREQ_64B);
      the copy kernel's figures (1 GiB each way) are shown as a check.

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


READ_COUNTERS = ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum")
WRITE_COUNTERS = ("TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum")


def _per_dispatch(vals: dict, kernel: str, counter: str) -> float:
    xs = [v for n in _match(vals, kernel) for v in vals[n].get(counter, [])]
    if not xs:
        raise KeyError(f"no {counter} values for {kernel}")
    return sum(xs) / len(xs)


def reqs_summary(read_dir: str, write_dir: str, kernel: str):
    """Bytes per dispatch of `kernel` and of the copy kernel from the request counters by size."""
    r = counter_values(read_dir)
    w = counter_values(write_dir)
    out = {}
    for name in (kernel, COPY_KERNEL):
        n32, n64, n128 = (_per_dispatch(r, name, c) for c in READ_COUNTERS)
        wr, wr64 = (_per_dispatch(w, name, c) for c in WRITE_COUNTERS)
        out[name] = {"rd32": n32, "rd64": n64, "rd128": n128, "wr": wr, "wr64": wr64,
                     "read_bytes": 32 * n32 + 64 * n64 + 128 * n128, "write_bytes": 64 * wr64 + 32 * (wr - wr64)}
        out[name]["bytes"] = out[name]["read_bytes"] + out[name]["write_bytes"]
    return out


def _cmd_reqs(a):
    s = reqs_summary(a.read_dir, a.write_dir, a.kernel)
    sha = kernel_source_hash()
    k, c = s[a.kernel], s[COPY_KERNEL]
    print(f"# {a.title}\n")
    print("Commands (run from the repository root on one MI355X, one counter pass per run):\n")
    print("```\n" + a.command + "\n```\n")
    print(f"Kernel: names containing `{a.kernel}`; kernel source hash `{sha}`.\n")
    print("L2-to-fabric requests per dispatch by size, and the bytes they carry:\n")
    print("| kernel | 32 B reads | 64 B reads | 128 B reads | write requests (64 B of them) | read bytes | write bytes |")
    print("|---|---|---|---|---|---|---|")
    for name, x in ((a.kernel, k), ("copy_kernel (1 GiB each way)", c)):
        print(f"| `{name}` | {x['rd32']:.4g} | {x['rd64']:.4g} | {x['rd128']:.4g} | {x['wr']:.4g} ({x['wr64']:.4g}) | "
              f"{x['read_bytes']:.4e} | {x['write_bytes']:.4e} |")
    print(f"\nHBM traffic per launch of the kernel (reads + writes): **{k['bytes']:.4e} bytes**; "
          f"the copy kernel reads {c['read_bytes'] / 2**30:.3f} GiB and writes {c['write_bytes'] / 2**30:.3f} GiB.")
    if a.json:
        d = {}
        if os.path.exists(a.json):
            with open(a.json) as fh:
                d = json.load(fh)
        d.setdefault(a.workload, {})[a.kernel_class] = {
            "kernel_sha": sha, "bytes_per_launch": k["bytes"], "read_bytes_per_launch": k["read_bytes"],
            "write_bytes_per_launch": k["write_bytes"], "read_requests": {"32": k["rd32"], "64": k["rd64"],
                                                                          "128": k["rd128"]},
            "copy_check_read_gib": c["read_bytes"] / 2**30, "copy_check_write_gib": c["write_bytes"] / 2**30,
            "kernel": a.kernel, "counters": "TCC_EA0_RDREQ_{32B,64B,128B}, TCC_EA0_WRREQ{,_64B}"}
        with open(a.json, "w") as fh:
            json.dump(d, fh, indent=1, sort_keys=True)


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
    q = sub.add_parser("reqs")
    q.add_argument("read_dir")
    q.add_argument("write_dir")
    q.add_argument("--kernel", required=True)
    q.add_argument("--workload", required=True)
    q.add_argument("--kernel-class", required=True)
    q.add_argument("--title", required=True)
    q.add_argument("--command", required=True)
    q.add_argument("--json")
    a = ap.parse_args(argv)
    {"trace": _cmd_trace, "pmc": _cmd_pmc, "reqs": _cmd_reqs}[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
