"""HBM traffic of one kernel from two rocprofv3 counter runs.

`FETCH_SIZE` and `WRITE_SIZE` (KiB per dispatch) are collected in separate
`rocprofv3 --pmc` runs of the same command.  The command first runs one plain
device copy of a known size; what the counters read for that copy, divided by
the bytes it really moves, calibrates each counter.  The kernel's traffic per
launch is then (FETCH / f_fetch + WRITE / f_write), averaged over its
dispatches.

The summary written here records a hash of the library sources; the bench
reports the traffic only while the sources still hash the same (a changed
kernel needs new counters).

    python -m paper_2010_10232_amd.profiling --fetch F.csv --write W.csv \\
        --kernel arnoldi_reg_kernel --copy-mib 256 --workload NAME \\
        --command "..." --out profiles/<kernel>_<workload>_traffic.md

With --stats it turns a rocprofv3 --stats kernel summary into a markdown table.
"""
import argparse
import csv
import hashlib
import os
import re
import shutil
import subprocess

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def source_hash(files=None):
    """sha256 over library sources (name and contents, sorted by name): the given
    files of csrc/ (those that define the profiled kernel), or all of them."""
    h = hashlib.sha256()
    names = sorted(files) if files else sorted(n for n in os.listdir(CSRC) if n.endswith((".hip", ".h", ".cpp")))
    for name in names:
        h.update(name.encode())
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _per_kernel(path, counter, grid=None):
    """Counter values per kernel name; with grid, only dispatches of that grid size
    (one level's launches of a kernel that also runs on other levels) and the
    calibration copy."""
    out = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            if grid is not None and int(r["Grid_Size"]) != grid and "copy" not in r["Kernel_Name"].lower():
                continue
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def _copy_value(vals):
    """The calibration copy: the largest copy-kernel dispatch of the run."""
    vs = [v for name, lst in vals.items() if "copy" in name.lower() for v in lst]
    if not vs:
        raise SystemExit("no copy dispatch in the counter file")
    return max(vs)


def summarize(fetch_csv, write_csv, kernel, copy_mib, grid=None):
    fv = _per_kernel(fetch_csv, "FETCH_SIZE", grid)
    wv = _per_kernel(write_csv, "WRITE_SIZE", grid)
    copy_kib = copy_mib * 1024.0
    f_fetch = _copy_value(fv) / copy_kib
    f_write = _copy_value(wv) / copy_kib
    pat = re.compile(kernel)
    fk = [v for name, vs in fv.items() if pat.search(name) for v in vs]
    wk = [v for name, vs in wv.items() if pat.search(name) for v in vs]
    if not fk or not wk:
        raise SystemExit(f"kernel {kernel!r} not in the counter files")
    fetch = sum(fk) / len(fk)
    write = sum(wk) / len(wk)
    traffic = 1024.0 * (fetch / f_fetch + write / f_write)
    return dict(fetch_kib=fetch, write_kib=write, n_fetch=len(fk), n_write=len(wk), f_fetch=f_fetch,
                f_write=f_write, traffic=traffic)


def write_summary(out, kernel, workload, command, s, sources=None):
    lines = [
        f"# HBM traffic of `{kernel}` on {workload}",
        "",
        "Commands (repository root on the GPU host; one counter per run):",
        "",
        "```",
        command,
        "```",
        "",
        "| quantity | value |",
        "|---|---|",
        f"| FETCH_SIZE per launch (KiB, mean of {s['n_fetch']}) | {s['fetch_kib']:.1f} |",
        f"| WRITE_SIZE per launch (KiB, mean of {s['n_write']}) | {s['write_kib']:.1f} |",
        f"| copy calibration: FETCH_SIZE / true bytes | {s['f_fetch']:.4f} |",
        f"| copy calibration: WRITE_SIZE / true bytes | {s['f_write']:.4f} |",
        f"| traffic per launch (bytes) | {s['traffic']:.0f} |",
    ]
    if s.get("grid"):
        lines.append(f"| dispatches counted | grid size {s['grid']} threads only |")
    lines += [
        "",
        f"traffic_bytes_per_launch: {s['traffic']:.0f}",
        f"kernel_regex: {kernel}",
        f"sources: {','.join(sorted(sources)) if sources else 'all'}",
        f"source_sha256: {source_hash(sources)}",
        "",
    ]
    with open(out, "w") as fh:
        fh.write("\n".join(lines))


def read_summary(path):
    """(traffic bytes per launch, kernel regex) if the summary matches the current sources, else None."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            m = re.match(r"^(traffic_bytes_per_launch|kernel_regex|sources|source_sha256): (.+)$", line.strip())
            if m:
                vals[m.group(1)] = m.group(2)
    files = None if vals.get("sources", "all") == "all" else vals["sources"].split(",")
    if vals.get("source_sha256") != source_hash(files) or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"]), vals.get("kernel_regex")


def stats_from_trace(trace_csv, after, exclude=None):
    """Rows in the form of a rocprofv3 --stats summary, built from a kernel trace
    and counting only the dispatches that start after the last one whose name
    matches the regular expression `after` (one phase of a run), without those
    matching `exclude` (for instance a set-up that falls inside the phase)."""
    with open(trace_csv) as fh:
        tr = sorted(csv.DictReader(fh), key=lambda r: int(r["Start_Timestamp"]))
    pat = re.compile(after)
    skip = re.compile(exclude) if exclude else None
    last = max((i for i, r in enumerate(tr) if pat.search(r["Kernel_Name"])), default=-1)
    per = {}
    for r in tr[last + 1:]:
        if skip and skip.search(r["Kernel_Name"]):
            continue
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        per.setdefault(r["Kernel_Name"], []).append(d)
    total = sum(sum(v) for v in per.values()) or 1
    rows = [{"Name": name, "Calls": str(len(v)), "TotalDurationNs": str(sum(v)),
             "AverageNs": str(sum(v) / len(v)), "MinNs": str(min(v)), "MaxNs": str(max(v)),
             "Percentage": str(100.0 * sum(v) / total)} for name, v in per.items()]
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    return rows


def grid_rows(trace_csv, after, kernel):
    """Launch durations of the kernels matching `kernel`, split by launch shape
    (one row per kernel name and grid: the levels of a multilevel solve), over the
    dispatches after the last one matching `after`; largest grid first."""
    with open(trace_csv) as fh:
        tr = sorted(csv.DictReader(fh), key=lambda r: int(r["Start_Timestamp"]))
    pat, kpat = re.compile(after), re.compile(kernel)
    last = max((i for i, r in enumerate(tr) if pat.search(r["Kernel_Name"])), default=-1)
    per = {}
    for r in tr[last + 1:]:
        if not kpat.search(r["Kernel_Name"]):
            continue
        wg = max(1, int(r["Workgroup_Size_X"]) * int(r.get("Workgroup_Size_Y") or 1) * int(r.get("Workgroup_Size_Z") or 1))
        grid = int(r["Grid_Size_X"]) * int(r.get("Grid_Size_Y") or 1) * int(r.get("Grid_Size_Z") or 1)
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        per.setdefault((r["Kernel_Name"], grid // wg, wg), []).append(d)
    rows = []
    for (name, wgs, wg), v in per.items():
        v.sort()
        rows.append({"name": name, "workgroups": wgs, "wg_size": wg, "calls": len(v), "avg_us": sum(v) / len(v),
                     "median_us": v[len(v) // 2], "min_us": v[0], "max_us": v[-1]})
    rows.sort(key=lambda r: (-r["workgroups"], r["name"]))
    return rows


def write_grid_table(rows, title, command, out):
    lines = [f"# {title}", "", "Command (repository root on the GPU host):", "", "```", command, "```", "",
             "| kernel | workgroups | threads each | calls | avg us | median us | min us | max us |",
             "|---|---|---|---|---|---|---|---|"]
    for r in rows:
        name = _demangle(r["name"]).replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        lines.append(f"| `{name}` | {r['workgroups']} | {r['wg_size']} | {r['calls']} | {r['avg_us']:.2f} | "
                     f"{r['median_us']:.2f} | {r['min_us']:.2f} | {r['max_us']:.2f} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def _demangle(name):
    """Readable form of a mangled kernel name: c++filt when installed and able,
    else the nested name of `_ZN<len><id>...` with `<...>` for template arguments."""
    if not name.startswith("_Z"):
        return name
    if shutil.which("c++filt") is not None:
        r = subprocess.run(["c++filt", name], capture_output=True, text=True)
        out = r.stdout.strip()
        if out and out != name:
            return out
    if not name.startswith("_ZN"):
        return name
    parts, pos = [], 3
    while pos < len(name) and name[pos].isdigit():
        end = pos
        while name[end].isdigit():
            end += 1
        k = int(name[pos:end])
        parts.append(name[end:end + k])
        pos = end + k
    if not parts:
        return name
    return "::".join(parts) + ("<...>" if name[pos:pos + 1] == "I" else "")


def write_stats(stats_csv, title, command, out, top=18, rows=None):
    """Markdown table of a rocprofv3 --stats kernel summary (most device time
    first); rows given directly (stats_from_trace) instead of the file."""
    if rows is None:
        with open(stats_csv) as fh:
            rows = list(csv.DictReader(fh))
    lines = [f"# {title}", "", "Command (repository root on the GPU host):", "", "```", command, "```", "",
             "| kernel | calls | total ms | avg us | min us | max us | % of GPU time |",
             "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = _demangle(r["Name"]).replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        if len(name) > 72:
            name = name[:72] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    rest = rows[top:]
    if rest:
        lines.append(f"| ({len(rest)} more kernels) | {sum(int(r['Calls']) for r in rest)} | "
                     f"{sum(float(r['TotalDurationNs']) for r in rest) / 1e6:.3f} | | | | "
                     f"{sum(float(r['Percentage']) for r in rest):.2f} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", help="rocprofv3 kernel_stats.csv: write a kernel table instead")
    ap.add_argument("--trace", help="rocprofv3 kernel_trace.csv: write a kernel table of the dispatches after --after")
    ap.add_argument("--after", help="regular expression: the table starts after its last dispatch")
    ap.add_argument("--exclude", help="regular expression: kernels left out of the --trace table")
    ap.add_argument("--per-grid", action="store_true",
                    help="with --trace and --kernel: one row per launch shape of the matching kernels")
    ap.add_argument("--title")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--kernel", help="regular expression matching the kernel name")
    ap.add_argument("--grid", type=int, help="only dispatches of this grid size (threads)")
    ap.add_argument("--copy-mib", type=float)
    ap.add_argument("--sources", help="comma-separated csrc/ files that define the kernel (hash scope)")
    ap.add_argument("--workload")
    ap.add_argument("--command", required=True)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.stats:
        write_stats(a.stats, a.title or "Kernel statistics", a.command, a.out)
        return
    if a.trace and a.per_grid:
        write_grid_table(grid_rows(a.trace, a.after or "^$", a.kernel or "."), a.title or "Launches by shape",
                         a.command, a.out)
        return
    if a.trace:
        write_stats(None, a.title or "Kernel statistics", a.command, a.out,
                    rows=stats_from_trace(a.trace, a.after or "^$", a.exclude))
        return
    s = summarize(a.fetch, a.write, a.kernel, a.copy_mib, a.grid)
    s["grid"] = a.grid
    write_summary(a.out, a.kernel, a.workload, a.command, s, a.sources.split(",") if a.sources else None)
    print(s)


if __name__ == "__main__":
    main()
