"""Summaries of rocprofv3 output (kernel-trace statistics and HBM counters).

Used by hand after a profiling run:

    python -m paper_1910_08535_amd.profiling stats  <kernel_stats.csv> <out.md> "<command>"
        [<per launch shape csv>]
    python -m paper_1910_08535_amd.profiling grid <kernel_trace.csv> <per launch shape csv>
    python -m paper_1910_08535_amd.profiling traffic <fetch_counter_collection.csv>
        <write_counter_collection.csv> <kernel substring> <copy MiB> <workload> "<commands>"
    python -m paper_1910_08535_amd.profiling pmc <out.md> <kernel substring> "<commands>"
        <counter_collection.csv> [...]

`traffic` scales each counter by what it reads for a plain copy of known size (the
torch copy kernel the benchmark runs with --copy-probe-mb), giving HBM bytes per launch
of the kernel, and writes profiles/traffic_<workload>.json stamped with the hash of the
sources of that kernel (bench.py reports the figure only while they are unchanged).
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# sources each profiled kernel is compiled from (its code and the types it uses)
KERNEL_SOURCES = {
    "apply2d": ("apply.hpp", "common.hpp"),
    "apply3d": ("apply3d.hpp", "apply.hpp", "common.hpp"),
    "batch2d": ("batch.hpp", "apply.hpp", "common.hpp"),
    "ads_seg": ("ads.hpp", "common.hpp"),
}


def kernel_source_hash(kernel: str = "apply2d") -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1910_08535_amd", "csrc")
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def stats_markdown(stats_csv: str, out_md: str, command: str, grid_csv: str = "") -> None:
    """rocprofv3 --stats summary; grid_csv (optional): per (kernel, grid size) call counts
    and average durations from the same run's kernel trace."""
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ["# rocprofv3 kernel statistics", "", "Command (from the repository root, after "
             "`cd /tmp && export TMPDIR=/tmp` as the profiler needs):", "", "```", command, "```",
             "", "| kernel | calls | average (us) | min (us) | max (us) | share |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.3f} | "
                     f"{float(r['MinNs']) / 1e3:.3f} | {float(r['MaxNs']) / 1e3:.3f} | "
                     f"{float(r['Percentage']):.1f}% |")
    lines.append("")
    if grid_csv:
        lines += ["Per launch shape (grid size in threads), from the same run's kernel trace:", "",
                  "| kernel | grid | calls | average (us) | min (us) | max (us) |", "|---|---|---|---|---|---|"]
        for r in csv.DictReader(open(grid_csv)):
            lines.append(f"| `{r['kernel'][:90]}` | {r['grid']} | {r['calls']} | "
                         f"{float(r['average_ns']) / 1e3:.3f} | {float(r['min_ns']) / 1e3:.3f} | "
                         f"{float(r['max_ns']) / 1e3:.3f} |")
        lines.append("")
    for k in KERNEL_SOURCES:
        lines.append(f"Sources hash of {k} ({', '.join(KERNEL_SOURCES[k])}): `{kernel_source_hash(k)}`")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def grid_table(trace_csv: str, out_csv: str, keep=("apply2d", "apply3d", "batch2d", "copy2_kernel", "serve")) -> None:
    """Per (kernel, grid size) call counts and durations of a rocprofv3 --kernel-trace CSV,
    for the kernels whose names contain one of `keep`, largest total time first."""
    d = {}
    for r in csv.DictReader(open(trace_csv)):
        if any(k in r["Kernel_Name"] for k in keep):
            g = r.get("Grid_Size", r.get("Grid_Size_X"))
            d.setdefault((r["Kernel_Name"], g), []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    with open(out_csv, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["kernel", "grid", "calls", "average_ns", "min_ns", "max_ns"])
        for (n, g), v in sorted(d.items(), key=lambda x: -sum(x[1])):
            w.writerow([n, g, len(v), sum(v) / len(v), min(v), max(v)])


def _per_dispatch(csv_path: str, counter: str, grid: str = ""):
    """Counter values per kernel name, of the dispatches with that grid size if given."""
    vals = {}
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] != counter or (grid and r["Grid_Size"] != grid):
            continue
        vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return vals


def _probe_value(csv_path: str, counter: str, first: int = 8) -> float:
    """The counter of the copy probe: the largest value among the copy dispatches in the
    first `first` dispatches of the run (bench.py --copy-probe-mb runs the probe before
    anything else; later copies or fills of other sizes are not it)."""
    rows = [r for r in csv.DictReader(open(csv_path)) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    vals = [float(r["Counter_Value"]) for r in rows[:first] if "copy" in r["Kernel_Name"].lower()]
    if not vals:
        raise SystemExit(f"no copy dispatch among the first {first} of {csv_path}")
    return max(vals)


def _family(kernel: str) -> str:
    for k in KERNEL_SOURCES:
        if k in kernel:
            return k
    raise SystemExit(f"no source list for kernel {kernel!r}")


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_mib: float, workload: str,
            commands: str, out_dir: str = "") -> dict:
    """HBM bytes per launch of `kernel` ("name" or "name@grid size", the grid size in
    threads picking one launch shape of a kernel that runs at several; without one, the
    shape most dispatches have), written to traffic_<workload>.json in out_dir (default
    profiles/)."""
    kernel, _, grid = kernel.partition("@")
    grid = grid or _common_grid([fetch_csv], kernel)
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE", grid)
    write = _per_dispatch(write_csv, "WRITE_SIZE", grid)

    def pick(vals, needle):
        keys = [k for k in vals if needle in k]
        if not keys:
            raise SystemExit(f"no kernel matching {needle!r} in {list(vals)[:5]}")
        return keys[0], vals[keys[0]]

    copy_bytes = copy_mib * 2**20
    cf = _probe_value(fetch_csv, "FETCH_SIZE")
    cw = _probe_value(write_csv, "WRITE_SIZE")
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    kf, fv = pick(fetch, kernel)
    kw, wv = pick(write, kernel)
    fb = statistics.median(fv) * 1024.0 * f_scale
    wb = statistics.median(wv) * 1024.0 * w_scale
    rec = {"workload": workload, "kernel": kf, "grid_size": grid, "dispatches": [len(fv), len(wv)],
           "fetch_kib_per_dispatch_median": statistics.median(fv),
           "write_kib_per_dispatch_median": statistics.median(wv),
           "copy_probe_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_scale": f_scale, "write_scale": w_scale,
           "bytes_per_launch": fb + wb, "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
           "family": _family(kernel), "kernel_source_hash": kernel_source_hash(_family(kernel)),
           "commands": commands}
    out = os.path.join(out_dir or os.path.join(ROOT, "profiles"), f"traffic_{workload}.json")
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


# counters summed over the device per dispatch, and what each ratio below means
_RATIOS = (
    ("VALU instructions per wave", "SQ_INSTS_VALU", "SQ_WAVES"),
    ("FP64 FMA instructions per wave", "SQ_INSTS_VALU_FMA_F64", "SQ_WAVES"),
    ("LDS instructions per wave", "SQ_INSTS_LDS", "SQ_WAVES"),
    ("vector memory instructions per wave", "SQ_INSTS_VMEM", "SQ_WAVES"),
    ("scalar ALU instructions per wave", "SQ_INSTS_SALU", "SQ_WAVES"),
    ("share of wave time waiting on a dependency (s_waitcnt)", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES"),
    ("share of wave time waiting for anything", "SQ_WAIT_ANY", "SQ_WAVE_CYCLES"),
    ("share of wave time issuing VALU", "SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES"),
)


def _common_grid(csvs, kernel: str) -> str:
    """The grid size (threads) most dispatches of the kernels matching `kernel` have."""
    seen = {}
    for path in csvs:
        for r in csv.DictReader(open(path)):
            if kernel in r["Kernel_Name"]:
                seen.setdefault(r["Grid_Size"], set()).add(r["Dispatch_Id"])
    if not seen:
        raise SystemExit(f"no dispatch of a kernel matching {kernel!r}")
    return max(seen, key=lambda g: len(seen[g]))


def pmc_markdown(out_md: str, kernel: str, command: str, csvs) -> dict:
    """Median per dispatch of every counter collected for the kernels matching `kernel`
    ("name" or "name@grid size"; without a grid size, the launch shape most dispatches
    have) in rocprofv3 --pmc CSV files (one per pass), and the ratios above."""
    kernel, _, grid = kernel.partition("@")
    grid = grid or _common_grid(csvs, kernel)
    vals = {}
    name = None
    for path in csvs:
        for r in csv.DictReader(open(path)):
            if kernel not in r["Kernel_Name"] or r["Grid_Size"] != grid:
                continue
            name = r["Kernel_Name"]
            vals.setdefault(r["Counter_Name"], {}).setdefault(r["Dispatch_Id"], 0.0)
            vals[r["Counter_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
    if not vals:
        raise SystemExit(f"no dispatch of a kernel matching {kernel!r}")
    med = {c: statistics.median(d.values()) for c, d in vals.items()}
    lines = ["# rocprofv3 counters", "", f"Kernel: `{name}`, grid of {grid} threads", "",
             "Commands (from the repository root, after `cd /tmp && export TMPDIR=/tmp` as the "
             "profiler needs), one per pass:", "", "```", command, "```", "",
             "| counter | median per dispatch | dispatches |", "|---|---|---|"]
    for c in sorted(med):
        lines.append(f"| {c} | {med[c]:.6g} | {len(vals[c])} |")
    lines += ["", "| ratio | value |", "|---|---|"]
    ratios = {}
    for label, a, b in _RATIOS:
        if a in med and b in med and med[b] > 0:
            ratios[label] = med[a] / med[b]
            lines.append(f"| {label} ({a} / {b}) | {ratios[label]:.4g} |")
    fam = [k for k in KERNEL_SOURCES if k in name]
    if fam:
        lines += ["", f"Sources hash of {fam[0]} ({', '.join(KERNEL_SOURCES[fam[0]])}): "
                      f"`{kernel_source_hash(fam[0])}`"]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return {"median": med, "ratios": ratios}


if __name__ == "__main__":
    if sys.argv[1] == "pmc":
        print(json.dumps(pmc_markdown(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5:]), indent=1))
    elif sys.argv[1] == "stats":
        stats_markdown(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5] if len(sys.argv) > 5 else "")
    elif sys.argv[1] == "grid":   # grid TRACE_CSV OUT_CSV [comma-separated name parts to keep]
        if len(sys.argv) > 4:
            grid_table(sys.argv[2], sys.argv[3], tuple(sys.argv[4].split(",")))
        else:
            grid_table(sys.argv[2], sys.argv[3])
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], sys.argv[4], float(sys.argv[5]),
                                 sys.argv[6], sys.argv[7]), indent=1))
    else:
        raise SystemExit(__doc__)
