"""Summaries of rocprofv3 runs for profiles/, and the figures bench.py reads
back from them.

A summary is a short Markdown file: the commands that made it, a table of
kernel times, and a block of ``key = value`` lines with the figures the
benchmark uses for its roofline (HBM traffic, VALU and LDS instructions per
launch of the kernel it times).  It also records a hash of the kernel sources
it was measured with, so the benchmark reports those figures only while the
kernel is unchanged.

Build one from the CSV directories of four rocprofv3 runs (kernel trace, then
FETCH_SIZE, WRITE_SIZE and one or more sets of SQ counters, each in a run of
its own):

    python -m paper_0912_4506_amd.profiling --kernel 'tblock_kernel<double, 4, 1, 6, 12, 0>' \\
        --trace DIR --fetch DIR --write DIR --sq DIR --title '...' --command '...' \\
        --out profiles/NAME.md

HBM bytes come from FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by
what the same counters read for the library's copy kernel, whose bytes are
known (the benchmark measures the copy bandwidth in the same process).
"""
import argparse
import csv
import glob
import hashlib
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# sources that decide the code of the blocked kernels and the sweep kernels
KERNEL_SOURCES = ["csrc/tblock.h", "csrc/device_common.h", "csrc/kernels.h", "csrc/kernels.hip",
                  "csrc/tb_plain_f64.hip", "csrc/tb_plain_f32.hip", "csrc/tb_batch_f64.hip",
                  "csrc/tb_comp_f64.hip", "csrc/lbm.hip", "csrc/build.py"]


def kernel_source_hash():
    """Hash of the kernel sources (16 hex digits)."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        path = os.path.join(HERE, rel)
        h.update(rel.encode())
        if os.path.exists(path):
            with open(path, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def _rows(directory, suffix):
    rows = []
    for path in sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True)):
        with open(path, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    if not rows:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    return rows


def kernel_times(directory):
    """{kernel name: [duration in us, ...]} from a --kernel-trace run."""
    out = {}
    for r in _rows(directory, "kernel_trace.csv"):
        dt = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        out.setdefault(r["Kernel_Name"], []).append(dt)
    return out


def counters(directory):
    """{kernel name: {counter: [value per dispatch, ...]}} from a --pmc run
    (rows of one dispatch and counter are summed)."""
    per = {}
    for r in _rows(directory, "counter_collection.csv"):
        key = (r["Kernel_Name"], r.get("Dispatch_Id") or r.get("Correlation_Id"), r["Counter_Name"])
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    out = {}
    for (name, _, counter), v in per.items():
        out.setdefault(name, {}).setdefault(counter, []).append(v)
    return out


def _match(table, fragment):
    names = [n for n in table if fragment in n]
    if len(names) != 1:
        raise KeyError(f"{fragment!r} matches {len(names)} kernels: {names[:4]}")
    return names[0]


def median(v):
    return statistics.median(v)


def summarize(kernel, trace=None, fetch=None, write=None, sq=None, copy="jac::copy_kernel",
              copy_bytes=2 << 30):
    """Figures of `kernel` (a fragment of its name) from the run directories
    (sq: one directory of SQ/GRBM counter runs, or a list of them)."""
    fig = {"kernel_source_sha": kernel_source_hash()}
    if trace:
        times = kernel_times(trace)
        name = _match(times, kernel)
        fig.update(kernel=name, launches=len(times[name]), median_us=round(median(times[name]), 1),
                   mean_us=round(statistics.fmean(times[name]), 1),
                   min_us=round(min(times[name]), 1), max_us=round(max(times[name]), 1))
        fig["_times"] = times
    for label, d, counter in (("fetch", fetch, "FETCH_SIZE"), ("write", write, "WRITE_SIZE")):
        if not d:
            continue
        c = counters(d)
        name = _match(c, kernel)
        cname = _match(c, copy)
        kib = median(c[name][counter])
        copy_kib = median(c[cname][counter])
        scale = copy_bytes / 1024.0 / copy_kib
        fig[f"{label}_kib_per_launch"] = round(kib, 1)
        fig[f"{label}_scale"] = round(scale, 4)
        fig[f"{label}_gb_per_launch"] = round(kib * 1024.0 * scale / 1e9, 4)
    if "fetch_gb_per_launch" in fig and "write_gb_per_launch" in fig:
        fig["traffic_gb_per_launch"] = round(fig["fetch_gb_per_launch"] + fig["write_gb_per_launch"], 4)
    for d in ([sq] if isinstance(sq, str) else (sq or [])):
        c = counters(d)
        name = _match(c, kernel)
        for counter, vals in sorted(c[name].items()):
            fig[counter.lower() + "_per_launch"] = round(median(vals))
    return fig


def write_summary(path, fig, title, commands, notes=""):
    lines = [f"# {title}", "", "Commands (from the repository root):", ""]
    lines += ["    " + c for c in commands]
    times = fig.pop("_times", None)
    if times:
        lines += ["", "## Kernel times (rocprofv3 kernel trace)", "",
                  "| kernel | calls | median (us) | mean (us) | min (us) | max (us) |",
                  "|---|---|---|---|---|---|"]
        total = {k: sum(v) for k, v in times.items()}
        for k in sorted(total, key=total.get, reverse=True)[:8]:
            v = times[k]
            lines.append(f"| `{k}` | {len(v)} | {median(v):.1f} | {statistics.fmean(v):.1f} | "
                         f"{min(v):.1f} | {max(v):.1f} |")
    if notes:
        lines += ["", notes.strip()]
    lines += ["", "## Figures", "", "```"]
    lines += [f"{k} = {v}" for k, v in fig.items()]
    lines += ["```", ""]
    with open(path, "w") as fh:
        fh.write("\n".join(lines))


def read_figures(path):
    """The ``key = value`` figures of a summary (numbers as floats), or {}."""
    if not os.path.exists(path):
        return {}
    out, inside = {}, False
    with open(path) as fh:
        for line in fh:
            s = line.strip()
            if s == "## Figures":
                inside = True
                continue
            if inside and " = " in s:
                k, v = s.split(" = ", 1)
                try:
                    out[k] = float(v)
                except ValueError:
                    out[k] = v
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--sq", action="append", help="SQ counter run (repeatable)")
    ap.add_argument("--title", required=True)
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--notes", default="")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    fig = summarize(a.kernel, a.trace, a.fetch, a.write, a.sq)
    write_summary(a.out, fig, a.title, a.command, a.notes)
    print(a.out)


if __name__ == "__main__":
    main()
