"""Summaries of rocprofv3 output for the amplitude kernel.

HBM traffic of a kernel comes from two counter passes over the same command,
one collecting FETCH_SIZE and one WRITE_SIZE (both in KiB per dispatch).  The
same command also runs a plain device copy of known size (bench.py
--copy-calibration: an element-wise negation of 256 MiB of float32), so each
counter is scaled by bytes_known / counter_of_copy; the scaled figures are
HBM bytes per launch of the kernel.

    python -m paper_0908_4403_amd.profiling traffic \\
        --fetch run_fetch/counter_collection.csv --write run_write/counter_collection.csv \\
        --kernel "me2_kernel<float,4,4,16,2,1>" --out profiles/NAME.md --command "..."

    python -m paper_0908_4403_amd.profiling trace --trace kernel_trace.csv \\
        --out profiles/NAME.md --command "..." [--title "..."]

    python -m paper_0908_4403_amd.profiling issue --pmc passA/ passB/ ... \\
        --out profiles/NAME.md --command "..." [--title "..."]

The issue summary averages every SQ counter per dispatch (largest grid of
each kernel) and relates VALU issue to that of the FMA probe kernel, which
issues one VALU instruction in every cycle it can.

The traffic summary records a digest of the device sources (csrc/); a
consumer treats the figure as stale (None) once the sources differ.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
CALIB_BYTES = 256 << 20     # bytes read and bytes written by the calibration copy
CALIB_KERNEL = "neg_kernel"  # substring of the calibration kernel's name


def source_digest() -> str:
    """sha256 over the device and launcher sources, in name order."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(CSRC, "*"))):
        if os.path.splitext(path)[1] in (".hip", ".hpp", ".cpp", ".h"):
            h.update(os.path.basename(path).encode())
            with open(path, "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def short_name(kernel: str) -> str:
    """'void heget::me2_kernel<float, 4, 4, 16, 2, 1>(double const*, ...)' -> 'me2_kernel<float,4,4,16,2,1>'."""
    k = kernel.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").replace(" ", "")
    return k[len("heget::"):] if k.startswith("heget::") else k


def _find_csv(path: str, suffix: str) -> str:
    if os.path.isdir(path):
        hits = sorted(glob.glob(os.path.join(path, "**", "*" + suffix), recursive=True))
        if not hits:
            raise FileNotFoundError(f"no *{suffix} under {path}")
        return hits[0]
    return path


def read_counters(path: str):
    """Rows of a rocprofv3 counter_collection.csv as (kernel, grid, counter, value)."""
    out = []
    with open(_find_csv(path, "counter_collection.csv"), newline="") as f:
        for row in csv.DictReader(f):
            out.append((row.get("Kernel_Name", ""), int(float(row.get("Grid_Size", 0) or 0)),
                        row.get("Counter_Name", ""), float(row.get("Counter_Value", 0) or 0)))
    return out


def per_dispatch(rows, counter: str, match):
    """Values of `counter` for dispatches whose short kernel name satisfies match()."""
    return [(g, v) for k, g, c, v in rows if c == counter and match(short_name(k), k)]


def traffic(fetch_csv: str, write_csv: str, kernel: str):
    """HBM bytes per launch of `kernel` (largest grid among its dispatches)."""
    fr, wr = read_counters(fetch_csv), read_counters(write_csv)
    want = kernel.replace(" ", "")

    def is_kernel(s, full):
        return s == want

    def is_calib(s, full):
        return CALIB_KERNEL in full

    out = {}
    for name, rows, counter in (("fetch", fr, "FETCH_SIZE"), ("write", wr, "WRITE_SIZE")):
        cal = [v for g, v in per_dispatch(rows, counter, is_calib)]
        ker = per_dispatch(rows, counter, is_kernel)
        if not cal or not ker:
            raise ValueError(f"{counter}: calibration dispatches {len(cal)}, kernel dispatches {len(ker)}")
        gmax = max(g for g, _ in ker)
        vals = [v for g, v in ker if g == gmax]
        cal_kib = max(cal)
        scale = CALIB_BYTES / (cal_kib * 1024.0)
        out[name] = {"kib_per_launch": sum(vals) / len(vals), "launches": len(vals), "grid": gmax,
                     "calib_kib": cal_kib, "scale": scale,
                     "bytes_per_launch": sum(vals) / len(vals) * 1024.0 * scale}
    out["bytes_per_launch"] = out["fetch"]["bytes_per_launch"] + out["write"]["bytes_per_launch"]
    return out


def traffic_markdown(kernel: str, t: dict, command: str, title: str) -> str:
    f, w = t["fetch"], t["write"]
    return "\n".join([
        f"# {title}",
        "",
        "Commands (on the MI355X host, from the repository root):",
        "",
        "    " + command,
        "",
        f"Calibration: element-wise negation of {CALIB_BYTES >> 20} MiB float32 "
        f"(reads and writes {CALIB_BYTES >> 20} MiB each).",
        "",
        "| counter | kernel KiB/launch | launches | grid | copy KiB | scale | HBM bytes/launch |",
        "|---|---|---|---|---|---|---|",
        f"| FETCH_SIZE | {f['kib_per_launch']:.0f} | {f['launches']} | {f['grid']} | {f['calib_kib']:.0f} "
        f"| {f['scale']:.4f} | {f['bytes_per_launch']:.4e} |",
        f"| WRITE_SIZE | {w['kib_per_launch']:.0f} | {w['launches']} | {w['grid']} | {w['calib_kib']:.0f} "
        f"| {w['scale']:.4f} | {w['bytes_per_launch']:.4e} |",
        "",
        f"kernel: {kernel}",
        f"hbm_bytes_per_launch: {t['bytes_per_launch']:.6e}",
        f"source_digest: {source_digest()}",
        "",
    ])


def read_traffic(md_path: str, kernel: str):
    """HBM bytes per launch from a traffic summary, or None if absent, for
    another kernel, or taken on other sources."""
    if not os.path.exists(md_path):
        return None
    text = open(md_path).read()
    k = re.search(r"^kernel: (\S+)$", text, re.M)
    b = re.search(r"^hbm_bytes_per_launch: (\S+)$", text, re.M)
    d = re.search(r"^source_digest: (\S+)$", text, re.M)
    if not (k and b and d) or k.group(1) != kernel.replace(" ", "") or d.group(1) != source_digest():
        return None
    return float(b.group(1))


PROBE_KERNEL = "fma_peak_kernel<float>"
ISSUE_KERNELS = ("me2_kernel", "gen_kernel", "compact_kernel", "final_kernel", "fma_peak_kernel")


def issue(pmc_dirs):
    """{short kernel name: {counter: mean per dispatch}} over the given counter
    passes, for the largest-grid dispatches of the kernels of the path."""
    sums = {}
    for d in pmc_dirs:
        rows = read_counters(d)
        gmax = {}
        for k, g, c, v in rows:
            s = short_name(k)
            if s.split("<")[0] in ISSUE_KERNELS:
                gmax[s] = max(gmax.get(s, 0), g)
        for k, g, c, v in rows:
            s = short_name(k)
            if s in gmax and g == gmax[s]:
                t = sums.setdefault(s, {}).setdefault(c, [0.0, 0])
                t[0] += v
                t[1] += 1
    return {k: {c: t[0] / t[1] for c, t in cs.items()} for k, cs in sums.items()}


def issue_markdown(stats: dict, command: str, title: str) -> str:
    counters = sorted({c for cs in stats.values() for c in cs})
    probe = stats.get(PROBE_KERNEL, {})

    def ratio(cs, a, b):
        return cs[a] / cs[b] if a in cs and cs.get(b) else None

    ref = ratio(probe, "SQ_ACTIVE_INST_VALU", "SQ_BUSY_CYCLES")
    lines = [f"# {title}", "", "Commands (on the MI355X host, from the repository root):", "", "    " + command, "",
             "Mean per dispatch (largest launch of each kernel). VALU issue = (SQ_ACTIVE_INST_VALU / "
             f"SQ_BUSY_CYCLES) relative to `{PROBE_KERNEL}`, the FMA probe; waits are shares of "
             "SQ_WAVE_CYCLES.", "",
             "| kernel | VALU instr per wave | VALU issue | SQ_WAIT_INST_ANY | SQ_WAIT_ANY |",
             "|---|---|---|---|---|"]
    fmt = lambda x, f: "-" if x is None else f.format(x)
    for k in sorted(stats):
        cs = stats[k]
        per_wave = ratio(cs, "SQ_INSTS_VALU", "SQ_WAVES")
        r = ratio(cs, "SQ_ACTIVE_INST_VALU", "SQ_BUSY_CYCLES")
        lines.append(f"| `{k}` | {fmt(per_wave, '{:.0f}')} | "
                     f"{fmt(r / ref if r is not None and ref else None, '{:.1%}')} | "
                     f"{fmt(ratio(cs, 'SQ_WAIT_INST_ANY', 'SQ_WAVE_CYCLES'), '{:.1%}')} | "
                     f"{fmt(ratio(cs, 'SQ_WAIT_ANY', 'SQ_WAVE_CYCLES'), '{:.1%}')} |")
    lines += ["", "Raw means per dispatch:", "",
              "| kernel | " + " | ".join(counters) + " |", "|---|" + "---|" * len(counters)]
    for k in sorted(stats):
        lines.append(f"| `{k}` | " + " | ".join(fmt(stats[k].get(c), "{:.4g}") for c in counters) + " |")
    return "\n".join(lines) + "\n"


def trace_markdown(trace_csv: str, command: str, title: str, top: int = 14) -> str:
    """Per-(kernel, grid) statistics of a rocprofv3 --kernel-trace run
    (kernel_trace.csv), so launches of one kernel at different sizes (the
    autotuner's, the timed steps') are not averaged together."""
    groups = {}
    with open(_find_csv(trace_csv, "kernel_trace.csv"), newline="") as f:
        for r in csv.DictReader(f):
            grid = int(r.get("Grid_Size_X") or r.get("Grid_Size") or 0)
            dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            groups.setdefault((short_name(r["Kernel_Name"]), grid), []).append(dur)
    total = sum(sum(v) for v in groups.values()) or 1.0
    rows = sorted(groups.items(), key=lambda kv: -sum(kv[1]))
    lines = [f"# {title}", "", "Command (on the MI355X host, from the repository root):", "", "    " + command, "",
             "Durations in microseconds, per kernel and launch size (grid = threads).", "",
             "| kernel | grid | calls | total us | average us | min us | max us | % |",
             "|---|---|---|---|---|---|---|---|"]
    for (name, grid), d in rows[:top]:
        lines.append(f"| `{name}` | {grid} | {len(d)} | {sum(d):.1f} | {sum(d) / len(d):.1f} | "
                     f"{min(d):.1f} | {max(d):.1f} | {100 * sum(d) / total:.1f} |")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_0908_4403_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--title", default="HBM traffic of the amplitude kernel")
    s = sub.add_parser("trace")
    s.add_argument("--trace", required=True, help="kernel_trace.csv or the folder holding it")
    s.add_argument("--out", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="rocprofv3 kernel trace")
    i = sub.add_parser("issue")
    i.add_argument("--pmc", nargs="+", required=True, help="counter_collection.csv files or folders")
    i.add_argument("--out", required=True)
    i.add_argument("--command", required=True)
    i.add_argument("--title", default="rocprofv3 SQ counters of the path's kernels")
    a = ap.parse_args(argv)
    if a.cmd == "issue":
        text = issue_markdown(issue(a.pmc), a.command, a.title)
    elif a.cmd == "traffic":
        tr = traffic(a.fetch, a.write, a.kernel)
        text = traffic_markdown(a.kernel.replace(" ", ""), tr, a.command, a.title)
    else:
        text = trace_markdown(a.trace, a.command, a.title)
    with open(a.out, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    sys.exit(main())
