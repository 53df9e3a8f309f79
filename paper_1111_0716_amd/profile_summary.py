"""Short text summaries of rocprofv3 output for the library's kernels.

  python -m paper_1111_0716_amd.profile_summary trace DIR --title T --command C [--out FILE]
      per-kernel calls / average / share from DIR/*_kernel_stats.csv
      (a `rocprofv3 --kernel-trace --stats --output-format csv` run)

  python -m paper_1111_0716_amd.profile_summary traffic --fetch DIR --write DIR
         --kernel SUBSTR --copy-bytes B --kind KIND --units-per-launch U
         --bytes-per-unit A --command C [--command C2] [--out FILE]
      HBM bytes per launch of the kernel whose name contains SUBSTR, from two
      `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs; each counter is scaled by
      the factor that makes the same counter read B bytes on the largest plain
      device-to-device copy (`__amd_rocclr_copyBuffer`) of the same run.

  python -m paper_1111_0716_amd.profile_summary counters DIR [DIR ...]
         --kernel SUBSTR --title T --command C [--command C2 ...] [--out FILE]
      every counter of the kernel whose name contains SUBSTR (mean over its
      dispatches after the first) from one or more `--pmc` runs, with the
      derived shares of wave time (VALU, LDS, waits) and the L2 hit rate

The traffic summary carries machine-readable lines (`key: value`) that
bench.py reads back; `sources_sha256` fingerprints the kernel's source files
so that a later change of the kernel voids the figure.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import shlex
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
# source files of each kernel kind's device code (the .hip file and the
# headers its kernels use)
KIND_SOURCES = {
    "fused": ["pair_fused.hip", "reg_fft.hpp", "fft_lds.hpp", "twiddle_ce.hpp"],
    "energy_fused": ["pair_fused.hip", "reg_fft.hpp", "fft_lds.hpp", "twiddle_ce.hpp"],
    "plane": ["kernels.hip", "pass_reg.hip", "reg_fft.hpp", "split_fft.hpp", "fft_lds.hpp", "twiddle_ce.hpp", "fock_internal.hpp"],
    "pencil": ["kernels.hip", "pass_reg.hip", "reg_fft.hpp", "split_fft.hpp", "fft_lds.hpp", "twiddle_ce.hpp", "fock_internal.hpp"],
    "accumulate": ["kernels.hip", "pass_reg.hip", "reg_fft.hpp", "split_fft.hpp", "fft_lds.hpp", "twiddle_ce.hpp", "fock_internal.hpp"],
    "energy_plane": ["kernels.hip", "pass_reg.hip", "reg_fft.hpp", "split_fft.hpp", "fft_lds.hpp", "twiddle_ce.hpp", "fock_internal.hpp"],
    "energy_pencil": ["kernels.hip", "pass_reg.hip", "reg_fft.hpp", "split_fft.hpp", "fft_lds.hpp", "twiddle_ce.hpp", "fock_internal.hpp"],
    "overlap": ["overlap_mfma.hip", "fft_lds.hpp", "fock_internal.hpp"],
}
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def sources_sha256(kind):
    h = hashlib.sha256()
    for name in KIND_SOURCES[kind]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def short_name(name, limit=100):
    """Kernel name without the argument list: `void ns::k<T, 32>(...)` ->
    `ns::k<T, 32>`; names longer than `limit` are cut (template arguments of
    other libraries' kernels run to kilobytes)."""
    name = re.sub(r"^void ", "", name).replace("(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            name = name[:i]
            break
    return name if len(name) <= limit else name[:limit] + " ..."


def _one(pattern):
    files = sorted(glob.glob(pattern, recursive=True))
    if not files:
        raise SystemExit(f"no file matches {pattern}")
    return files[0]


def read_kernel_stats(d):
    with open(_one(os.path.join(d, "**", "*kernel_stats.csv"))) as f:
        return list(csv.DictReader(f))


def read_counter(d, counter):
    """[(kernel name, value)] per dispatch, in dispatch order."""
    rows = []
    with open(_one(os.path.join(d, "**", "*counter_collection.csv"))) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    return [(k, v) for _, k, v in rows]


def trace_summary(d, title, command):
    rows = read_kernel_stats(d)
    out = [f"# {title}", "", "Command (from the repository root):", "", "```", command, "```", "",
           "| kernel | calls | average (ms) | min (ms) | max (ms) | share |", "|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                   f"{float(r['MinNs']) / 1e6:.3f} | {float(r['MaxNs']) / 1e6:.3f} | {float(r['Percentage']):.2f} % |")
    return "\n".join(out) + "\n"


def calibrated(d, counter, kernel, copy_bytes):
    """(scaled bytes per kernel dispatch, kernel dispatches, factor, copy KiB read)."""
    rows = read_counter(d, counter)
    copies = [v for k, v in rows if k == COPY_KERNEL]
    if not copies:
        raise SystemExit(f"{d}: no {COPY_KERNEL} dispatch to calibrate {counter} against")
    copy_kib = max(copies)
    factor = copy_bytes / (copy_kib * 1024.0)
    vals = [v for k, v in rows if kernel in k]
    if not vals:
        raise SystemExit(f"{d}: no dispatch of a kernel containing {kernel!r}")
    # the first dispatch is a warm-up (cold caches, first touch); average the rest
    use = vals[1:] if len(vals) > 1 else vals
    return sum(use) / len(use) * 1024.0 * factor, len(use), factor, copy_kib


def traffic_summary(a, argv):
    fb, nf, ff, fk = calibrated(a.fetch, "FETCH_SIZE", a.kernel, a.copy_bytes)
    wb, nw, fw, wk = calibrated(a.write, "WRITE_SIZE", a.kernel, a.copy_bytes)
    alg = a.units_per_launch * a.bytes_per_unit
    total = fb + wb
    lines = [f"# HBM traffic: {a.title}", "",
             "Commands (from the repository root; one counter per run):", "", "```", *a.command,
             "python -m paper_1111_0716_amd.profile_summary " + shlex.join(argv), "```", "",
             f"Calibration: the largest `{COPY_KERNEL}` dispatch of each run is a device-to-device copy of "
             f"{a.copy_bytes} bytes, so it must read and write that many bytes.", "",
             "| counter | copy reads (KiB) | scale factor | kernel dispatches averaged | scaled bytes per launch |",
             "|---|---|---|---|---|",
             f"| FETCH_SIZE | {fk:.1f} | {ff:.4f} | {nf} | {fb:.4e} |",
             f"| WRITE_SIZE | {wk:.1f} | {fw:.4f} | {nw} | {wb:.4e} |", "",
             f"Algorithmic bytes per launch: {a.units_per_launch} units x {a.bytes_per_unit} B = {alg:.4e} B; "
             f"measured / algorithmic = {total / alg:.3f}.", "",
             f"kind: {a.kind}",
             f"kernel: {a.kernel}",
             f"fetch_bytes_per_launch: {fb:.6e}",
             f"write_bytes_per_launch: {wb:.6e}",
             f"traffic_bytes_per_launch: {total:.6e}",
             f"units_per_launch: {a.units_per_launch:.6e}",
             f"sources_sha256: {sources_sha256(a.kind)}", ""]
    return "\n".join(lines)


def read_all_counters(d, kernel):
    """{counter: [values per dispatch of the kernel]} of one --pmc run."""
    out = {}
    with open(_one(os.path.join(d, "**", "*counter_collection.csv"))) as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Dispatch_Id"]))
    for r in rows:
        if kernel in r["Kernel_Name"]:
            out.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return out


def counters_summary(dirs, kernel, title, commands):
    vals = {}
    for d in dirs:
        for name, v in read_all_counters(d, kernel).items():
            use = v[1:] if len(v) > 1 else v
            vals[name] = sum(use) / len(use)
    if not vals:
        raise SystemExit(f"no dispatch of a kernel containing {kernel!r}")
    lines = [f"# Counters: {title}", "", "Commands (from the repository root; one counter set per run):", "", "```",
             *commands, "```", "", f"Kernel: `{kernel}`; mean over its dispatches after the first.", "",
             "| counter | value per dispatch |", "|---|---|"]
    lines += [f"| {k} | {v:.4e} |" for k, v in sorted(vals.items())]
    derived = []
    wc = vals.get("SQ_WAVE_CYCLES")
    if wc:
        for k, label in (("SQ_ACTIVE_INST_VALU", "VALU issuing"), ("SQ_ACTIVE_INST_LDS", "LDS issuing"),
                         ("SQ_WAIT_INST_ANY", "waiting on s_waitcnt"), ("SQ_WAIT_INST_LDS", "waiting on LDS"),
                         ("SQ_WAIT_ANY", "waiting (any)")):
            if k in vals:
                derived.append(f"- {label}: {100.0 * vals[k] / wc:.1f} % of wave cycles")
    if "TCC_HIT_sum" in vals and "TCC_MISS_sum" in vals:
        tot = vals["TCC_HIT_sum"] + vals["TCC_MISS_sum"]
        if tot > 0:
            derived.append(f"- L2 hit rate: {100.0 * vals['TCC_HIT_sum'] / tot:.1f} %")
    if "SQ_LDS_BANK_CONFLICT" in vals and "SQ_INSTS_LDS" in vals:
        derived.append(f"- LDS bank-conflict cycles per LDS instruction: "
                       f"{vals['SQ_LDS_BANK_CONFLICT'] / max(vals['SQ_INSTS_LDS'], 1.0):.3f}")
    if derived:
        lines += ["", "Derived:", "", *derived]
    return "\n".join(lines) + "\n"


def read_traffic(path, kind, per_unit=False):
    """Scaled HBM bytes per launch from a traffic summary (per unit of work
    when `per_unit`: per launch divided by the units per launch the summary
    was taken with), or None when the file is absent or the kernel's sources
    changed since it was taken."""
    try:
        with open(path) as f:
            kv = dict(re.findall(r"^(\w+): (\S+)$", f.read(), flags=re.M))
    except OSError:
        return None
    if kv.get("kind") != kind or kv.get("sources_sha256") != sources_sha256(kind):
        return None
    b = float(kv["traffic_bytes_per_launch"])
    if per_unit:
        if "units_per_launch" not in kv:
            return None
        return b / float(kv["units_per_launch"])
    return b


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--out")
    c = sub.add_parser("traffic")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--kernel", required=True)
    c.add_argument("--kind", required=True, choices=sorted(KIND_SOURCES))
    c.add_argument("--copy-bytes", type=int, required=True)
    c.add_argument("--units-per-launch", type=float, required=True)
    c.add_argument("--bytes-per-unit", type=float, required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--command", action="append", required=True)
    c.add_argument("--out")
    k = sub.add_parser("counters")
    k.add_argument("dirs", nargs="+")
    k.add_argument("--kernel", required=True)
    k.add_argument("--title", required=True)
    k.add_argument("--command", action="append", required=True)
    k.add_argument("--out")
    argv = sys.argv[1:] if argv is None else list(argv)
    a = ap.parse_args(argv)
    if a.mode == "trace":
        text = trace_summary(a.dir, a.title, a.command)
    elif a.mode == "traffic":
        text = traffic_summary(a, argv)
    else:
        text = counters_summary(a.dirs, a.kernel, a.title, a.command)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    else:
        sys.stdout.write(text)


if __name__ == "__main__":
    main()
