"""Text summaries of rocprofv3 output, and the HBM traffic they record.

    python -m paper_2603_14641_amd.profsum stats KERNEL_STATS_CSV --title T --command C
    python -m paper_2603_14641_amd.profsum hbm FETCH_CSV WRITE_CSV --title T --command C

``stats`` turns a ``--kernel-trace --stats`` kernel table into markdown.
``hbm`` averages FETCH_SIZE and WRITE_SIZE (KiB per dispatch) per kernel and
scales each by what the same counter reads for the plain 1 GiB device copy
(``__amd_rocclr_copyBuffer``, 1 GiB read and 1 GiB written) in the same run.
Each kernel's line also records the SHA-256 of the sources it is built from,
so ``traffic_per_dispatch`` can tell whether the counters still describe the
kernel as it is now (and returns None when they do not).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import re
import sys
from collections import defaultdict
from typing import Dict, Optional

_PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(_PKG, "csrc")
PROFILES = os.path.join(os.path.dirname(_PKG), "profiles")
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_KIB = 1 << 20   # the calibration copy moves 1 GiB each way

# kernel name prefix (after "sq::") -> the source file it lives in
KERNEL_SOURCES = {
    "k_layer": "sq_gates.hip", "k_sign_reduce": "sq_gates.hip",
    "k_pivot": "sq_measure.hip", "k_gather": "sq_measure.hip", "k_rowsum": "sq_measure.hip",
    "k_post": "sq_measure.hip", "k_cursor_init": "sq_measure.hip",
    "k_blk_": "sq_block.hip", "k_inj_": "sq_inject.hip", "k_transpose": "sq_rows.hip", "k_row_": "sq_rows.hip",
    "k_sample_init": "sq_sample.hip", "k_coins": "sq_sample.hip", "k_eval": "sq_sample.hip",
    "k_batch": "sq_batch.hip",
    "k_frame_": "sq_frames.hip",
    "k_fill_zero": "sq_io.hip", "k_init_diag": "sq_io.hip", "k_export_rows": "sq_io.hip", "k_import": "sq_io.hip",
}
COMMON = ("sq_device.h", "sq_internal.h")


def short_name(full: str) -> str:
    """'void sq::k_layer<2, 4>(unsigned long long*, ...)' -> 'k_layer<2, 4>'."""
    s = re.sub(r"^void\s+", "", full)
    depth = 0
    for i, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            s = s[:i]
            break
    return s.replace("sq::", "")


def source_of(kernel: str) -> Optional[str]:
    for prefix, src in KERNEL_SOURCES.items():
        if kernel.startswith(prefix):
            return src
    return None


def source_hash(kernel: str) -> Optional[str]:
    src = source_of(kernel)
    if src is None:
        return None
    h = hashlib.sha256()
    for f in (src,) + COMMON:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _per_kernel(path: str, counter: str) -> Dict[str, list]:
    vals = defaultdict(list)
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            vals[short_name(row["Kernel_Name"])].append(float(row["Counter_Value"]))
    return vals


def calibration(path: str, counter: str) -> float:
    """Counter value of the 1 GiB calibration copy: bench.py --copy-calibration
    runs three such copies before any other work, so they are the run's first
    three large copy dispatches; they must agree within 1%."""
    rows = []
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] == counter and short_name(row["Kernel_Name"]) == COPY_KERNEL \
                    and int(row["Grid_Size"]) >= 65536:
                rows.append((int(row["Dispatch_Id"]), float(row["Counter_Value"])))
    rows.sort()
    if len(rows) < 3:
        raise SystemExit("no calibration copies in the run (pass --copy-calibration to bench.py)")
    vals = [v for _, v in rows[:3]]
    if max(vals) > 1.01 * min(vals):
        raise SystemExit(f"calibration copies disagree: {vals}")
    return sum(vals) / 3


def hbm_summary(fetch_csv: str, write_csv: str, title: str, command: str) -> str:
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    f_raw, w_raw = calibration(fetch_csv, "FETCH_SIZE"), calibration(write_csv, "WRITE_SIZE")
    f_cal = COPY_KIB / f_raw
    w_cal = COPY_KIB / w_raw
    lines = [f"# {title}", "", "Commands (one counter per run):", "", "```", command, "```", "",
             f"Calibration: the plain 1 GiB device copy (`{COPY_KERNEL}`, the run's first three copies) reads "
             f"FETCH_SIZE = {f_raw:.1f} KiB and WRITE_SIZE = {w_raw:.1f} KiB for "
             f"{COPY_KIB} KiB moved each way, so FETCH_SIZE is scaled by {f_cal:.4f} and WRITE_SIZE by "
             f"{w_cal:.4f}.", "",
             "| Kernel | Dispatches | FETCH_SIZE avg (KiB) | WRITE_SIZE avg (KiB) | scaled read (GB) | "
             "scaled write (GB) |", "|---|---|---|---|---|---|"]
    machine = []
    for k in sorted(set(fetch) & set(write)):
        if k == COPY_KERNEL or source_of(k) is None:
            continue
        fa = sum(fetch[k]) / len(fetch[k])
        wa = sum(write[k]) / len(write[k])
        rb = fa * f_cal * 1024
        wb = wa * w_cal * 1024
        lines.append(f"| `{k}` | {len(fetch[k])} | {fa:.1f} | {wa:.1f} | {rb / 1e9:.3f} | {wb / 1e9:.3f} |")
        machine.append(f"traffic {k.replace(' ', '')} read={int(rb)} write={int(wb)} "
                       f"dispatches={len(fetch[k])} source={source_hash(k)}")
    lines += ["", "Scaled bytes per dispatch, with the SHA-256 (first 16 hex digits) of each kernel's "
              "source file plus the shared headers when the counters were taken:", "", "```"]
    lines += machine + ["```", ""]
    return "\n".join(lines)


def stats_summary(stats_csv: str, title: str, command: str) -> str:
    lines = [f"# {title}", "", "Command:", "", "```", command, "```", "",
             "| Kernel | Calls | Average (us) | % of GPU time |", "|---|---|---|---|"]
    with open(stats_csv, newline="") as f:
        for row in csv.DictReader(f):
            lines.append(f"| `{short_name(row['Name'])}` | {row['Calls']} | "
                         f"{float(row['AverageNs']) / 1e3:.1f} | {float(row['Percentage']):.2f} |")
    return "\n".join(lines + [""])


def traffic_per_dispatch(kernel_prefix: str, summary: str) -> Optional[int]:
    """Scaled read + write bytes per dispatch of the first kernel in `summary`
    (a profiles/ file written by `hbm`) whose name starts with kernel_prefix,
    or None if absent or if its source has changed since."""
    path = summary if os.path.isabs(summary) else os.path.join(PROFILES, summary)
    try:
        with open(path) as f:
            text = f.read()
    except OSError:
        return None
    for m in re.finditer(r"^traffic (\S+) read=(\d+) write=(\d+) dispatches=\d+ source=(\S+)$", text, re.M):
        name, rd, wr, src = m.group(1), int(m.group(2)), int(m.group(3)), m.group(4)
        if not name.startswith(kernel_prefix):
            continue
        return rd + wr if src == source_hash(name) else None
    return None


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    b = sub.add_parser("hbm")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    for p in (a, b):
        p.add_argument("--title", required=True)
        p.add_argument("--command", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        sys.stdout.write(stats_summary(args.csv, args.title, args.command))
    else:
        sys.stdout.write(hbm_summary(args.fetch_csv, args.write_csv, args.title, args.command))


if __name__ == "__main__":
    main()
