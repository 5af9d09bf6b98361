"""Text summaries of rocprofv3 output for this library's kernels.

Kernel-time table from a ``--kernel-trace --stats`` run::

    python -m paper_2505_02350_amd.prof_summary stats RUN_kernel_stats.csv \\
        --title "..." --command "rocprofv3 ..." > profiles/NAME.md

HBM traffic per launch from two ``--pmc`` runs (FETCH_SIZE, then
WRITE_SIZE; both counters are KiB per dispatch), each scaled by what the same
counter reads for the largest plain copy kernel in the run, whose size is
known (``--copy-bytes``)::

    python -m paper_2505_02350_amd.prof_summary traffic --fetch F.csv --write W.csv \\
        --copy-bytes 268435456 --kernels k_forward k_bwd_tiles \\
        --command-fetch "..." --command-write "..." > profiles/NAME.md

The traffic summary embeds a JSON block with the SHA-256 of the kernel
source it was measured on; a reader of the numbers checks that hash before
using them.
"""

import argparse
import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

COPY_KERNEL = "__amd_rocclr_copyBuffer"
KERNEL_SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "erbf_kernels.hip")


def kernel_source_sha256(path: str = KERNEL_SOURCE) -> str:
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def stats_table(path: str, title: str, command: str, top: int = 24) -> str:
    rows = list(csv.DictReader(open(path)))
    out = [f"# {title}", "", "Command (from the repository root; `cd /tmp && export TMPDIR=/tmp` first, with "
           "`R` the repository root):", "", "```", command, "```", "",
           "| kernel | calls | avg us | min us | max us | share % |", "|---|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        name = r["Name"].replace("|", "/")
        if len(name) > 90:
            name = name[:87] + "..."
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} "
                   f"| {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def _per_dispatch(path: str, counter: str):
    """{kernel name: [value per dispatch]} for one counter (KiB)."""
    vals = defaultdict(dict)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        vals[r["Kernel_Name"]][int(r["Dispatch_Id"])] = float(r["Counter_Value"])
    return {k: [v[d] for d in sorted(v)] for k, v in vals.items()}


def _match(name: str, short: str) -> bool:
    base = name.split("(")[0]
    return base.endswith("::" + short) or base.endswith(" " + short) or base == short or \
        base.split("<")[0].endswith("::" + short)


def traffic_summary(fetch_csv: str, write_csv: str, copy_bytes: int, kernels, cmd_fetch: str, cmd_write: str):
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(write_csv, "WRITE_SIZE")
    if COPY_KERNEL not in fetch or COPY_KERNEL not in write:
        raise SystemExit("no copy kernel in the counter runs (run the benchmark with --copy-calibration)")
    # the calibration copy is the copy dispatch that moves the most bytes
    copy_fetch = max(fetch[COPY_KERNEL])
    copy_write = max(write[COPY_KERNEL])
    expect_kib = copy_bytes / 1024.0
    scale_f = expect_kib / copy_fetch
    scale_w = expect_kib / copy_write
    entries = {}
    for short in kernels:
        fk = [n for n in fetch if _match(n, short)]
        wk = [n for n in write if _match(n, short)]
        if not fk or not wk:
            raise SystemExit(f"kernel {short} not found in the counter runs")
        fv = [x for n in fk for x in fetch[n]]
        wv = [x for n in wk for x in write[n]]
        f_kib = sum(fv) / len(fv)
        w_kib = sum(wv) / len(wv)
        entries[short] = {
            "dispatches": len(fv),
            "fetch_kib_per_dispatch": f_kib,
            "write_kib_per_dispatch": w_kib,
            "traffic_bytes_per_launch": 1024.0 * (f_kib * scale_f + w_kib * scale_w),
        }
    block = {
        "source": "paper_2505_02350_amd/csrc/erbf_kernels.hip",
        "source_sha256": kernel_source_sha256(),
        "copy_bytes": copy_bytes,
        "copy_fetch_kib": copy_fetch,
        "copy_write_kib": copy_write,
        "scale_fetch": scale_f,
        "scale_write": scale_w,
        "kernels": entries,
    }
    lines = ["# HBM traffic per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)", "",
             "Commands (from the repository root; `cd /tmp && export TMPDIR=/tmp` first, with `R` the "
             "repository root):", "", "```", cmd_fetch, cmd_write, "```", "",
             f"Calibration: the largest `{COPY_KERNEL}` dispatch copies {copy_bytes} bytes and read "
             f"FETCH_SIZE {copy_fetch:.0f} KiB, WRITE_SIZE {copy_write:.0f} KiB; scale factors "
             f"{scale_f:.4f} (fetch) and {scale_w:.4f} (write).", "",
             "| kernel | dispatches | FETCH KiB | WRITE KiB | traffic MB per launch |",
             "|---|---:|---:|---:|---:|"]
    for k, e in entries.items():
        lines.append(f"| `{k}` | {e['dispatches']} | {e['fetch_kib_per_dispatch']:.0f} | "
                     f"{e['write_kib_per_dispatch']:.0f} | {e['traffic_bytes_per_launch'] / 1e6:.2f} |")
    lines += ["", "```json", json.dumps(block, indent=1), "```", ""]
    return "\n".join(lines)


def read_traffic(path: str):
    """The JSON block of a traffic summary, or None if absent or taken on a
    different kernel source."""
    try:
        text = open(path).read()
    except OSError:
        return None
    if "```json" not in text:
        return None
    block = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    if block.get("source_sha256") != kernel_source_sha256():
        return None
    return block


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--top", type=int, default=24)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--kernels", nargs="+", required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        sys.stdout.write(stats_table(a.csv, a.title, a.command, a.top))
    else:
        sys.stdout.write(traffic_summary(a.fetch, a.write, a.copy_bytes, a.kernels, a.command_fetch,
                                         a.command_write))


if __name__ == "__main__":
    main()
