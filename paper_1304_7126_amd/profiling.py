"""Summaries of rocprofv3 runs (CSV output) for profiles/, and the figures
bench.py reads back from them.

Each summary is a short markdown file: the command that made it, a table
for the reader, and one JSON line (after the marker ``figures:``) with the
numbers bench.py uses, keyed to a hash of the kernel sources, so that a
summary of other kernels is never mistaken for the current ones.

  python -m paper_1304_7126_amd.profiling stats  TRACE_CSV OUT.md --command ... --kernel NAME --first A --count K
  python -m paper_1304_7126_amd.profiling bytes  FETCH_CSV WRITE_CSV OUT.md --command ... --kernel NAME --first A --count K
  python -m paper_1304_7126_amd.profiling counters PMC_CSV OUT.md --command ... --kernel NAME --first A --count K

--kernel selects the kernel by a substring of its name; --first/--count the
window of its launches (1-based, in time order) the figures average over.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
from collections import OrderedDict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
MARK = "figures: "


def kernel_source_hash() -> str:
    """Hash of every kernel source file (csrc/*.hip, csrc/*.h)."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(f.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def read_figures(path: str):
    """The JSON figures of a summary, or None if the file is missing."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            if line.startswith(MARK):
                return json.loads(line[len(MARK):])
    return None


def _short(name: str) -> str:
    name = name.split("(")[0]
    return name.replace("void ", "")


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _launches(trace_rows, kernel):
    """(start, end) of the launches of the kernel whose name contains `kernel`, in time order."""
    out = []
    for r in trace_rows:
        if kernel in r["Kernel_Name"]:
            out.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), _short(r["Kernel_Name"])))
    out.sort()
    return out


def _write(path, title, command, body, figures):
    figures = dict(figures)
    figures["kernel_source_hash"] = kernel_source_hash()
    with open(path, "w") as f:
        f.write(f"# {title}\n\nCommands (the profiled run from /tmp, the summary from the repository root):\n\n")
        for c in command:
            f.write(f"    {c}\n")
        f.write("\n" + body.rstrip() + "\n\n")
        f.write(MARK + json.dumps(figures) + "\n")


def stats(trace_csv, out_md, command, kernel, first, count, title):
    rows = _rows(trace_csv)
    per = OrderedDict()
    for r in rows:
        k = _short(r["Kernel_Name"])
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        e = per.setdefault(k, [0, 0])
        e[0] += 1
        e[1] += d
    tot = sum(v[1] for v in per.values())
    body = ["| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for k, (n, d) in sorted(per.items(), key=lambda kv: -kv[1][1])[:20]:
        body.append(f"| `{k}` | {n} | {d / n / 1e3:.1f} | {d / 1e6:.2f} | {100 * d / tot:.2f} |")
    la = _launches(rows, kernel)
    win = la[first - 1:first - 1 + count]
    avg = sum(e - s for s, e, _ in win) / max(len(win), 1) / 1e3
    body.append("")
    body.append(f"Launches {first}-{first + len(win) - 1} of `{win[0][2] if win else kernel}` (in time order): "
                f"{avg:.1f} us on average.")
    _write(out_md, title, command, "\n".join(body),
           {"kernel": win[0][2] if win else kernel, "window": [first, first + len(win) - 1], "avg_us": avg})


def _pmc_per_dispatch(rows, kernel, counter):
    """{dispatch id: summed counter value} for one kernel, dispatches in order."""
    acc = OrderedDict()
    for r in rows:
        if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter:
            d = int(r["Dispatch_Id"])
            acc[d] = acc.get(d, 0.0) + float(r["Counter_Value"])
    return [acc[k] for k in sorted(acc)]


def bytes_(fetch_csv, write_csv, out_md, command, kernel, first, count, title, copy_kernel="copyBuffer",
           copy_bytes=None):
    fr, wr = _rows(fetch_csv), _rows(write_csv)
    f = _pmc_per_dispatch(fr, kernel, "FETCH_SIZE")[first - 1:first - 1 + count]
    w = _pmc_per_dispatch(wr, kernel, "WRITE_SIZE")[first - 1:first - 1 + count]
    fk = sum(f) / len(f)
    wk = sum(w) / len(w)
    fs = ws = 1.0
    note = "no copy calibration in the run: counters unscaled"
    if copy_bytes:
        cf = _pmc_per_dispatch(fr, copy_kernel, "FETCH_SIZE")
        cw = _pmc_per_dispatch(wr, copy_kernel, "WRITE_SIZE")
        big_f = [v for v in cf if v > 0.25 * copy_bytes / 1024]
        big_w = [v for v in cw if v > 0.25 * copy_bytes / 1024]
        if big_f and big_w:
            fs = (copy_bytes / 1024) / (sum(big_f) / len(big_f))
            ws = (copy_bytes / 1024) / (sum(big_w) / len(big_w))
            note = (f"calibration: a device-to-device copy of {copy_bytes / 2**20:.0f} MiB reads FETCH_SIZE "
                    f"{sum(big_f) / len(big_f):,.0f} KiB and WRITE_SIZE {sum(big_w) / len(big_w):,.0f} KiB per launch, "
                    f"so FETCH_SIZE is scaled by {fs:.3f} and WRITE_SIZE by {ws:.3f}")
    rb, wb = fk * 1024 * fs, wk * 1024 * ws
    body = [note + ".", "",
            "| kernel | launches | FETCH_SIZE KiB / launch | WRITE_SIZE KiB / launch | read GB | write GB |",
            "|---|---|---|---|---|---|",
            f"| `{kernel}` | {first}-{first + len(f) - 1} | {fk:,.0f} | {wk:,.0f} | {rb / 1e9:.3f} | {wb / 1e9:.3f} |"]
    _write(out_md, title, command, "\n".join(body),
           {"kernel": kernel, "window": [first, first + len(f) - 1], "read_bytes": rb, "write_bytes": wb,
            "fetch_scale": fs, "write_scale": ws})


# the two SQ passes bench.py reads: issue rate and lane use, then the
# instruction mix (wave-instructions of each kind)
VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_THREAD_CYCLES_VALU", "SQ_WAVES", "SQ_BUSY_CYCLES",
                 "SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY")
MIX_COUNTERS = ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_TRANS_F64",
                "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_TRANS_F32")


def counters(pmc_csv, out_md, command, kernel, first, count, title):
    """Per-launch averages of every counter the run collected for the
    kernel, over its launches first .. first+count-1."""
    rows = _rows(pmc_csv)
    names = []
    for r in rows:
        if kernel in r["Kernel_Name"] and r["Counter_Name"] not in names:
            names.append(r["Counter_Name"])
    fig = {"kernel": kernel}
    body = ["| counter | per launch |", "|---|---|"]
    n = 0
    for c in names:
        v = _pmc_per_dispatch(rows, kernel, c)[first - 1:first - 1 + count]
        if v:
            fig[c] = sum(v) / len(v)
            n = len(v)
            body.append(f"| {c} | {fig[c]:,.0f} |")
    fig["window"] = [first, first + n - 1]
    _write(out_md, title, command, "\n".join(body), fig)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["stats", "bytes", "counters"])
    ap.add_argument("inputs", nargs="+")
    ap.add_argument("--command", action="append", required=True)
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--first", type=int, default=1)
    ap.add_argument("--count", type=int, default=1 << 30)
    ap.add_argument("--title", default="rocprofv3 summary")
    ap.add_argument("--copy-bytes", type=float, default=None)
    a = ap.parse_args(argv)
    if a.what == "stats":
        stats(a.inputs[0], a.inputs[1], a.command, a.kernel, a.first, a.count, a.title)
    elif a.what == "bytes":
        bytes_(a.inputs[0], a.inputs[1], a.inputs[2], a.command, a.kernel, a.first, a.count, a.title,
               copy_bytes=a.copy_bytes)
    else:
        counters(a.inputs[0], a.inputs[1], a.command, a.kernel, a.first, a.count, a.title)


if __name__ == "__main__":
    main()
