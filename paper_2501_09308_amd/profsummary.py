"""Short markdown summaries of rocprofv3 CSV output, for the committed
profile notes.

    python -m paper_2501_09308_amd.profsummary SPEC.json

SPEC: {"out", "title", "cmd", "stats_csv", optional "fetch", "write",
"cfetch", "cwrite" (FETCH_SIZE / WRITE_SIZE counter CSVs of the measured
program and of the 1 GiB copy calibration), optional "sq" (SQ counter CSV,
with SQ_WAVES, SQ_INSTS_VALU, SQ_WAVE_CYCLES and SQ_WAIT_ANY for the
derived table), optional "flops" (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F32
counter CSV), optional "record_kernel" and "extra"}.  With "record_kernel" the summary
ends with a traffic record: the calibrated HBM bytes per dispatch of that
kernel and a hash of the kernel sources, which the benchmark reports as the
kernel's measured traffic while the sources are unchanged.
"""
from __future__ import annotations

import collections
import csv
import glob
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
KERNEL_SOURCES = ("xrdvi_device.h", "xrdvi_steps.h", "xrdvi_kernels.hip")
RECORD_PREFIX = "traffic-record: "


def kernel_sources_sha256() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(PKG, "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def recorded(kernel: str):
    """The profile record of `kernel` under profiles/ (calibrated HBM bytes,
    executed FP32 flops and VALU instruction counts per dispatch), or None
    when none was recorded for the current kernel sources."""
    want = kernel_sources_sha256()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                if line.startswith(RECORD_PREFIX):
                    rec = json.loads(line[len(RECORD_PREFIX):])
                    if rec.get("kernel") == kernel and rec.get("sources_sha256") == want:
                        return rec
    return None


def recorded_traffic(kernel: str):
    """Calibrated HBM bytes per dispatch recorded for `kernel`, or None."""
    rec = recorded(kernel)
    return None if rec is None else float(rec["bytes_per_dispatch"])


def _stats(path):
    rows = list(csv.DictReader(open(path)))
    return [(r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3,
             float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
             float(r["Percentage"])) for r in rows]


def _counters(path):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: (len(v), sum(v) / len(v)) for k, v in agg.items()}


def short(name: str) -> str:
    n = name.replace("xrdvi::", "").replace("(anonymous namespace)::", "")
    return n.split("(")[0] if "(" in n else n


def summarize(out, title, cmd, stats_csv, fetch=None, write=None, cfetch=None,
              cwrite=None, sq=None, flops=None, record_kernel=None, extra=""):
    L = [f"# {title}", "", "Commands (run from the repository root on an MI355X):",
         "", "```", cmd, "```", "",
         "| kernel | calls | avg us | min us | max us | % time |",
         "|---|---|---|---|---|---|"]
    for n, c, a, mn, mx, p in _stats(stats_csv):
        if "xrdvi" in n:
            L.append(f"| `{short(n)}` | {c} | {a:.2f} | {mn:.2f} | {mx:.2f} | {p:.1f} |")
    record = None
    if fetch:
        f, w = _counters(fetch), _counters(write)
        cf, cw = _counters(cfetch), _counters(cwrite)
        copy_f = [v for (k, _), v in cf.items() if "k_copy" in k][0][1]
        copy_w = [v for (k, _), v in cw.items() if "k_copy" in k][0][1]
        fscale, wscale = 1048576.0 / copy_f, 1048576.0 / copy_w
        L += ["", "Counter calibration with a 1 GiB plain copy kernel (`k_copy` of "
              f"the microbenchmarks): FETCH_SIZE reads {copy_f:.0f} KiB (scale "
              f"{fscale:.3f}), WRITE_SIZE reads {copy_w:.0f} KiB (scale {wscale:.3f}).",
              "", "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | "
              "calibrated HBM MB / dispatch |", "|---|---|---|---|---|"]
        for (k, _), (n, v) in sorted(f.items()):
            if "xrdvi" not in k:
                continue
            wv = w.get((k, "WRITE_SIZE"), (0, 0.0))[1]
            b = (v * fscale + wv * wscale) * 1024
            L.append(f"| `{short(k)}` | {n} | {v:.1f} | {wv:.1f} | {b / 1e6:.3f} |")
            if record_kernel and short(k) == record_kernel:
                record = b
    if sq:
        c = _counters(sq)
        names = sorted({k for k, _ in c if "xrdvi" in k})
        cols = sorted({n for _, n in c})
        L += ["", "SQ counters (averages per dispatch):", "",
              "| kernel | " + " | ".join(cols) + " |",
              "|---|" + "---|" * len(cols)]
        for k in names:
            L.append(f"| `{short(k)}` | " + " | ".join(
                f"{c[(k, n)][1]:.4g}" if (k, n) in c else "" for n in cols) + " |")
    avg_us = {short(n): a for n, _, a, _, _, _ in _stats(stats_csv)}
    if flops:
        c = _counters(flops)
        L += ["", "Counter-measured FP32 VALU work (flops = 64 lanes x (ADD + MUL "
              "+ 2 FMA + TRANS)):", "",
              "| kernel | ADD | MUL | FMA | TRANS | executed GFLOP / dispatch | "
              "avg us | executed TFLOP/s |", "|---|---|---|---|---|---|---|---|"]
        for k in sorted({k for k, _ in c if "xrdvi" in k}):
            v = {n: c.get((k, f"SQ_INSTS_VALU_{n}_F32"), (0, 0.0))[1]
                 for n in ("ADD", "MUL", "FMA", "TRANS")}
            if v["FMA"] + v["ADD"] + v["MUL"] < 1e5:
                continue
            gf = 64 * (v["ADD"] + v["MUL"] + 2 * v["FMA"] + v["TRANS"]) / 1e9
            us = avg_us.get(short(k), float("nan"))
            L.append(f"| `{short(k)}` | {v['ADD']:.3e} | {v['MUL']:.3e} | "
                     f"{v['FMA']:.3e} | {v['TRANS']:.3e} | {gf:.2f} | {us:.1f} | "
                     f"{gf / (us * 1e-6) / 1e3:.1f} |")
    if sq:
        c = _counters(sq)
        rows = []
        for k in sorted({k for k, _ in c if "xrdvi" in k}):
            g = lambda n: c.get((k, n), (0, 0.0))[1]  # noqa: E731
            if g("SQ_WAVES") > 0 and g("SQ_WAVE_CYCLES") > 0:
                rows.append(f"| `{short(k)}` | {g('SQ_WAVES'):.0f} | "
                            f"{g('SQ_INSTS_VALU') / g('SQ_WAVES'):.0f} | "
                            f"{g('SQ_WAIT_ANY') / g('SQ_WAVE_CYCLES'):.2f} |")
        if rows:
            L += ["", "Fraction of wave-cycles spent waiting (SQ_WAIT_ANY / "
                  "SQ_WAVE_CYCLES) and VALU instructions per wave:", "",
                  "| kernel | waves | VALU / wave | waiting |", "|---|---|---|---|"]
            L += rows
    if extra:
        L += ["", extra]
    if record is not None:
        rec = dict(kernel=record_kernel, bytes_per_dispatch=round(record))
        # executed FP32 flops and the VALU instruction mix of the recorded
        # kernel, for the benchmark's counter-measured rates
        for path, names in ((flops, ("ADD", "MUL", "FMA", "TRANS")), (sq, ())):
            if not path:
                continue
            c = _counters(path)
            k = next((k for k, _ in c if short(k) == record_kernel), None)
            if k is None:
                continue
            if names:
                v = {n: c.get((k, f"SQ_INSTS_VALU_{n}_F32"), (0, 0.0))[1] for n in names}
                rec["flops_per_dispatch"] = round(
                    64 * (v["ADD"] + v["MUL"] + 2 * v["FMA"] + v["TRANS"]))
                rec["valu_trans_per_dispatch"] = round(v["TRANS"])
            elif (k, "SQ_INSTS_VALU") in c:
                rec["valu_per_dispatch"] = round(c[(k, "SQ_INSTS_VALU")][1])
        rec["sources_sha256"] = kernel_sources_sha256()
        L += ["", RECORD_PREFIX + json.dumps(rec)]
    with open(out, "w") as fh:
        fh.write("\n".join(L) + "\n")


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    with open(argv[0]) as f:
        summarize(**json.load(f))


if __name__ == "__main__":
    sys.exit(main())
