"""Summaries of rocprofv3 output for this library's kernels.

    python -m paper_1908_06096_amd.profiling stats  <kernel_stats.csv> <out.md> "<command>"
    python -m paper_1908_06096_amd.profiling traffic <fetch_counter_collection.csv> \
        <write_counter_collection.csv> <copy_bytes> <out.json> "<commands>"
    python -m paper_1908_06096_amd.profiling sq <counter_collection.csv> <out.md> "<command>"
    python -m paper_1908_06096_amd.profiling lds <counter_collection.csv> <out.md> "<command>"

``stats`` turns a ``--kernel-trace --stats`` summary into a short markdown
table.  ``sq`` summarises an SQ/GRBM counter run per kernel: MFMA pipe busy
(SQ_VALU_MFMA_BUSY_CYCLES over the active cycles of all 1024 SIMDs; the
GRBM_GUI_ACTIVE reading is the sum over the 8 XCDs), the MFMA work issued
(SQ_INSTS_VALU_MFMA_MOPS_* x 512 flops) and VALU issue (SQ_INSTS_VALU, a
wave64 instruction holding a SIMD for 4 cycles).  ``lds`` summarises an LDS
counter run: bank-conflict cycles against the cycles LDS instructions were
active, LDS instructions issued, wave-cycles spent waiting on LDS, and MFMA
busy as in ``sq``.  ``traffic`` turns two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE``
runs into HBM bytes per dispatch for each kernel, scaled by what the same
counters read for a plain device copy of ``copy_bytes`` bytes captured in the
same runs (the runtime's ``copyBuffer`` dispatch whose write counter is the
largest), and records a hash
of the kernel sources so that a figure is only reported while the kernels are
unchanged.
"""

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["csrc/legendre.hip", "csrc/fft.hip", "csrc/sht_internal.h", "csrc/capi.hip"]
STAGE_KERNELS = {
    "legendre_inverse": "legendre_inverse",
    "fourier_synthesis": "fourier_synthesis_kernel",
    "fourier_analysis": "fourier_analysis_kernel",
    "legendre_direct": "legendre_direct",
}


def source_hash():
    h = hashlib.sha256()
    for rel in SOURCES:
        with open(os.path.join(HERE, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _short(name):
    return name.split("(")[0].replace("void ", "").replace("shtmi::", "")


def stats_markdown(csv_path, out_md, command):
    rows = list(csv.DictReader(open(csv_path)))
    lines = [
        "# Kernel trace summary",
        "",
        "Command:",
        "",
        "```",
        command,
        "```",
        "",
        "| kernel | calls | total ms | average ms | % of GPU time |",
        "|---|---|---|---|---|",
    ]
    for r in rows:
        lines.append("| `%s` | %s | %.3f | %.3f | %.2f |" % (
            _short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e6,
            float(r["Percentage"])))
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def _per_dispatch(csv_path, counter):
    vals = defaultdict(list)
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] == counter:
            vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return vals


def traffic_json(fetch_csv, write_csv, copy_bytes, out_json, commands):
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(write_csv, "WRITE_SIZE")

    def copy_dispatch(path, counter):
        best = None
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"]:
                v = float(r["Counter_Value"])
                if best is None or v > best[1]:
                    best = (r["Dispatch_Id"], v)
        return best

    wd = copy_dispatch(write_csv, "WRITE_SIZE")
    fd = copy_dispatch(fetch_csv, "FETCH_SIZE")
    cf, cw = (fd[1] if fd else None), (wd[1] if wd else None)
    if not cf or not cw:
        raise SystemExit("no copy-kernel dispatch found for calibration")
    # KiB reading -> bytes: the copy moved copy_bytes in and copy_bytes out
    scale_f = copy_bytes / cf
    scale_w = copy_bytes / cw
    # A stage may be several kernels, each dispatched once per stage (the FFT
    # stages run one launch per work-group size): its bytes are the sum of
    # their per-dispatch averages.
    kernels = {}
    for stage, key in STAGE_KERNELS.items():
        fk = sorted(k for k in fetch if key in k and "shtmi" in k)
        wk = sorted(k for k in write if key in k and "shtmi" in k)
        if not fk or not wk:
            continue
        f = sum(sum(fetch[k]) / len(fetch[k]) for k in fk)
        w = sum(sum(write[k]) / len(write[k]) for k in wk)
        kernels[stage] = {"kernel": " + ".join(_short(k) for k in fk), "fetch_bytes": f * scale_f,
                          "write_bytes": w * scale_w, "fetch_kib_raw": f, "write_kib_raw": w}
    out = {
        "source_sha256": source_hash(),
        "copy_bytes": copy_bytes,
        "copy_fetch_kib": cf,
        "copy_write_kib": cw,
        "scale_fetch_bytes_per_kib": scale_f,
        "scale_write_bytes_per_kib": scale_w,
        "commands": commands,
        "kernels": kernels,
    }
    with open(out_json, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


SIMDS = 1024  # 256 CUs x 4 SIMDs
XCDS = 8


def sq_markdown(csv_path, out_md, command):
    per = defaultdict(lambda: defaultdict(list))  # kernel -> counter -> per-dispatch values
    dur = defaultdict(dict)
    for r in csv.DictReader(open(csv_path)):
        k = _short(r["Kernel_Name"])
        per[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
        dur[k][r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
    lines = [
        "# SQ counters per kernel (averages per dispatch)",
        "",
        "Command:",
        "",
        "```",
        command,
        "```",
        "",
        "MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 x 1024 SIMDs); MFMA Tflop issued = "
        "SQ_INSTS_VALU_MFMA_MOPS_{F32,BF16,F64} x 512 (padding included); VALU busy = SQ_INSTS_VALU x 4 / "
        "(GRBM_GUI_ACTIVE / 8 x 1024).",
        "",
        "| kernel | dispatches | ms | MFMA busy | MFMA Tflop issued (F32 / BF16 / F64) | VALU instr | VALU busy |",
        "|---|---|---|---|---|---|---|",
    ]
    for k in sorted(per, key=lambda x: -sum(dur[x].values())):
        c = per[k]
        if "shtmi" not in k and "legendre" not in k and "fourier" not in k:
            continue

        def avg(name):
            v = c.get(name, [0.0])
            return sum(v) / len(v)

        active = avg("GRBM_GUI_ACTIVE") / XCDS * SIMDS
        mfma = avg("SQ_VALU_MFMA_BUSY_CYCLES") / active if active else 0.0
        valu = avg("SQ_INSTS_VALU") * 4 / active if active else 0.0
        mops = [avg("SQ_INSTS_VALU_MFMA_MOPS_" + t) * 512 / 1e12 for t in ("F32", "BF16", "F64")]
        ms = sum(dur[k].values()) / len(dur[k])
        lines.append("| `%s` | %d | %.3f | %.1f%% | %.3f / %.3f / %.3f | %.3g | %.1f%% |" % (
            k, len(dur[k]), ms, 100 * mfma, mops[0], mops[1], mops[2], avg("SQ_INSTS_VALU"), 100 * valu))
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def measured_traffic(path, stage):
    """HBM bytes per call of ``stage`` (all its kernels) from a committed
    traffic file, or None when the file is absent or the kernel sources
    changed since."""
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("source_sha256") != source_hash():
        return None
    k = d.get("kernels", {}).get(stage)
    if not k:
        return None
    return k["fetch_bytes"] + k["write_bytes"]


def lds_markdown(csv_path, out_md, command):
    per = defaultdict(lambda: defaultdict(list))
    dur = defaultdict(dict)
    for r in csv.DictReader(open(csv_path)):
        k = _short(r["Kernel_Name"])
        per[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
        dur[k][r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
    lines = [
        "# LDS counters per kernel (averages per dispatch)",
        "",
        "Command:",
        "",
        "```",
        command,
        "```",
        "",
        "Bank-conflict cycles (SQ_LDS_BANK_CONFLICT) against the cycles LDS instructions were active "
        "(SQ_ACTIVE_INST_LDS), LDS instructions (SQ_INSTS_LDS), wave-cycles waiting on LDS (SQ_WAIT_INST_LDS); "
        "MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 x 1024 SIMDs).",
        "",
        "| kernel | dispatches | ms | bank-conflict cycles | LDS active cycles | LDS instr | LDS wait | MFMA busy |",
        "|---|---|---|---|---|---|---|---|",
    ]
    for k in sorted(per, key=lambda x: -sum(dur[x].values())):
        c = per[k]
        if "legendre" not in k and "fourier" not in k:
            continue

        def avg(name):
            v = c.get(name, [0.0])
            return sum(v) / len(v)

        active = avg("GRBM_GUI_ACTIVE") / XCDS * SIMDS
        mfma = avg("SQ_VALU_MFMA_BUSY_CYCLES") / active if active else 0.0
        ms = sum(dur[k].values()) / len(dur[k])
        lines.append("| `%s` | %d | %.3f | %.3g | %.3g | %.3g | %.3g | %.1f%% |" % (
            k, len(dur[k]), ms, avg("SQ_LDS_BANK_CONFLICT"), avg("SQ_ACTIVE_INST_LDS"), avg("SQ_INSTS_LDS"),
            avg("SQ_WAIT_INST_LDS"), 100 * mfma))
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats_markdown(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic_json(sys.argv[2], sys.argv[3], float(sys.argv[4]), sys.argv[5], sys.argv[6])
    elif sys.argv[1] == "sq":
        sq_markdown(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "lds":
        lds_markdown(sys.argv[2], sys.argv[3], sys.argv[4])
    else:
        raise SystemExit(__doc__)
