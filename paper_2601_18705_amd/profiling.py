"""Summaries of rocprofv3 CSV output (kernel statistics and HBM counters).

Used to turn `rocprofv3 --kernel-trace --stats -f csv` and `rocprofv3 --pmc
FETCH_SIZE` / `--pmc WRITE_SIZE` runs of bench.py into the short text and JSON
records kept with the repository.  Reads CSV files only; runs nothing.

    python -m paper_2601_18705_amd.profiling stats <kernel_stats.csv> <title> <command> [note]
        [comma-separated kernel name prefixes to leave out]
    python -m paper_2601_18705_amd.profiling traffic <fetch counter_collection.csv>
        <write counter_collection.csv> <calibration MiB> <kernel source> <out.json> [kernel name prefix]

    python -m paper_2601_18705_amd.profiling traffic-table <fetch counter_collection.csv>
        <write counter_collection.csv> <calibration MiB> <title> <command>...

    python -m paper_2601_18705_amd.profiling mfma <counter_collection.csv> <agent_info.csv>
        <kernel_stats.csv> <title> <command>...

The kernel name prefix (default k_sweep, the degree-0 sweep) selects the dispatches
averaged, e.g. "k_q1_sweep<double>" for the FP64 bilinear DG sweep.
"""
from __future__ import annotations

import csv
import hashlib
import json
import re
import sys


def short_name(name):
    name = re.sub(r"dlr::\(anonymous namespace\)::", "", name)
    name = re.sub(r"\(.*", "", name)
    return name.replace("void ", "")


def kernel_stats_md(path, title, command, note="", exclude=()):
    """Markdown table of a kernel-statistics CSV; kernels whose short name starts with one of the
    exclude prefixes are dropped and the shares recomputed over the rest."""
    rows = [r for r in csv.DictReader(open(path)) if not short_name(r["Name"]).startswith(tuple(exclude))]
    total = sum(float(r["TotalDurationNs"]) for r in rows) or 1.0
    out = [f"# {title}", "", "Command (from the repository root on an MI355X, ROCm 7.2):", "", "```",
           "cd /tmp && export TMPDIR=/tmp", command, "```", ""]
    if note:
        out += [note, ""]
    out += ["| kernel | calls | total (ms) | average (us) | min (us) | max (us) | share (%) |",
            "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                   f"{float(r['MaxNs']) / 1e3:.1f} | {100.0 * float(r['TotalDurationNs']) / total:.1f} |")
    return "\n".join(out) + "\n"


def _per_kernel(path, counter):
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        vals.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return vals


def sweep_traffic(fetch_csv, write_csv, calib_mib, sweep_source, sweep_prefix="k_sweep"):
    """HBM bytes per sweep launch.  Each counter (KiB per dispatch) is scaled by the factor that
    makes it read the known size of the calibration kernel (an elementwise kernel that reads and
    writes calib_mib MiB, the last 'elementwise' dispatch of the run)."""
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    calib = [k for k in fetch if "elementwise" in k and "Mul" in k] or [k for k in fetch if "elementwise" in k]
    if not calib:
        raise SystemExit("no calibration kernel in the FETCH_SIZE run")
    known_kib = calib_mib * 1024.0
    f_scale = known_kib / fetch[calib[-1]][-1]
    w_scale = known_kib / write[calib[-1]][-1] if calib[-1] in write else 1.0
    sk = [k for k in fetch if k.startswith(sweep_prefix)]
    if not sk:
        raise SystemExit(f"no dispatch of {sweep_prefix} in the FETCH_SIZE run")
    f = [v for k in sk for v in fetch[k]]
    w = [v for k in sk for v in write.get(k, [])]
    fetch_b = sum(f) / len(f) * 1024.0 * f_scale
    write_b = sum(w) / len(w) * 1024.0 * w_scale if w else 0.0
    sha = hashlib.sha256(open(sweep_source, "rb").read()).hexdigest()[:16]
    return {"sweep_source_sha": sha, "hbm_bytes_per_launch": fetch_b + write_b, "fetch_bytes_per_launch": fetch_b,
            "write_bytes_per_launch": write_b, "fetch_scale": f_scale, "write_scale": w_scale,
            "sweep_launches": len(f), "kernel": sweep_prefix, "calibration_kernel": calib[-1],
            "calibration_mib": calib_mib}


def traffic_table_md(fetch_csv, write_csv, calib_mib, title, commands, min_mb=20.0):
    """Markdown table of HBM bytes per dispatch for every kernel of two counter runs (FETCH_SIZE and
    WRITE_SIZE), each scaled by the calibration kernel's factor as in sweep_traffic; kernels that
    move less than min_mb per dispatch are left out."""
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    calib = [k for k in fetch if "elementwise" in k and "Mul" in k] or [k for k in fetch if "elementwise" in k]
    if not calib:
        raise SystemExit("no calibration kernel in the FETCH_SIZE run")
    known_kib = calib_mib * 1024.0
    f_scale = known_kib / fetch[calib[-1]][-1]
    w_scale = known_kib / write[calib[-1]][-1] if calib[-1] in write else 1.0
    out = [f"# {title}", "", "Commands (from the repository root on an MI355X, ROCm 7.2):", "", "```",
           "cd /tmp && export TMPDIR=/tmp", *commands, "```", "",
           f"Counters scaled by the factors that make them read the {calib_mib:g} MiB of `{calib[-1][:60]}`: "
           f"FETCH_SIZE x {f_scale:.2f}, WRITE_SIZE x {w_scale:.2f}.  Averages over the dispatches of each kernel.", "",
           "| kernel | dispatches | read (MB) | written (MB) |", "|---|---:|---:|---:|"]
    for k, fv in fetch.items():
        if k in calib:
            continue
        f = sum(fv) / len(fv) * 1024.0 * f_scale / 1e6
        wv = write.get(k, [])
        w = sum(wv) / len(wv) * 1024.0 * w_scale / 1e6 if wv else 0.0
        if f + w >= min_mb:
            out.append(f"| `{k}` | {len(fv)} | {f:.1f} | {w:.1f} |")
    return "\n".join(out) + "\n"


# dense matrix-core peaks of the MI355X (TFLOP/s), by operand type
MFMA_PEAK_TFLOPS = {"F32": 157.3, "F64": 78.6}


def mfma_md(counter_csv, agent_csv, stats_csv, title, commands, kernel_mark="mfma"):
    """Markdown table of matrix-core use per kernel from one counter run with
    SQ_INSTS_VALU_MFMA_MOPS_F32, SQ_INSTS_VALU_MFMA_MOPS_F64, SQ_VALU_MFMA_BUSY_CYCLES and
    GRBM_GUI_ACTIVE: MFMA flops per dispatch (MOPS x 512), the achieved rate over the kernel's average
    duration in the kernel-trace run (stats_csv) against the dense peak of its operand type, and the
    matrix-core busy fraction busy / (GUI_ACTIVE per XCC x SIMDs).  GRBM_GUI_ACTIVE comes summed over
    the XCCs; the agent record gives their number and the SIMD count."""
    gpu = [r for r in csv.DictReader(open(agent_csv)) if r.get("Agent_Type", r.get("Type")) == "GPU"][0]
    n_xcc = int(gpu["Num_Xcc"])
    simds = int(gpu["Simd_Count"])
    per = {}
    for r in csv.DictReader(open(counter_csv)):
        k = short_name(r["Kernel_Name"])
        if kernel_mark not in k:
            continue
        d = per.setdefault(k, {}).setdefault(r["Dispatch_Id"], {})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
    avg_ns = {short_name(r["Name"]): float(r["AverageNs"]) for r in csv.DictReader(open(stats_csv))}
    out = [f"# {title}", "", "Commands (from the repository root on an MI355X, ROCm 7.2):", "", "```",
           "cd /tmp && export TMPDIR=/tmp", *commands, "```", "",
           f"MFMA flops = MOPS x 512 per dispatch; rate over the average duration of the kernel-trace run; "
           f"busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / {n_xcc} XCC x {simds} SIMDs).  Dense peaks: "
           + ", ".join(f"{t} {v} TFLOP/s" for t, v in MFMA_PEAK_TFLOPS.items()) + ".", "",
           "| kernel | dispatches | type | GFLOP per dispatch | average (us) | TFLOP/s | of peak (%) | MFMA busy (%) |",
           "|---|---:|---|---:|---:|---:|---:|---:|"]
    for k, ds in per.items():
        n = len(ds)
        f32 = sum(d.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) for d in ds.values()) / n * 512.0
        f64 = sum(d.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) for d in ds.values()) / n * 512.0
        busy = sum(d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for d in ds.values()) / n
        gui = sum(d.get("GRBM_GUI_ACTIVE", 0.0) for d in ds.values()) / n
        kind, flops = ("F32", f32) if f32 >= f64 else ("F64", f64)
        t = avg_ns.get(k)
        rate = flops / (t * 1e-9) / 1e12 if t else float("nan")
        util = 100.0 * busy / (gui / n_xcc * simds) if gui > 0 else float("nan")
        out.append(f"| `{k}` | {n} | {kind} | {flops / 1e9:.3f} | {t / 1e3 if t else float('nan'):.1f} | "
                   f"{rate:.1f} | {100.0 * rate / MFMA_PEAK_TFLOPS[kind]:.1f} | {util:.1f} |")
    return "\n".join(out) + "\n"


def main(argv):
    if len(argv) >= 4 and argv[0] == "stats":
        sys.stdout.write(kernel_stats_md(argv[1], argv[2], argv[3], argv[4] if len(argv) > 4 else "",
                                         argv[5].split(",") if len(argv) > 5 else ()))
    elif len(argv) >= 6 and argv[0] == "traffic-table":
        sys.stdout.write(traffic_table_md(argv[1], argv[2], float(argv[3]), argv[4], argv[5:]))
    elif len(argv) >= 6 and argv[0] == "mfma":
        sys.stdout.write(mfma_md(argv[1], argv[2], argv[3], argv[4], argv[5:]))
    elif len(argv) in (6, 7) and argv[0] == "traffic":
        rec = sweep_traffic(argv[1], argv[2], float(argv[3]), argv[4], *argv[6:7])
        with open(argv[5], "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
