"""Measurement helpers: summaries of rocprofv3 output and the HBM-traffic
record of a kernel.

    python -m paper_1907_11678_amd.profiling stats <kernel_stats.csv>
        Markdown table of a `rocprofv3 --kernel-trace --stats
        --output-format csv` run (per kernel: calls, total, average, share).

    python -m paper_1907_11678_amd.profiling trace <kernel_trace.csv>
        The same per (kernel, grid size), so that full launches and a
        tuner's sample launches of one kernel are told apart.

    python -m paper_1907_11678_amd.profiling counters <kernel-substring> <evals> <csv> [<csv> ...]
        SQ counters of the largest-grid dispatches of a kernel from
        `rocprofv3 --pmc` runs, and the instruction counts per 64-lane
        evaluation, LDS busy fraction and wave wait fraction.

    python -m paper_1907_11678_amd.profiling counter-record <out.txt> <kernel>=<evals> ... -- <csv> ...
        The per-evaluation rates of each kernel (VALU and FP32-FMA
        instructions, LDS instructions and bytes read, LDS busy fraction,
        waits) from `rocprofv3 --pmc` runs, with the source digest; bench.py
        reports executed VALU and LDS rates from it while the digest matches.

    python -m paper_1907_11678_amd.profiling traffic <fetch_csv> <write_csv>
            <kernel-substring> <copy-bytes> <out.txt>
        Reduce two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs
        (counter_collection.csv) to bytes per launch of the kernel whose name
        contains <kernel-substring>.  The same runs must contain a plain
        device-to-device copy of <copy-bytes> bytes (bench.py
        --calibrate-copy); the copy's own FETCH_SIZE and WRITE_SIZE give the
        factor that turns the counters into bytes.  The record carries the
        digest of the kernel sources, so a reader can tell whether it still
        describes the code that is built.
"""
from __future__ import annotations

import csv
import hashlib
import os
import sys
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
# sources whose change (with the compiler flags) invalidates a traffic record
# of the scan kernels
KERNEL_SOURCES = ("csrc/tile.h", "csrc/scan_cmp.hip", "csrc/scan_crs.hip", "csrc/scan.hip", "csrc/internal.h",
                  "csrc/traveltime.h")
COPY_KERNEL = "copyBuffer"


def source_digest() -> str:
    from paper_1907_11678_amd.build import FLAGS
    h = hashlib.sha256()
    h.update(" ".join(f for f in FLAGS if not f.startswith("-I")).encode())
    for rel in KERNEL_SOURCES:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def kernel_stats_table(path: str, top: int = 12) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | total ms | average ms | min ms | max ms | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        ns = float(r["TotalDurationNs"])
        out.append(f"| `{r['Name']}` | {r['Calls']} | {ns / 1e6:.3f} | {float(r['AverageNs']) / 1e6:.3f} | "
                   f"{float(r['MinNs']) / 1e6:.3f} | {float(r['MaxNs']) / 1e6:.3f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def _per_dispatch(path: str, counter: str):
    """{kernel name: [(grid size, value) per dispatch]} for one counter (summed
    over the dimensions rocprofv3 may report separately)."""
    acc = defaultdict(float)
    meta = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        d = int(r["Dispatch_Id"])
        acc[d] += float(r["Counter_Value"])
        meta[d] = (r["Kernel_Name"], int(r["Grid_Size"]))
    by = defaultdict(list)
    for d in sorted(acc):
        by[meta[d][0]].append((meta[d][1], acc[d]))
    return by


def _mean_of(by, sub: str, largest: bool = False):
    """Mean counter value over the largest-grid dispatches of the kernel
    matching `sub` (the full launches, not a tuner's sample runs); with
    largest=True over the dispatches whose value is within 2x of the largest
    (the calibration copies, not the small uploads that use the same kernel)."""
    items = [gv for k, gvs in by.items() if sub in k for gv in gvs]
    if not items:
        raise SystemExit(f"no dispatch of a kernel matching {sub!r}")
    if largest:
        top = max(v for _, v in items)
        vals = [v for _, v in items if v >= 0.5 * top]
    else:
        gmax = max(g for g, _ in items)
        vals = [v for g, v in items if g == gmax]
    return sum(vals) / len(vals), len(vals), [k for k in by if sub in k][0]


def kernel_trace_table(path: str, top: int = 12) -> str:
    """Per (kernel, grid size) from a kernel_trace.csv: launches and mean /
    min / max duration, largest total first."""
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        ns = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        grid = int(r.get("Grid_Size_X", r.get("Grid_Size", 0)) or 0)
        acc[(r["Kernel_Name"], grid)].append(ns)
    rows = sorted(acc.items(), key=lambda kv: -sum(kv[1]))[:top]
    out = ["| kernel | grid (work-items) | launches | mean ms | min ms | max ms |", "|---|---|---|---|---|---|"]
    for (name, grid), v in rows:
        out.append(f"| `{name}` | {grid} | {len(v)} | {sum(v) / len(v) / 1e6:.3f} | {min(v) / 1e6:.3f} | "
                   f"{max(v) / 1e6:.3f} |")
    return "\n".join(out)


def traffic_record(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int) -> dict:
    fb = _per_dispatch(fetch_csv, "FETCH_SIZE")
    wb = _per_dispatch(write_csv, "WRITE_SIZE")
    cf, ncf, _ = _mean_of(fb, COPY_KERNEL, largest=True)
    cw, ncw, _ = _mean_of(wb, COPY_KERNEL, largest=True)
    kf, nkf, name = _mean_of(fb, kernel)
    kw, nkw, _ = _mean_of(wb, kernel)
    f_fetch = copy_bytes / cf  # bytes per counter unit, from the copy's reads
    f_write = copy_bytes / cw
    return {
        "kernel": name, "source_digest": source_digest(),
        "copy_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
        "fetch_factor": f_fetch, "write_factor": f_write,
        "fetch_kib_per_launch": kf, "write_kib_per_launch": kw, "launches": min(nkf, nkw),
        "fetch_bytes_per_launch": kf * f_fetch, "write_bytes_per_launch": kw * f_write,
        "traffic_bytes_per_launch": kf * f_fetch + kw * f_write,
    }


def counter_summary(csvs, kernel: str, evals: int) -> dict:
    """Per-launch SQ counters of the largest-grid dispatches of `kernel` from
    one or more `rocprofv3 --pmc` counter_collection.csv files, and the rates
    per 64-lane evaluation (evals = intersections per launch).  The largest
    grid is taken over all the files: a file whose launches of the kernel are
    all smaller (another, smaller workload) adds nothing."""
    acc = defaultdict(float)
    nl = defaultdict(int)
    gui = []
    tables = [list(csv.DictReader(open(path))) for path in csvs]
    grids = [int(r["Grid_Size"]) for rows in tables for r in rows if kernel in r["Kernel_Name"]]
    if not grids:
        raise SystemExit(f"{', '.join(csvs)}: no dispatch of {kernel!r}")
    gmax = max(grids)
    for rows in tables:
        part = defaultdict(float)
        seen = defaultdict(set)
        for r in rows:
            if kernel not in r["Kernel_Name"] or int(r["Grid_Size"]) != gmax:
                continue
            c = r["Counter_Name"]
            part[c] += float(r["Counter_Value"])
            seen[c].add(r["Dispatch_Id"])
        if "GRBM_GUI_ACTIVE" in part:  # one value per pass, averaged over the passes below
            gui.append(part.pop("GRBM_GUI_ACTIVE") / len(seen.pop("GRBM_GUI_ACTIVE")))
        for c, v in part.items():
            acc[c] += v
            nl[c] += len(seen[c])
    per = {c: v / max(nl[c], 1) for c, v in acc.items()}
    we = evals / 64.0
    out = {"counters_per_launch": per, "wave_evals_per_launch": we}
    if "SQ_INSTS_VALU" in per:
        out["valu_insts_per_wave_eval"] = per["SQ_INSTS_VALU"] / we
    if "SQ_INSTS_LDS" in per:
        out["lds_insts_per_wave_eval"] = per["SQ_INSTS_LDS"] / we
    if gui:
        cyc = sum(gui) / len(gui) / 8.0  # GRBM_GUI_ACTIVE is summed over the 8 XCDs
        out["gpu_cycles_per_launch"] = cyc
        if "SQ_LDS_IDX_ACTIVE" in per:
            out["lds_busy_fraction"] = per["SQ_LDS_IDX_ACTIVE"] / (cyc * 256)
        if "SQ_LDS_BANK_CONFLICT" in per and "SQ_LDS_IDX_ACTIVE" in per:
            out["lds_bank_conflict_fraction"] = per["SQ_LDS_BANK_CONFLICT"] / per["SQ_LDS_IDX_ACTIVE"]
    if "SQ_INSTS_LDS_LOAD_BANDWIDTH" in per:
        # the counter is in 64-byte units of bytes read by LDS instructions
        lb = per["SQ_INSTS_LDS_LOAD_BANDWIDTH"] * 64.0
        out["lds_load_bytes_per_launch"] = lb
        out["lds_load_bytes_per_lane_eval"] = lb / evals
        if gui:
            out["lds_load_bytes_per_clk_per_cu"] = lb / (out["gpu_cycles_per_launch"] * 256)
    if "SQ_ACTIVE_INST_VALU2" in per and "SQ_ACTIVE_INST_VALU" in per:
        out["valu_dual_issue_fraction"] = per["SQ_ACTIVE_INST_VALU2"] / per["SQ_ACTIVE_INST_VALU"]
    if "SQ_WAIT_ANY" in per and "SQ_WAVE_CYCLES" in per:
        out["wave_wait_fraction"] = per["SQ_WAIT_ANY"] / per["SQ_WAVE_CYCLES"]
    return out


def write_record(rec: dict, path: str, header: str = ""):
    with open(path, "w") as f:
        if header:
            f.write(header.rstrip() + "\n\n")
        for k, v in rec.items():
            f.write(f"{k}: {v}\n")


def comment_header(path: str) -> str:
    """The leading '#' lines of an existing record (kept when it is rewritten)."""
    if not os.path.exists(path):
        return ""
    out = []
    for line in open(path):
        if not line.startswith("#"):
            break
        out.append(line.rstrip("\n"))
    return "\n".join(out)


def read_record(path: str) -> dict | None:
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ": " in line and not line.startswith(("#", " ", "|", "`")):
            k, v = line.rstrip("\n").split(": ", 1)
            rec[k.strip()] = v.strip()
    return rec if "traffic_bytes_per_launch" in rec else None


def current_traffic(path: str) -> float | None:
    """Bytes per launch from a traffic record, or None when the record is
    missing or was taken on kernel sources other than the ones built now."""
    rec = read_record(path)
    if rec is None or rec.get("source_digest") != source_digest():
        return None
    return float(rec["traffic_bytes_per_launch"])


# Per-kernel rates kept in a counter record (the rest of counter_summary's
# output is context for the reader of the record).
COUNTER_FIELDS = ("valu_insts_per_wave_eval", "fma_f32_per_wave_eval", "lds_insts_per_wave_eval",
                  "lds_load_bytes_per_lane_eval", "lds_busy_fraction", "lds_load_bytes_per_clk_per_cu",
                  "wave_wait_fraction")


def counter_record(kernels: dict, csvs) -> dict:
    """{kernel substring: {field: value}} for every kernel of `kernels`
    ({substring: intersections per launch}), from rocprofv3 --pmc runs."""
    out = {}
    for k, evals in kernels.items():
        sm = counter_summary([c for c in csvs if _has_kernel(c, k)], k, int(evals))
        per = sm["counters_per_launch"]
        rec = {"evals_per_launch": int(evals)}
        if "SQ_INSTS_VALU_FMA_F32" in per:
            sm["fma_f32_per_wave_eval"] = per["SQ_INSTS_VALU_FMA_F32"] / sm["wave_evals_per_launch"]
        for f in COUNTER_FIELDS:
            if f in sm:
                rec[f] = sm[f]
        out[k] = rec
    return out


def _has_kernel(path: str, kernel: str) -> bool:
    with open(path) as f:
        return any(kernel in line for line in f)


def write_counter_record(rec: dict, path: str, header: str = ""):
    with open(path, "w") as f:
        if header:
            f.write(header.rstrip() + "\n\n")
        f.write(f"source_digest: {source_digest()}\n")
        for k, fields in rec.items():
            f.write(f"\n[{k}]\n")
            for n, v in fields.items():
                f.write(f"{n}: {v}\n")


def read_counter_record(path: str) -> tuple[str | None, dict]:
    if not os.path.exists(path):
        return None, {}
    digest, cur, out = None, None, {}
    for line in open(path):
        line = line.rstrip("\n")
        if line.startswith("#") or not line.strip():
            continue
        if line.startswith("[") and line.endswith("]"):
            cur = line[1:-1]
            out[cur] = {}
        elif ": " in line:
            k, v = line.split(": ", 1)
            if cur is None:
                if k == "source_digest":
                    digest = v.strip()
            else:
                out[cur][k.strip()] = float(v)
    return digest, out


def current_counters(path: str, kernel: str) -> dict | None:
    """The recorded rates of `kernel`, or None when the record is missing,
    holds no such kernel or was taken on other kernel sources."""
    digest, rec = read_counter_record(path)
    if digest != source_digest() or kernel not in rec:
        return None
    r = rec[kernel]
    need = ("valu_insts_per_wave_eval", "fma_f32_per_wave_eval", "lds_load_bytes_per_lane_eval")
    return r if all(n in r for n in need) else None


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        print(kernel_stats_table(argv[1]))
    elif len(argv) >= 2 and argv[0] == "trace":
        print(kernel_trace_table(argv[1]))
    elif len(argv) >= 4 and argv[0] == "counters":
        import json
        print(json.dumps(counter_summary(argv[3:], argv[1], int(float(argv[2]))), indent=1))
    elif len(argv) >= 4 and argv[0] == "counter-record" and "--" in argv:
        # counter-record <out.txt> <kernel>=<evals> ... -- <csv> ...
        cut = argv.index("--")
        kernels = {}
        for a in argv[2:cut]:
            k, e = a.rsplit("=", 1)
            kernels[k] = int(float(e))
        rec = counter_record(kernels, argv[cut + 1:])
        write_counter_record(rec, argv[1], header=comment_header(argv[1]))
        print(open(argv[1]).read())
    elif len(argv) == 6 and argv[0] == "traffic":
        rec = traffic_record(argv[1], argv[2], argv[3], int(argv[4]))
        write_record(rec, argv[5], header=comment_header(argv[5]))
        print("\n".join(f"{k}: {v}" for k, v in rec.items()))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
