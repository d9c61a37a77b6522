"""Algorithmic byte models of the compositing kernels, and the short text
summaries of rocprofv3 CSV output kept in profiles/.

    python -m paper_2601_17354_amd.profiling stats <kernel_stats.csv> <out.txt> "<command>"
    python -m paper_2601_17354_amd.profiling pmc <fetch_dir> <write_dir> <kernel substring>
           <copy_bytes> <source file[,file...]> <out.txt> "<command>"
           [<fetch_log.json>,<write_log.json> <kind> [<phase>]]
    python -m paper_2601_17354_amd.profiling trace <kernel_trace.csv> <kernel substring> <work_log.json> <kind>
           <out.txt> "<command>" [<phase>]
    python -m paper_2601_17354_amd.profiling counters <run_dir> <kernel substring> <out.txt> "<command>"
           [<work_log.json> <kind> [<phase> [<source file[,file...]>]]]

The PMC summary scales each kernel's FETCH_SIZE / WRITE_SIZE (KiB per
dispatch) by the ratio known-bytes / counter-reading of the plain copy kernel
(`k_copy16`, which reads and writes exactly copy_bytes) measured in the same
runs, and records the SHA-256 of the kernel's source so a reader can tell
whether the counters still describe the current code.  Given the work log
the profiled program wrote (pair count P, trace entries E and pixels of
every launch, in launch order), it also writes the algorithmic bytes of
exactly the profiled launches beside the counters.
"""

from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys


# Algorithmic bytes per unit of work of the compositing launches.
#
# Scope-table model (per pixel, per (tile, Gaussian) pair, per trace entry):
#   render_fwd   20 B/pixel written (colour, T_final, n_contrib) + 40 B/pair
#                gathered (the splat's 2D attributes) + 20 B/entry written
#                (the trace record) when the trace is recorded;
#   render_bwd   cached: 20 B/entry read + 28 B/pixel (dL/dimage and the
#                pixel state) + 40 B/pair gathered + 36 B/pair of atomic
#                payload (nine fields); recompute: 32 B/pixel + 76 B/pair.
# Design model (this implementation's layout): a splat record gathers 48 B
# and its sorted id 4 B; the trace keeps per (tile, splat) one 8-byte ballot
# mask per wave of 64 pixels (4 waves for 16x16 tiles: 32 B per pair,
# written forward and read backward) and 12 B per entry (C_in; 16 B with
# alpha in the paper's layout); forward pixels
# write 24 B with the trace (count too), backward pixels read 12 B
# (dL/dimage; 20 B for recompute, which also reads T_final and n_contrib).
def sec8d_bytes(kernel: str, cached: bool, P: int, E: int, pixels: int) -> int:
    if kernel == "render_fwd":
        return 20 * pixels + 40 * P + (20 * E if cached else 0)
    if cached:
        return 20 * E + 28 * pixels + 76 * P
    return 32 * pixels + 76 * P


def design_bytes(kernel: str, cached: bool, P: int, E: int, pixels: int, waves: int = 4,
                 entry_bytes: int = 12) -> int:
    masks = 8 * waves
    if kernel == "render_fwd":
        return 24 * pixels + (52 + masks) * P + entry_bytes * E if cached else 20 * pixels + 52 * P
    return 12 * pixels + (88 + masks) * P + entry_bytes * E if cached else 20 * pixels + 88 * P


def source_sha(paths: str) -> str:
    """SHA-256 (first 16 hex digits) of one source file, or of several
    comma-separated files concatenated in order."""
    h = hashlib.sha256()
    for p in paths.split(","):
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def _names(paths: str) -> str:
    return "+".join(os.path.basename(p) for p in paths.split(","))


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0] if "(" in name else name


def summarize_stats(stats_csv: str, out_txt: str, command: str, top: int = 25) -> None:
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"command: {command}", "", f"{'kernel':70s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for r in rows[:top]:
        lines.append(f"{_short(r['Name'])[:70]:70s} {int(r['Calls']):6d} "
                     f"{float(r['AverageNs']) / 1e3:10.2f} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                     f"{float(r['Percentage']):6.2f}")
    open(out_txt, "w").write("\n".join(lines) + "\n")


def _counter(run_dir: str, counter: str):
    """{kernel name: [values per dispatch]} for one counter."""
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    out = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def _pick(d: dict, sub: str):
    keys = [k for k in d if sub in k]
    if not keys:
        raise KeyError(f"no kernel matching {sub!r} in {list(d)[:8]}")
    vals = [v for k in keys for v in d[k]]
    return keys[0], sum(vals) / len(vals), len(vals)


def _dispatch_rows(run_dir: str, counter: str, kernel: str):
    """[(dispatch id, counter value)] of the dispatches of the one kernel
    whose name contains `kernel`, in dispatch order."""
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    rows, names = [], set()
    for f in files:
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter and kernel in r["Kernel_Name"]:
                rows.append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
                names.add(r["Kernel_Name"])
    if len(names) != 1:
        raise SystemExit(f"{kernel!r} matches {len(names)} kernels")
    return sorted(rows), names.pop()


def _logged(work_log: str, kind: str, cached: bool, n_dispatch: int):
    """The logged launches of one kind, in launch order; the log must hold
    exactly the profiled launches.  Entries carry P, E, pixels, ok (the
    buffers held the pass), tag (camera) and phase (part of the run)."""
    log = [w for w in json.load(open(work_log)) if w["kernel"] == kind and w["cached"] == cached]
    if len(log) != n_dispatch:
        raise SystemExit(f"work log has {len(log)} {kind} launches, the counters {n_dispatch}")
    return log


def _work_means(log):
    """Mean P, E, pixels and algorithmic bytes (both models) of launches."""
    n = len(log)
    mean = lambda k: sum(w[k] for w in log) / n
    kind, cached = log[0]["kernel"], log[0]["cached"]
    sec = sum(sec8d_bytes(kind, cached, w["P"], w["E"], w["pixels"]) for w in log) / n
    des = sum(design_bytes(kind, cached, w["P"], w["E"], w["pixels"]) for w in log) / n
    tags = sorted({w["tag"] for w in log if w.get("tag") is not None})
    return dict(P=mean("P"), E=mean("E"), pixels=mean("pixels"), sec8d=sec, design=des, views=tags)


def _keep(w, phase):
    return w.get("ok", True) and (phase is None or w.get("phase") == phase)


def summarize_pmc(fetch_dir, write_dir, kernel, copy_bytes, source, out_txt, command, work_log=None,
                  kind=None, phase=None):
    """FETCH_SIZE / WRITE_SIZE of one kernel scaled by the copy kernel's
    readings; with a work log, the means are over the launches whose buffers
    held the pass (launches that overflowed while the buffers were being
    sized are dropped from counters and bytes alike) and, if given, of one
    phase of the run."""
    fr, name = _dispatch_rows(fetch_dir, "FETCH_SIZE", kernel)
    wr, _ = _dispatch_rows(write_dir, "WRITE_SIZE", kernel)
    _, fc, _ = _pick(_counter(fetch_dir, "FETCH_SIZE"), "k_copy16")
    _, wc, _ = _pick(_counter(write_dir, "WRITE_SIZE"), "k_copy16")
    keep_f = [True] * len(fr)
    keep_w = [True] * len(wr)
    work = None
    if work_log:
        # the FETCH_SIZE run's work log, then (comma-separated) the WRITE_SIZE run's
        logs = work_log.split(",")
        cached = "true" in name or "cached" in name
        lf = _logged(logs[0], kind, cached, len(fr))
        lw = _logged(logs[-1], kind, cached, len(wr))
        keep_f = [_keep(w, phase) for w in lf]
        keep_w = [_keep(w, phase) for w in lw]
        work = _work_means([w for w, k in zip(lf, keep_f) if k])
    fk = [v for (_, v), k in zip(fr, keep_f) if k]
    wk = [v for (_, v), k in zip(wr, keep_w) if k]
    fk, wk = sum(fk) / len(fk), sum(wk) / len(wk)
    kib = copy_bytes / 1024.0
    ff, fw = kib / fc, kib / wc
    traffic = (fk * ff + wk * fw) * 1024.0
    lines = [
        f"command: {command}",
        f"kernel: {_short(name)}",
        f"source: {_names(source)} sha256[:16]={source_sha(source)}",
        f"dispatches: fetch {len(fr)}, write {len(wr)}; used {sum(keep_f)} / {sum(keep_w)} "
        f"(launches that held the pass)",
        f"FETCH_SIZE_KiB_per_dispatch: {fk:.1f}",
        f"WRITE_SIZE_KiB_per_dispatch: {wk:.1f}",
        f"copy_kernel_bytes_each_way: {copy_bytes}",
        f"copy_FETCH_SIZE_KiB: {fc:.1f}  (factor {ff:.4f})",
        f"copy_WRITE_SIZE_KiB: {wc:.1f}  (factor {fw:.4f})",
        f"fetch_bytes_per_launch: {fk * ff * 1024.0:.0f}",
        f"write_bytes_per_launch: {wk * fw * 1024.0:.0f}",
        f"traffic_bytes_per_launch: {traffic:.0f}",
    ]
    if work:
        lines += [
            f"work_log: {kind} launches {sum(keep_f)}{'' if phase is None else ' of phase ' + phase}, "
            f"views {work['views']}",
            f"pairs_per_launch: {work['P']:.0f}",
            f"entries_per_launch: {work['E']:.0f}",
            f"pixels_per_launch: {work['pixels']:.0f}",
            f"algorithmic_bytes_per_launch: {work['sec8d']:.0f}  (scope-table model)",
            f"algorithmic_bytes_design_per_launch: {work['design']:.0f}  (design model)",
            f"traffic_over_algorithmic: {traffic / work['sec8d']:.3f}  (design model {traffic / work['design']:.3f})",
        ]
    open(out_txt, "w").write("\n".join(lines) + "\n")


def summarize_trace(trace_csv, kernel, work_log, kind, out_txt, command, phase=None):
    """Average duration of one kernel's dispatches from a kernel trace, over
    the launches that held the pass, with their work and the bandwidth the
    scope-table bytes imply at the profiler's own timing."""
    rows, names = [], set()
    for r in csv.DictReader(open(trace_csv)):
        if kernel in r["Kernel_Name"]:
            rows.append((int(r["Dispatch_Id"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9))
            names.add(r["Kernel_Name"])
    if len(names) != 1:
        raise SystemExit(f"{kernel!r} matches {len(names)} kernels")
    name = names.pop()
    rows.sort()
    cached = "true" in name or "cached" in name
    log = _logged(work_log, kind, cached, len(rows))
    kept = [(d, w) for (_, d), w in zip(rows, log) if _keep(w, phase)]
    avg = sum(d for d, _ in kept) / len(kept)
    work = _work_means([w for _, w in kept])
    lines = [
        f"command: {command}",
        f"kernel: {_short(name)}",
        f"dispatches: {len(rows)}, used {len(kept)} (launches that held the pass"
        f"{'' if phase is None else ', phase ' + phase}), views {work['views']}",
        f"avg_duration_us: {avg * 1e6:.2f}",
        f"pairs_per_launch: {work['P']:.0f}",
        f"entries_per_launch: {work['E']:.0f}",
        f"pixels_per_launch: {work['pixels']:.0f}",
        f"algorithmic_bytes_per_launch: {work['sec8d']:.0f}  (scope-table model)",
        f"achieved_GBps: {work['sec8d'] / avg / 1e9:.1f}  (fraction of 8 TB/s: {work['sec8d'] / avg / 8e12:.3f})",
    ]
    open(out_txt, "w").write("\n".join(lines) + "\n")


# Vector issue of the chip: a SIMD issues one wave64 VALU instruction every
# 4 cycles (16 lanes per cycle without packed FP32), 4 SIMDs per CU, 256 CUs
# at 2.4 GHz: 614.4e9 wave instructions/s (78.6 TFLOP/s of FP32 FMA).
VALU_WAVE_INSTR_PER_S = 256 * 2.4e9
XCDS = 8  # GRBM_GUI_ACTIVE is summed over the eight XCDs


def summarize_counters(run_dir, kernel, out_txt, command, work_log=None, kind=None, phase=None, source=None):
    """Mean per dispatch of every counter collected for one kernel, with the
    vector-issue time its VALU instruction count implies, the GPU-active time
    and the LDS bank-conflict rate.  With the run's work log (and a phase),
    only the launches that held the pass (of that phase) are averaged."""
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    per, name = {}, None
    for fpath in files:
        for r in csv.DictReader(open(fpath)):
            if kernel not in r["Kernel_Name"]:
                continue
            name = r["Kernel_Name"]
            per.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
    if not per:
        raise SystemExit(f"no counters for {kernel!r}")
    ids = sorted(per)
    note = f"dispatches {len(ids)}"
    if work_log:
        log = _logged(work_log, kind, "true" in name or "cached" in name, len(ids))
        ids = [d for d, w in zip(ids, log) if _keep(w, phase)]
        note += f", used {len(ids)}" + ("" if phase is None else f" of phase {phase}")
    acc = {}
    for d in ids:
        for c, v in per[d].items():
            acc.setdefault(c, []).append(v)
    lines = [f"command: {command}", f"kernel: {_short(name)}", f"averaged over: {note}"]
    if source:
        lines.append(f"source: {_names(source)} sha256[:16]={source_sha(source)}")
    mean = {c: sum(v) / len(v) for c, v in acc.items()}
    for c in sorted(acc):
        lines.append(f"{c}_per_dispatch: {mean[c]:.1f}")
    if "SQ_INSTS_VALU" in mean:
        issue = mean["SQ_INSTS_VALU"] / VALU_WAVE_INSTR_PER_S
        lines.append(f"valu_issue_time_us: {issue * 1e6:.1f}  (VALU wave instructions / 614.4e9 per s)")
        if "GRBM_GUI_ACTIVE" in mean:
            active = mean["GRBM_GUI_ACTIVE"] / XCDS / 2.4e9
            lines.append(f"gpu_active_us: {active * 1e6:.1f}  (GRBM_GUI_ACTIVE / 8 XCDs / 2.4 GHz)")
            lines.append(f"valu_issue_fraction: {issue / active:.3f}")
    if mean.get("SQ_LDS_IDX_ACTIVE"):
        lines.append(f"lds_bank_conflict_rate: {mean.get('SQ_LDS_BANK_CONFLICT', 0.0) / mean['SQ_LDS_IDX_ACTIVE']:.4f}"
                     "  (SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE)")
    open(out_txt, "w").write("\n".join(lines) + "\n")


def read_summary(summary_txt: str) -> dict:
    kv = {}
    for line in open(summary_txt):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv


def read_issue_fraction(summary_txt: str, source: str):
    """valu_issue_fraction from a counters summary, or None if the summary is
    missing or the kernel source changed since the counters were taken."""
    if not os.path.exists(summary_txt):
        return None
    kv = read_summary(summary_txt)
    if f"sha256[:16]={source_sha(source)}" not in kv.get("source", ""):
        return None
    try:
        return float(kv["valu_issue_fraction"].split()[0])
    except (KeyError, ValueError):
        return None


def read_traffic(summary_txt: str, source: str):
    """traffic_bytes_per_launch from a summary, or None if the summary is
    missing or the kernel source changed since the counters were taken."""
    if not os.path.exists(summary_txt):
        return None
    kv = {}
    for line in open(summary_txt):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if f"sha256[:16]={source_sha(source)}" not in kv.get("source", ""):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        summarize_stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "pmc":
        summarize_pmc(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), sys.argv[6], sys.argv[7],
                      sys.argv[8], *(sys.argv[9:12]))
    elif sys.argv[1] == "counters":
        summarize_counters(*sys.argv[2:10])
    elif sys.argv[1] == "trace":
        summarize_trace(*sys.argv[2:9])
    else:
        raise SystemExit(__doc__)
