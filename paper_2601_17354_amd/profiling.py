"""Turn rocprofv3 CSV output into the short text summaries kept in profiles/.

    python -m paper_2601_17354_amd.profiling stats <kernel_stats.csv> <out.txt> "<command>"
    python -m paper_2601_17354_amd.profiling pmc <fetch_dir> <write_dir> <kernel substring>
           <copy_bytes> <source file[,file...]> <out.txt> "<command>"

The PMC summary scales each kernel's FETCH_SIZE / WRITE_SIZE (KiB per
dispatch) by the ratio known-bytes / counter-reading of the plain copy kernel
(`k_copy16`, which reads and writes exactly copy_bytes) measured in the same
runs, and records the SHA-256 of the kernel's source so a reader can tell
whether the counters still describe the current code.
"""

from __future__ import annotations

import csv
import glob
import hashlib
import os
import sys


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


def summarize_pmc(fetch_dir, write_dir, kernel, copy_bytes, source, out_txt, command):
    f = _counter(fetch_dir, "FETCH_SIZE")
    w = _counter(write_dir, "WRITE_SIZE")
    name, fk, nf = _pick(f, kernel)
    _, wk, nw = _pick(w, kernel)
    _, fc, _ = _pick(f, "k_copy16")
    _, wc, _ = _pick(w, "k_copy16")
    kib = copy_bytes / 1024.0
    ff, fw = kib / fc, kib / wc
    traffic = (fk * ff + wk * fw) * 1024.0
    lines = [
        f"command: {command}",
        f"kernel: {_short(name)}",
        f"source: {_names(source)} sha256[:16]={source_sha(source)}",
        f"dispatches: fetch {nf}, write {nw}",
        f"FETCH_SIZE_KiB_per_dispatch: {fk:.1f}",
        f"WRITE_SIZE_KiB_per_dispatch: {wk:.1f}",
        f"copy_kernel_bytes_each_way: {copy_bytes}",
        f"copy_FETCH_SIZE_KiB: {fc:.1f}  (factor {ff:.4f})",
        f"copy_WRITE_SIZE_KiB: {wc:.1f}  (factor {fw:.4f})",
        f"fetch_bytes_per_launch: {fk * ff * 1024.0:.0f}",
        f"write_bytes_per_launch: {wk * fw * 1024.0:.0f}",
        f"traffic_bytes_per_launch: {traffic:.0f}",
    ]
    open(out_txt, "w").write("\n".join(lines) + "\n")


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
                      sys.argv[8])
    else:
        raise SystemExit(__doc__)
