"""Summaries of rocprofv3 output for the committed profiles.

    python -m paper_2609_07842_amd.profsum trace  <dir> [--out file.md] [--title T] [--cmd C]
    python -m paper_2609_07842_amd.profsum traffic <fetch_dir> <write_dir> [--sq <sq_dir>]
                                                   --workload W --out file.json [--cmd C ...]

`trace` reads the kernel-trace CSV of a `rocprofv3 --kernel-trace --stats` run and writes per
kernel the number of dispatches and the mean, median and total duration.  The list-build
kernels launch on every step and exit at once unless a build is due, so their dispatches
are split at a duration threshold into real builds and empty launches.

`traffic` reads two `rocprofv3 --pmc` runs (FETCH_SIZE, then WRITE_SIZE, both in KiB per
dispatch) and converts them to bytes with the factors measured on the run's last large
device copy (a 512 MiB copy kernel: FETCH_SIZE counts 64-byte units of 128-byte requests
on gfx950, so its factor is about 2), per dispatch of the hot-path kernels (list-build
kernels only over the dispatches that built).  The JSON it writes carries the sha256 of the
kernel source, so that readers can tell whether the counters still describe the kernels.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(HERE, "csrc", "vbc_kernels.hip")

# short names of the kernels of a time step (template arguments stripped)
# (the force pass with the energy and virial sums on is told apart by its template
# arguments, see short_name)
SHORT = {"k_force": "force", "k_count": "count", "k_embed": "embed", "k_nlist": "nlist",
         "k_resort": "resort", "k_worklist": "worklist", "k_kick_drift": "kick",
         "k_reduce": "reduce", "k_thermo_acc": "thermo"}
BUILD_KERNELS = ("nlist", "resort")
COPY_BYTES = 512 * 2**20


def source_sha256() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def short_name(kernel: str) -> str:
    head = kernel.split("(")[0]
    base = head.split("<")[0].strip().split("::")[-1]
    if base == "k_force" and "<" in head:
        # k_force<Real, MULTI, THERMO, ONE>: the pass with the energy and virial sums on
        args = [a.strip() for a in head.split("<", 1)[1].rsplit(">", 1)[0].split(",")]
        if len(args) > 2 and args[2] == "true":
            return "force_sums"
    return SHORT.get(base, base)


def _csv_files(d: str, suffix: str):
    return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))


def _read_rows(d: str, suffix: str):
    rows = []
    for fn in _csv_files(d, suffix):
        with open(fn, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no *{suffix} under {d}")
    return rows


def _col(row, *names):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    raise KeyError(names)


def trace_rows(d: str):
    """(short name, duration ns, full name) per dispatch of a kernel-trace run, in the order
    the dispatches started."""
    out = []
    for r in _read_rows(d, "kernel_trace.csv"):
        name = _col(r, "Kernel_Name", "KernelName")
        t0 = int(_col(r, "Start_Timestamp", "BeginNs"))
        t1 = int(_col(r, "End_Timestamp", "EndNs"))
        out.append((t0, short_name(name), t1 - t0, name))
    out.sort(key=lambda t: t[0])
    return [t[1:] for t in out]


def split_builds(durs):
    """Dispatches of a list-build kernel that built (duration above a third of the longest)."""
    if not durs:
        return [], []
    cut = max(durs) / 3.0
    return [d for d in durs if d > cut], [d for d in durs if d <= cut]


def trace_summary(d: str, last: int = 0):
    """Per kernel: dispatches, mean, median and total duration (with last > 0, of its last
    `last` dispatches only, e.g. the steps after a long relaxation)."""
    per = {}
    for k, dur, _ in trace_rows(d):
        per.setdefault(k, []).append(dur)
    if last > 0:
        per = {k: v[-last:] for k, v in per.items()}
    out = {}
    for k, durs in sorted(per.items()):
        e = {"dispatches": len(durs), "mean_us": statistics.fmean(durs) / 1e3,
             "median_us": statistics.median(durs) / 1e3, "total_ms": sum(durs) / 1e6}
        if k in BUILD_KERNELS:
            real, empty = split_builds(durs)
            e.update(builds=len(real), build_mean_us=statistics.fmean(real) / 1e3 if real else None,
                     empty_mean_us=statistics.fmean(empty) / 1e3 if empty else None)
        out[k] = e
    return out


def counter_rows(d: str, counter: str):
    """(short name, value, dispatch id) per dispatch for one counter of a --pmc run."""
    out = []
    for r in _read_rows(d, "counter_collection.csv"):
        if _col(r, "Counter_Name") != counter:
            continue
        out.append((short_name(_col(r, "Kernel_Name")), float(_col(r, "Counter_Value")),
                    int(_col(r, "Dispatch_Id", "Correlation_Id"))))
    return out


def _per_dispatch(rows):
    """Sum counter values that rocprofv3 reports per dispatch in several rows."""
    acc = {}
    for k, v, did in rows:
        key = (k, did)
        acc[key] = acc.get(key, 0.0) + v
    per = {}
    for (k, did), v in sorted(acc.items(), key=lambda t: t[0][1]):
        per.setdefault(k, []).append(v)
    return per


def _calibration(rows):
    """Counter value of the last copy dispatch: the profiled run ends with a 512 MiB device
    copy (earlier copies have other sizes, e.g. the bench's 1 GiB bandwidth probe)."""
    last = None
    for k, v, did in rows:
        if "copy" in k.lower() and (last is None or did > last[0]):
            last = (did, v)
    return None if last is None else last[1]


def traffic(fetch_dir: str, write_dir: str, sq_dir: str | None = None):
    frows = counter_rows(fetch_dir, "FETCH_SIZE")
    wrows = counter_rows(write_dir, "WRITE_SIZE")
    fetch = _per_dispatch(frows)
    write = _per_dispatch(wrows)
    copy_kib = COPY_BYTES / 1024
    f_cal = _calibration(frows)
    w_cal = _calibration(wrows)
    if not f_cal or not w_cal:
        raise SystemExit("no copy dispatch found for the calibration")
    ff, wf = copy_kib / f_cal, copy_kib / w_cal
    kernels = {}
    for k in ("force", "force_sums", "count", "embed", "nlist", "resort", "kick", "thermo"):
        fv, wv = fetch.get(k, []), write.get(k, [])
        if not fv or not wv:
            continue
        if k in BUILD_KERNELS:
            # dispatches that built: their traffic is far above the empty launches'
            cut = max(fv) / 3.0
            sel = [i for i, v in enumerate(fv) if v > cut and i < len(wv)]
            fv = [fv[i] for i in sel]
            wv = [wv[i] for i in sel]
        fk, wk = statistics.fmean(fv), statistics.fmean(wv)
        kernels[k] = {"dispatches": len(fv), "fetch_kib_raw": fk, "write_kib_raw": wk,
                      "read_bytes": fk * 1024 * ff, "write_bytes": wk * 1024 * wf,
                      "traffic_bytes": fk * 1024 * ff + wk * 1024 * wf}
    if "nlist" in kernels and "resort" in kernels:
        kernels["build"] = {"traffic_bytes": kernels["nlist"]["traffic_bytes"] + kernels["resort"]["traffic_bytes"],
                            "read_bytes": kernels["nlist"]["read_bytes"] + kernels["resort"]["read_bytes"],
                            "write_bytes": kernels["nlist"]["write_bytes"] + kernels["resort"]["write_bytes"],
                            "parts": ["resort", "nlist"]}
    return {"calibration": {"copy_bytes": COPY_BYTES, "fetch_kib": f_cal, "write_kib": w_cal,
                            "fetch_factor": ff, "write_factor": wf},
            "kernels": kernels}


def counters(dirs):
    """Mean value per dispatch of every counter in the given --pmc runs, per kernel of a
    time step (list-build kernels: the dispatches that built, told apart by their VALU
    instruction count, or by the run's first counter)."""
    out = {}
    for d in dirs:
        names = []
        for r in _read_rows(d, "counter_collection.csv"):
            n = _col(r, "Counter_Name")
            if n not in names:
                names.append(n)
        per = {n: _per_dispatch(counter_rows(d, n)) for n in names}
        key = "SQ_INSTS_VALU" if "SQ_INSTS_VALU" in per else names[0]
        for k in ("force", "force_sums", "count", "embed", "nlist", "resort", "kick", "thermo"):
            sel = None
            if k in BUILD_KERNELS and per[key].get(k):
                ref = per[key][k]
                cut = max(ref) / 3.0
                sel = [i for i, v in enumerate(ref) if v > cut]
            for n in names:
                vals = per[n].get(k, [])
                if sel is not None:
                    vals = [vals[i] for i in sel if i < len(vals)]
                if vals:
                    out.setdefault(k, {})[n] = statistics.fmean(vals)
                    out[k].setdefault("dispatches", len(vals))
    return out


def _md_trace(title, cmd, summ):
    lines = [f"# Kernel trace: {title}", "", "Command:", "", f"    {cmd}", "",
             "| kernel | dispatches | mean us | median us | total ms | real builds | mean us per build |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for k, e in sorted(summ.items(), key=lambda t: -t[1]["total_ms"]):
        b = e.get("builds")
        bm = e.get("build_mean_us")
        lines.append(f"| {k} | {e['dispatches']} | {e['mean_us']:.1f} | {e['median_us']:.1f} | "
                     f"{e['total_ms']:.2f} | {'' if b is None else b} | {'' if bm is None else f'{bm:.1f}'} |")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--out")
    t.add_argument("--title", default="")
    t.add_argument("--cmd", default="")
    t.add_argument("--last", type=int, default=0, help="only each kernel's last N dispatches")
    c = sub.add_parser("traffic")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--workload", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--cmd", action="append", default=[])
    q = sub.add_parser("counters")
    q.add_argument("dirs", nargs="+")
    q.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.what == "counters":
        rec = {"source_sha256": source_sha256(), "kernels": counters(a.dirs)}
        with open(a.out, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec["kernels"], indent=1))
        return 0
    if a.what == "trace":
        summ = trace_summary(a.dir, a.last)
        text = _md_trace(a.title, a.cmd, summ)
        if a.out:
            with open(a.out, "w") as fh:
                fh.write(text)
        print(text)
    else:
        rec = traffic(a.fetch_dir, a.write_dir)
        rec = {"workload": a.workload, "source_sha256": source_sha256(), "commands": a.cmd, **rec}
        with open(a.out, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec["kernels"], indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
