"""HBM traffic of one kernel from two rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE).

Usage (after profiling a run that launches the kernel and one plain copy of a
known size, e.g. ``bench.py --calib-copy-mib 256``):

    python -m paper_1911_01353_amd.traffic --fetch F.csv --write W.csv \
        --kernel-regex 'fft_correlate_kernel<512,' --bench-name 'fft_correlate_kernel<S=512>' \
        --points P --copy-mib 256 --command '...'

FETCH_SIZE / WRITE_SIZE are in KiB per dispatch. Each is scaled by what the
same counter reads for the copy kernel (known bytes / measured bytes), summed
over the kernel's dispatches and divided by the algorithmic plane points of
those dispatches (``--points``). Writes ``profiles/hbm_traffic.json`` (read by
bench.py, keyed by the bench kernel name and the hash of the kernel sources)
and a text summary next to it.
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = {"fft": ["fft_correlate.hip", "jerk_internal.h"], "gemm": ["gemm_correlate.hip", "jerk_internal.h"]}


def source_sha(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def per_dispatch(path, counter):
    vals = defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        d = int(r["Dispatch_Id"])
        vals[d] += float(r["Counter_Value"])
        names[d] = r["Kernel_Name"]
    return vals, names


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--kernel-regex", required=True)
    ap.add_argument("--bench-name", required=True)
    ap.add_argument("--points", type=float, required=True)
    ap.add_argument("--copy-mib", type=float, required=True)
    ap.add_argument("--first", type=int, default=0,
                    help="only the first N matching dispatches in dispatch order (0: all), e.g. when later "
                         "parts of the profiled run launch the same kernel")
    ap.add_argument("--algo-write", type=float, default=4.0,
                    help="algorithmic bytes written per point, for the summary (4: the plane)")
    ap.add_argument("--command", default="")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "hbm_traffic.json"))
    a = ap.parse_args()
    fv, fn = per_dispatch(a.fetch, "FETCH_SIZE")
    wv, wn = per_dispatch(a.write, "WRITE_SIZE")
    rx = re.compile(a.kernel_regex)
    copy_bytes = a.copy_mib * (1 << 20)

    def calib(vals, names):
        cands = [v for d, v in vals.items() if "copy" in names[d].lower() or "elementwise" in names[d].lower()]
        best = max(cands)  # the calibration copy is by far the largest copy
        return copy_bytes / (best * 1024.0), best

    fscale, fcopy = calib(fv, fn)
    wscale, wcopy = calib(wv, wn)
    def pick(vals, names):
        ds = sorted(d for d in vals if rx.search(names[d]))
        return ds[: a.first] if a.first > 0 else ds

    fd, wd = pick(fv, fn), pick(wv, wn)
    fk = sum(fv[d] for d in fd)
    wk = sum(wv[d] for d in wd)
    nk = len(fd)
    fetch_b = fk * 1024.0 * fscale
    write_b = wk * 1024.0 * wscale
    kind = "gemm" if "gemm" in a.bench_name else "fft"
    ent = {
        "bytes_per_point": (fetch_b + write_b) / a.points,
        "fetch_bytes_per_point": fetch_b / a.points,
        "write_bytes_per_point": write_b / a.points,
        "fetch_scale": fscale, "write_scale": wscale,
        "copy_fetch_kib": fcopy, "copy_write_kib": wcopy, "copy_mib": a.copy_mib,
        "dispatches": nk, "points": a.points,
        "sources": SOURCES[kind], "source_sha": source_sha(SOURCES[kind]),
        "command": a.command,
    }
    data = json.load(open(a.out)) if os.path.exists(a.out) else {}
    data[a.bench_name] = ent
    json.dump(data, open(a.out, "w"), indent=1)
    txt = os.path.splitext(a.out)[0] + "_" + re.sub(r"[^A-Za-z0-9]+", "_", a.bench_name).strip("_") + ".txt"
    with open(txt, "w") as fh:
        fh.write(f"# HBM traffic of {a.bench_name} (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)\n")
        fh.write(f"# command: {a.command}\n")
        fh.write(f"# calibration copy {a.copy_mib:.0f} MiB: FETCH_SIZE read {fcopy:.0f} KiB (scale {fscale:.3f}),"
                 f" WRITE_SIZE read {wcopy:.0f} KiB (scale {wscale:.3f})\n")
        fh.write(f"dispatches {nk}, algorithmic points {a.points:.4e}\n")
        fh.write(f"fetch  {fetch_b / 1e9:.3f} GB  = {fetch_b / a.points:.3f} B/point\n")
        fh.write(f"write  {write_b / 1e9:.3f} GB  = {write_b / a.points:.3f} B/point "
                 f"(algorithmic write {a.algo_write:g} B/point)\n")
        fh.write(f"total  {(fetch_b + write_b) / a.points:.3f} B/point\n")
    print(json.dumps(ent))


if __name__ == "__main__":
    main()
