"""Summary of rocprofv3 counter runs (``--pmc ... --output-format csv``) for chosen kernels.

    python -m paper_1911_01353_amd.counters RUN1_counter_collection.csv [RUN2...] \\
        --kernel-regex 'gemm_correlate_kernel' --group-by name --command '...' --out profiles/x.txt

Sums every counter over the matching dispatches (per kernel name, or all together), prints the
per-dispatch averages, and the derived figures the counters allow:

- MFMA work: 512 flops per SQ_INSTS_VALU_MFMA_MOPS_{BF16,F16}; SQ_VALU_MFMA_BUSY_CYCLES counts the
  busy cycles of every SIMD's matrix unit (one per 1024 bf16 flops), so over a dispatch of known
  duration (``--duration-ms``, per dispatch, e.g. from HIP events) and shader clock
  (``--clock-mhz``) the busy fraction is BUSY / (duration x clock x 256 CUs x 4 SIMDs); without a
  duration, the busy cycles per SIMD-cycle of CU activity, BUSY / (4 SQ_BUSY_CU_CYCLES), are given
  (GRBM_GUI_ACTIVE does not count one clock of one engine, so it is not used for rates);
- wave lifetime: SQ_WAVE_CYCLES / SQ_WAVES, and the shares of the wave cycles spent waiting
  (SQ_WAIT_INST_ANY) or issuing VALU work (SQ_ACTIVE_INST_VALU);
- HBM bytes: FETCH_SIZE and WRITE_SIZE (KiB) as measured (calibration is traffic.py's job).
"""

from __future__ import annotations

import argparse
import csv
import re
from collections import defaultdict

N_CU = 256
MFMA_PEAK = 2.5e15


def load(paths, rx):
    """{kernel name: {counter: [value per dispatch]}} over the matching dispatches."""
    per = defaultdict(lambda: defaultdict(lambda: defaultdict(float)))
    for path in paths:
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"]
            if not rx.search(name):
                continue
            per[name][r["Counter_Name"]][(path, int(r["Dispatch_Id"]))] += float(r["Counter_Value"])
    return {k: {c: list(d.values()) for c, d in v.items()} for k, v in per.items()}


def derived(c, duration_ms=0.0, clock_mhz=0.0):
    out = {}
    n = max((len(v) for v in c.values()), default=0)
    tot = {k: sum(v) for k, v in c.items()}
    busy = tot.get("SQ_VALU_MFMA_BUSY_CYCLES")
    if busy is not None and duration_ms > 0 and clock_mhz > 0:
        simd_cycles = n * duration_ms * 1e-3 * clock_mhz * 1e6 * N_CU * 4
        out["mfma_busy_frac"] = busy / simd_cycles
    if busy is not None and tot.get("SQ_BUSY_CU_CYCLES"):
        out["mfma_busy_per_simd_cycle_of_cu_activity"] = busy / (4 * tot["SQ_BUSY_CU_CYCLES"])
    for dt in ("BF16", "F16"):
        key = f"SQ_INSTS_VALU_MFMA_MOPS_{dt}"
        if key in tot and duration_ms > 0:
            rate = 512 * tot[key] / (n * duration_ms * 1e-3)
            out[f"mfma_{dt.lower()}_TFLOPs"] = rate / 1e12
            out[f"mfma_{dt.lower()}_frac_of_peak"] = rate / MFMA_PEAK
    if tot.get("SQ_WAVES"):
        if "SQ_WAVE_CYCLES" in tot:
            out["wave_cycles_per_wave"] = tot["SQ_WAVE_CYCLES"] / tot["SQ_WAVES"]
        if "SQ_WAIT_INST_ANY" in tot and tot.get("SQ_WAVE_CYCLES"):
            out["wait_inst_any_frac_of_wave_cycles"] = tot["SQ_WAIT_INST_ANY"] / tot["SQ_WAVE_CYCLES"]
        if "SQ_ACTIVE_INST_VALU" in tot and tot.get("SQ_WAVE_CYCLES"):
            out["active_valu_frac_of_wave_cycles"] = tot["SQ_ACTIVE_INST_VALU"] / tot["SQ_WAVE_CYCLES"]
    if "SQ_LDS_BANK_CONFLICT" in tot and tot.get("SQ_LDS_IDX_ACTIVE"):
        out["lds_bank_conflict_frac"] = tot["SQ_LDS_BANK_CONFLICT"] / tot["SQ_LDS_IDX_ACTIVE"]
    out["dispatches"] = n
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("csv", nargs="+")
    ap.add_argument("--kernel-regex", default=".")
    ap.add_argument("--group-by", choices=["name", "all"], default="name")
    ap.add_argument("--duration-ms", type=float, default=0.0, help="duration of one dispatch (for rates)")
    ap.add_argument("--clock-mhz", type=float, default=0.0, help="shader clock during the dispatches")
    ap.add_argument("--title", default="")
    ap.add_argument("--command", default="")
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)
    data = load(a.csv, re.compile(a.kernel_regex))
    if a.group_by == "all":
        merged = defaultdict(list)
        for c in data.values():
            for k, v in c.items():
                merged[k] += v
        data = {a.kernel_regex: dict(merged)}
    lines = []
    if a.title:
        lines.append(f"# {a.title}")
    if a.command:
        lines.append(f"# command: {a.command}")
    for name, c in sorted(data.items()):
        lines.append(f"kernel {name}")
        for k in sorted(c):
            v = c[k]
            lines.append(f"  {k:34s} total {sum(v):.6g}  per dispatch {sum(v) / len(v):.6g}  ({len(v)} dispatches)")
        for k, v in derived(c, a.duration_ms, a.clock_mhz).items():
            lines.append(f"  = {k:32s} {v:.4g}")
    text = "\n".join(lines) + "\n"
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)
    print(text, end="")


if __name__ == "__main__":
    main()
