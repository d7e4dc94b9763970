"""Times single width groups of a search on chosen paths (one GPU).

For each requested tap count, the width group of the lattice with that many taps is searched
over a seeded unit-power noise spectrum on each requested path, the plane written into a slab
buffer (every point goes to HBM), and the launches are timed with HIP events on the stream they
run on. One JSON line per (group, path): points/s, plane-write GB/s, and for the MFMA paths the
matrix-core rate (8 K flops per output point per product, three products for split-BF16).

    python -m paper_1911_01353_amd.groupbench --nbins 4194304 --zmax 200 --wmax 600 \\
        --taps 48,64,128 --paths split_bf16,fft --reps 5

Useful under ``rocprofv3`` to collect counters of one kernel at one tap count.
"""

from __future__ import annotations

import argparse
import json
import sys


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--nbins", type=int, default=1 << 22)
    ap.add_argument("--zmax", type=float, default=200.0)
    ap.add_argument("--wmax", type=float, default=600.0)
    ap.add_argument("--taps", default="48,64,128", help="tap counts of the groups to time (comma-separated)")
    ap.add_argument("--paths", default="split_bf16,fft", help="paths: fft, split_bf16, fp16 (comma-separated)")
    ap.add_argument("--members", type=int, default=0, help="templates of each group to search (0 = all)")
    ap.add_argument("--seg-len", type=int, default=0, help="FFT segment length (0 = the plan's default)")
    ap.add_argument("--tpb", type=int, default=0, help="FFT templates per block (0 = the plan's default)")
    ap.add_argument("--ept", type=int, default=0, help="FFT elements per thread (0 = the plan's default)")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=191102)
    ap.add_argument("--digest", action="store_true",
                    help="also print a checksum of the plane's bits (equal for bit-identical kernels)")
    args = ap.parse_args(argv)

    import numpy as np
    import torch

    import paper_1911_01353_amd as J

    if not torch.cuda.is_available():
        raise SystemExit("groupbench needs a GPU")
    n = args.nbins
    g = torch.Generator(device="cuda").manual_seed(args.seed)
    re = torch.randn(n, device="cuda", generator=g) / np.sqrt(2.0)
    im = torch.randn(n, device="cuda", generator=g) / np.sqrt(2.0)
    spec = torch.complex(re, im).contiguous()
    stream = torch.cuda.current_stream()
    for path in args.paths.split(","):
        plan = J.Plan(n, args.zmax, args.wmax, 2.0, 20.0, path=path)
        groups = plan.groups()
        want = [int(t) for t in args.taps.split(",")]
        sel = [i for i, gi in enumerate(groups) if gi["taps"] in want]
        for gidx in sel:
            gi = groups[gidx]
            if path == "fft" and (args.seg_len or args.tpb or args.ept):
                plan.set_group(gidx, args.seg_len or gi["seg_len"], args.tpb or gi["templates_per_block"],
                               path, args.ept)
        bank = plan.new_bank()
        plan.build_templates(bank)
        torch.cuda.synchronize()
        for gidx in sel:
            gi = plan.group(gidx)
            m = gi["n_members"] if args.members <= 0 else min(args.members, gi["n_members"])
            slab = torch.empty((m, 2 * n), dtype=torch.float32, device="cuda")
            for _ in range(args.warmup):
                plan.search_members(bank, spec, slab, gidx, 0, m)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(args.reps)]
            for e0, e1 in ev:
                e0.record(stream)
                plan.search_members(bank, spec, slab, gidx, 0, m)
                e1.record(stream)
            torch.cuda.synchronize()
            ms = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
            med = ms[len(ms) // 2] * 1e-3
            points = 2 * n * m
            K = gi["taps"]
            line = {"path": path, "group": gidx, "taps": K, "members": m, "seg_len": gi["seg_len"],
                    "templates_per_block": gi["templates_per_block"], "nbins": n, "ms_median": med * 1e3,
                    "ms_min": ms[0], "points_per_s": points / med, "write_GBps": 4 * points / med / 1e9}
            if args.digest:
                line["digest"] = int(torch.sum(slab.view(torch.int32), dtype=torch.int64))
            if path in ("split_bf16", "fp16"):
                prods = 3 if path == "split_bf16" else 1
                line["mfma_TFLOPs"] = 8 * K * prods * points / med / 1e12
            print(json.dumps(line), flush=True)
            del slab
        plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
