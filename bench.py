#!/usr/bin/env python3
"""Throughput benchmark of the jerk-search matched filter on one MI355X.

A step is one full search of the 2^22-bin spectrum (2^23 float32 samples,
four seeded tones) over the 201 x 61 = 12261-template lattice (zmax 200,
wmax 600, dz 2, dw 20) with half-bin r spacing: 1.03e11 plane points. The
plane (411 GB in FP32) does not fit in HBM, so each step writes it as slabs
of up to 476 template rows of one width group into one resident slab buffer
(every point is written to HBM; later slabs overwrite earlier ones). Inputs and the template bank are in
HBM before the timed region; template generation is timed separately.

Prints one JSON line (see the keys below). ``--gpus`` above 1 is refused:
this build runs on one GPU.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
MFMA_BF16_TFLOPS = 2500.0
MFMA_FP16_TFLOPS = 2500.0
FP32_VECTOR_PUBLISHED_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--path", default="auto", choices=["auto", "fft", "split_bf16", "fp16"])
    ap.add_argument("--slab-gb", type=float, default=16.0, help="slab buffer size (GB)")
    ap.add_argument("--compare-paths", type=int, default=1,
                    help="also time the FP32 and split-BF16 paths alone (steps each)")
    ap.add_argument("--cpu-templates", type=int, default=8,
                    help="templates (full rows) in the oracle's timed sample; 0 skips cpu_baseline")
    ap.add_argument("--errors", type=int, default=1, help="measure plane errors on the 2^15-bin search")
    ap.add_argument("--autotune", type=int, default=1, help="autotune the plan before timing (untimed)")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests per warm serving pass (one per offered load); 0 skips serving")
    ap.add_argument("--serve-cold-requests", type=int, default=48,
                    help="requests of the cold closed-loop pass that measures the service rate")
    ap.add_argument("--serve-load", default="0.5,0.8",
                    help="offered loads (arrival rate / service rate), comma-separated: one warm pass each")
    ap.add_argument("--batch-items", type=int, default=256,
                    help="spectra in the batched leg (uneven 2^20..2^22 bins); 0 skips it")
    ap.add_argument("--rocfft-groups", type=int, default=4,
                    help="width groups timed against an unfused rocFFT (torch.fft) overlap-save (0 = skip)")
    ap.add_argument("--rocfft-members", type=int, default=16, help="templates per group in that comparison")
    ap.add_argument("--cand-rows", type=int, default=512,
                    help="plane rows of the 2^22-bin search timed through candidate selection (0 = skip)")
    ap.add_argument("--cand-sigma", type=float, default=6.0, help="candidate threshold in row sigmas")
    ap.add_argument("--fused-reps", type=int, default=3,
                    help="time the whole search with fused candidate selection (no plane) this many times "
                         "(0 = skip)")
    ap.add_argument("--harm-templates", type=int, default=1,
                    help="time harmonic sums (H = 2, 4, 8) over a 1159-template plane of the 2^22-bin spectrum")
    ap.add_argument("--prep", type=int, default=1,
                    help="time the device spectrum preparation of a 2^23-sample series")
    ap.add_argument("--small-reps", type=int, default=200,
                    help="time the 2^15-bin search per repetition inside a graph of this many (0 = skip)")
    ap.add_argument("--save-plan", default="", help="write the main plan's per-group configuration (JSON)")
    ap.add_argument("--load-plan", default="", help="use a saved per-group configuration instead of autotuning")
    ap.add_argument("--copy-gib", type=float, default=4.0,
                    help="measure achievable HBM bandwidth with a device copy and a fill of this size (0 = skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the main leg, copy a buffer of this size once (HBM counter calibration)")
    return ap.parse_args()


def kernel_name(g):
    if g["path"] == 0:
        return f"fft_correlate_kernel<S={g['seg_len']},E={g['fft_ept']}>"
    return "gemm_correlate_kernel<split_bf16>" if g["path"] == 1 else "gemm_correlate_kernel<fp16>"


def launch_counts(g, m, nbins):
    """Algorithmic work of one launch of group g over m templates and nbins bins.

    FFT path (FP32 vector): per segment one forward FFT per template block, per
    (segment, template, phase) a complex multiply (6S), an inverse FFT
    (5 S log2 S) and the power of the U = S - K + 1 kept lags (3U); nominal FFT counts.
    MFMA path: 8 K real flops per output point per product (3 products for
    split-BF16, 1 for FP16).
    Bytes: 4 per plane point written plus 8 per spectrum bin read.
    """
    points = 2 * nbins * m
    bytes_ = 4 * points + 8 * nbins
    if g["path"] == 0:
        S, K, tpb = g["seg_len"], g["taps"], g["templates_per_block"]
        U = S - K + 1
        n_seg = math.ceil(nbins / U)
        n_tb = math.ceil(m / tpb)
        fft = 5 * S * math.log2(S)
        flops = n_seg * (n_tb * fft + m * 2 * (6 * S + fft + 3 * U))
    else:
        flops = points * 8 * g["taps"] * (3 if g["path"] == 1 else 1)
    return points, flops, bytes_


def source_sha(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1911_01353_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kname, launch_points_avg):
    """HBM bytes per launch from the committed counter summary, if it matches the current source."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
        ent = data.get(kname)
        if not ent or ent.get("source_sha") != source_sha(ent["sources"]):
            return None
        return ent["bytes_per_point"] * launch_points_avg
    except Exception:
        return None


def run_search_steps(J, torch, plan, bank, spec, slab, rows, steps, timing):
    """Runs `steps` full searches, the plane cut into slabs of up to `rows` members of one width
    group each (every launch works on whole template blocks); records (group, members, events)."""
    groups = plan.groups()
    recs = []
    for _ in range(steps):
        for g, gi in enumerate(groups):
            for m0 in range(0, gi["n_members"], rows):
                m1 = min(gi["n_members"], m0 + rows)
                if timing:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                plan.search_members(bank, spec, slab, g, m0, m1)
                if timing:
                    e1.record()
                    recs.append((g, m1 - m0, e0, e1))
    return recs


def time_path(J, torch, spec, n, path, steps, warmup, slab_gb, want_kernels, autotune=True, load_plan="",
              save_plan=""):
    plan = J.Plan(n, 200.0, 600.0, 2.0, 20.0, path=path)
    t_tune = 0.0
    if load_plan:
        cfg = json.load(open(load_plan))
        for g, c in enumerate(cfg["groups"]):
            plan.set_group(g, c["seg_len"], c["templates_per_block"], c["path"], c.get("fft_ept", 0))
    elif autotune and path in ("auto", "fft"):
        t0 = time.perf_counter()
        plan.autotune(spec)
        t_tune = time.perf_counter() - t0
    if save_plan:
        json.dump({"workload": "2^22 bins, zmax 200, wmax 600, dz 2, dw 20", "path": path,
                   "groups": [{k: g[k] for k in ("taps", "seg_len", "templates_per_block", "path", "fft_ept")}
                              for g in plan.groups()]}, open(save_plan, "w"), indent=1)
    info = plan.info()
    bank = plan.new_bank()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.build_templates(bank)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    T = info["n_templates"]
    row_bytes = 2 * n * 4
    rows = max(1, min(T, int(slab_gb * 1e9 // row_bytes)))
    slab = torch.empty((rows, 2 * n), dtype=torch.float32, device="cuda")
    run_search_steps(J, torch, plan, bank, spec, slab, rows, warmup, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = run_search_steps(J, torch, plan, bank, spec, slab, rows, steps, want_kernels)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    groups = plan.groups()
    del slab
    out = {"plan": plan, "bank": bank, "wall": wall, "t_build": t_build, "t_tune": t_tune, "T": T, "rows": rows, "kernels": None,
           "groups": groups}
    if want_kernels:
        agg = {}
        for g, m, e0, e1 in recs:
            gi = groups[g]
            ms_t = e0.elapsed_time(e1) * 1e-3
            pts, fl, by = launch_counts(gi, m, n)
            k = kernel_name(gi)
            d = agg.setdefault(k, {"launches": 0, "time": 0.0, "points": 0, "flops": 0.0, "bytes": 0.0,
                                   "path": gi["path"]})
            d["launches"] += 1
            d["time"] += ms_t
            d["points"] += pts
            d["flops"] += fl
            d["bytes"] += by
        out["kernels"] = agg
    return out


def kernel_table(ks):
    return {k: {"launches": v["launches"], "time_s": v["time"], "points": v["points"],
                "avg_launch_us": v["time"] / v["launches"] * 1e6, "points_per_s": v["points"] / v["time"],
                "tflops": v["flops"] / v["time"] / 1e12, "hbm_GBps": v["bytes"] / v["time"] / 1e9,
                **({"mfma_frac": v["flops"] / v["time"] / 1e12 / MFMA_BF16_TFLOPS} if v["path"] else {})}
            for k, v in ks.items()}


def peak_probe():
    """Measured arithmetic ceilings (MFMA bf16, FP32 FMA) from the package's peakprobe program,
    run as a child process; None when it has not been built."""
    import subprocess
    exe = os.path.join(ROOT, "paper_1911_01353_amd", "peakprobe")
    if not os.path.exists(exe):
        return None
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    if res.returncode != 0:
        print(f"[bench] peakprobe failed: {res.stderr.strip()}", file=sys.stderr, flush=True)
        return None
    out = json.loads(res.stdout)
    out["what"] = ("v_mfma_f32_32x32x16_bf16 and v_fma_f32 loops with no memory traffic over every SIMD at "
                   "8 waves per SIMD; plane-like tile stores (U float2 per workgroup, U = 512: whole lines, "
                   "U = 481: lines shared by tiles), plain and non-temporal "
                   "(paper_1911_01353_amd/peakprobe.hip), best of 3, HIP events")
    return out


def hbm_copy_leg(torch, gib=4.0, reps=10):
    """Achievable HBM bandwidth on this device: a device-to-device copy (read + write) and a
    fill (write only; the plane store is write-dominated) of `gib` GiB, timed with events."""
    nel = int(gib * (1 << 30)) // 4
    a = torch.ones(nel, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    b.copy_(a)
    b.fill_(2.0)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        b.copy_(a)
    ev[1].record()
    for _ in range(reps):
        b.fill_(3.0)
    ev[2].record()
    torch.cuda.synchronize()
    t_copy = ev[0].elapsed_time(ev[1]) * 1e-3 / reps
    t_fill = ev[1].elapsed_time(ev[2]) * 1e-3 / reps
    by = nel * 4
    del a, b
    return {"bytes": by, "copy_GBps": 2 * by / t_copy / 1e9, "fill_GBps": by / t_fill / 1e9,
            "copy_frac_of_spec": 2 * by / t_copy / 1e9 / HBM_PEAK_GBS,
            "fill_frac_of_spec": by / t_fill / 1e9 / HBM_PEAK_GBS,
            "what": f"torch copy_ and fill_ of a {gib:g} GiB float32 buffer, {reps} reps each, HIP events"}


def rocfft_leg(J, torch, plan, bank, spec, n, n_groups, members):
    """The fused kernels against unfused rocFFT overlap-save on the same rows (best segment length
    of the library path from 1024..8192), with the two planes compared."""
    from paper_1911_01353_amd.comparator import overlap_save, template_spectra
    groups = plan.groups()
    order = sorted(range(len(groups)), key=lambda g: groups[g]["taps"])
    pick = sorted({order[int(round(i * (len(order) - 1) / max(1, n_groups - 1)))] for i in range(n_groups)})
    res = []
    for g in pick:
        gi = groups[g]
        m = min(members, gi["n_members"])
        m0 = (gi["n_members"] - m) // 2
        K = gi["taps"]
        ours = torch.empty((m, 2 * n), dtype=torch.float32, device="cuda")
        ref = torch.empty_like(ours)
        plan.search_members(bank, spec, ours, g, m0, m0 + m)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        reps = 3
        ev[0].record()
        for _ in range(reps):
            plan.search_members(bank, spec, ours, g, m0, m0 + m)
        ev[1].record()
        torch.cuda.synchronize()
        t_ours = ev[0].elapsed_time(ev[1]) * 1e-3 / reps
        off = gi["taps_offset"] + (m0 * 2 * K) * 16
        taps = bank[off: off + m * 2 * K * 16].view(torch.complex128).view(m, 2, K)
        best = None
        for S in (1024, 2048, 4096, 8192):
            if S < 2 * K:
                continue
            spectra = template_spectra(taps, S)
            overlap_save(spec, spectra, K, ref)
            torch.cuda.synchronize()
            ev[0].record()
            for _ in range(reps):
                overlap_save(spec, spectra, K, ref)
            ev[1].record()
            torch.cuda.synchronize()
            t = ev[0].elapsed_time(ev[1]) * 1e-3 / reps
            if best is None or t < best[1]:
                best = (S, t)
            del spectra
        rowmean = ref.mean(dim=1, keepdim=True)
        diff = ((ours - ref).abs() / torch.maximum(ref, rowmean)).max().item()
        pts = m * 2 * n
        res.append({"group": g, "taps": K, "path": ["fft_fp32", "split_bf16", "fp16"][gi["path"]],
                    "members": m, "ours_points_per_s": pts / t_ours, "rocfft_points_per_s": pts / best[1],
                    "rocfft_seg_len": best[0], "speedup": best[1] / t_ours, "max_rel_diff": diff})
        print(f"[bench] rocFFT comparison group {g} K={K}: speedup {best[1] / t_ours:.2f} "
              f"(diff {diff:.1e})", file=sys.stderr, flush=True)
        del ours, ref
    return res


def candidates_leg(J, torch, plan, bank, spec, n, rows, k_sigma, reps=5):
    """Row statistics and threshold peak-finding over a slab of real search rows (each kernel reads
    the slab once: 4 B per point), timed with events on the current stream."""
    groups = plan.groups()
    members = plan.members()
    slab = torch.empty((rows, 2 * n), dtype=torch.float32, device="cuda")
    tmpl = []
    r = 0
    for g, gi in enumerate(groups):
        if r >= rows:
            break
        m = min(gi["n_members"], rows - r)
        plan.search_members(bank, spec, slab[r: r + m], g, 0, m)
        tmpl += members[gi["first_member"]: gi["first_member"] + m].tolist()
        r += m
    rt = torch.tensor(tmpl, dtype=torch.int32, device="cuda")
    stats = torch.empty((rows, 2), dtype=torch.float64, device="cuda")
    ws = torch.empty(max(1, J.stats_workspace_bytes(rows, 2 * n)), dtype=torch.uint8, device="cuda")
    cap = 1 << 22
    out = torch.empty((cap, 4), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_stats = t_cand = 0.0
    for i in range(reps + 1):
        count.zero_()
        ev[0].record()
        J.plane_stats(slab, stats, ws=ws)
        ev[1].record()
        J.find_candidates(slab, stats, k_sigma, out, count, row_template=rt)
        ev[2].record()
        torch.cuda.synchronize()
        if i:
            t_stats += ev[0].elapsed_time(ev[1]) * 1e-3 / reps
            t_cand += ev[1].elapsed_time(ev[2]) * 1e-3 / reps
    pts = rows * 2 * n
    found = int(count.item())
    del slab, out
    return {"rows": rows, "points": pts, "k_sigma": k_sigma, "candidates": found,
            "stats_ms": t_stats * 1e3, "candidates_ms": t_cand * 1e3,
            "points_per_s": pts / (t_stats + t_cand),
            "stats_GBps": 4 * pts / t_stats / 1e9, "candidates_GBps": 4 * pts / t_cand / 1e9,
            "stats_hbm_frac": 4 * pts / t_stats / 1e9 / HBM_PEAK_GBS,
            "candidates_hbm_frac": 4 * pts / t_cand / 1e9 / HBM_PEAK_GBS}


def search_candidates_leg(J, torch, spec, n, k_sigma, reps=3):
    """The whole search (every template) with candidate selection fused in: no plane is written.
    FFT path, autotuned plan (untimed). Speculative level 0.9 (1 + k) (the noise rows' thresholds lie
    near 1 + k on a unit-mean-power spectrum), staging slots sized by the library from that level.
    Timed with events around the whole call, median of `reps`."""
    import numpy as np
    plan = J.Plan(n, 200.0, 600.0, 2.0, 20.0, path="fft")
    plan.autotune(spec)
    bank = plan.new_bank()
    plan.build_templates(bank)
    T = plan.info()["n_templates"]
    groups = plan.groups()
    pre = 0.9 * (1.0 + k_sigma)
    ws = torch.empty(plan.search_candidates_workspace_bytes(n, pre, 0, T), dtype=torch.uint8, device="cuda")
    cap = 1 << 26
    out = torch.empty((cap, 4), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    stats = torch.empty((T, 2), dtype=torch.float64, device="cuda")
    times = []
    for i in range(reps + 1):
        count.zero_()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.search_candidates(bank, spec, k_sigma, pre, out, count, 0, T, stats=stats, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        if i:
            times.append(e0.elapsed_time(e1) * 1e-3)
    t = float(np.median(times))
    pts = 2 * n * T
    found = int(count.item())
    mean_sigma = stats.mean(dim=0).cpu().tolist()
    ws_bytes = ws.numel()
    del out, ws, bank
    plan.close()
    return {"templates": T, "points": pts, "k_sigma": k_sigma, "pre_level": pre, "workspace_bytes": ws_bytes,
            "candidates": found, "ms": t * 1e3, "ms_all": [x * 1e3 for x in times], "points_per_s": pts / t,
            "row_mean_sigma_avg": mean_sigma}


def small_search_leg(J, torch, reps=200):
    """The 2^15-bin search (147 templates, 9.6e6 points) on each path, timed per repetition
    inside a captured graph of `reps` searches (launch overhead excluded)."""
    import synth
    cfg = synth.CONFIGS["bins2e15_z20_w60"]
    spec = torch.from_numpy(synth.make_spectrum(cfg)).cuda()
    n = spec.shape[0]
    res = {"workload": "2^15 bins, zmax 20, wmax 60 (147 templates), plane in HBM", "reps": reps}
    for path in ("fft", "split_bf16", "fp16", "auto"):
        plan = J.Plan(n, cfg.zmax, cfg.wmax, cfg.dz, cfg.dw, path=path)
        if path in ("fft", "auto"):
            plan.autotune(spec)
        bank = plan.new_bank()
        plan.build_templates(bank)
        T = plan.info()["n_templates"]
        out = torch.empty((T, 2 * n), dtype=torch.float32, device="cuda")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            plan.search(bank, spec, out, 0, T)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(reps):
                plan.search(bank, spec, out, 0, T)
        g.replay()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        g.replay()
        ev[1].record()
        torch.cuda.synchronize()
        t = ev[0].elapsed_time(ev[1]) * 1e-3 / reps
        pts = T * 2 * n
        res[path] = {"us_per_search": t * 1e6, "points_per_s": pts / t,
                     "groups": [{"taps": g["taps"], "path": ["fft", "split_bf16", "fp16"][g["path"]],
                                 "seg_len": g["seg_len"], "templates_per_block": g["templates_per_block"]}
                                for g in plan.groups()]}
        del g, out, bank
        plan.close()
    return res


def spectrum_leg(J, torch, n_samples, reps=5):
    """Device spectrum preparation (FP64) of an N(0,1) series of n_samples float32 samples;
    algorithmic bytes: 4 B per sample read + 8 B per bin written."""
    g = torch.Generator(device="cuda")
    g.manual_seed(191106)
    x = torch.randn(n_samples, generator=g, device="cuda", dtype=torch.float32)
    out, ws = J.prepare_spectrum(x)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        J.prepare_spectrum(x, out=out, ws=ws)
    ev[1].record()
    torch.cuda.synchronize()
    t = ev[0].elapsed_time(ev[1]) * 1e-3 / reps
    by = 4 * n_samples + 8 * (n_samples // 2)
    return {"n_samples": n_samples, "ms": t * 1e3, "samples_per_s": n_samples / t, "GBps": by / t / 1e9,
            "hbm_frac": by / t / 1e9 / HBM_PEAK_GBS}


def harmonic_touched_bytes(plan, n_r, H):
    """HBM bytes the harmonic sum cannot avoid: every 128-byte line of the plane that holds a
    point some output reads, plus the output. Harmonic h reads its row at stride h, so for
    h <= 32 every line of the span [0, h (n_pf - 1)] is touched although only 1/h of its points
    are used; rows read by several (fundamental, h) pairs count once, at their longest span."""
    info = plan.info()
    n_z, n_w = info["n_z"], info["n_w"]
    i0, Jw = n_z // 2, n_w // 2
    n_zf, n_wf, n_pf = plan.harmonic_shape(n_r, H)
    lines = {}
    for row in range(n_zf * n_wf):
        di, dj = row % n_zf - n_zf // 2, row // n_zf - n_wf // 2
        for h in range(1, H + 1):
            t = (Jw + h * dj) * n_z + (i0 + h * di)
            nl = -(-(h * (n_pf - 1) + 1) * 4 // 128) if h <= 32 else n_pf
            lines[t] = max(lines.get(t, 0), nl)
    return sum(min(nl * 128, 4 * n_r) for nl in lines.values()) + 4 * n_pf * n_zf * n_wf


def harmonics_leg(J, torch, spec, n, reps=5):
    """Harmonic sums of the full plane of a 61 x 19 = 1159-template grid (zmax 60, wmax 180) of the
    2^22-bin spectrum (38.9 GB), for H = 2, 4, 8 (279, 75 and 21 fundamental rows of 2^23 / H
    points); algorithmic bytes 4 (H + 1) per output point. Harmonic h reads its row at stride h,
    so the bytes of the 128-byte lines touched are reported beside them."""
    plan = J.Plan(n, 60.0, 180.0, 2.0, 20.0, path="fft")
    bank = plan.new_bank()
    plan.build_templates(bank)
    T = plan.info()["n_templates"]
    plane = torch.empty((T, 2 * n), dtype=torch.float32, device="cuda")
    plan.search(bank, spec, plane, 0, T)
    res = {"workload": f"full plane of {T} templates (zmax 60, wmax 180) x {2 * n} points"}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for H in (2, 4, 8):
        out = plan.harmonic_sum(plane, H)
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            plan.harmonic_sum(plane, H, out=out)
        ev[1].record()
        torch.cuda.synchronize()
        t = ev[0].elapsed_time(ev[1]) * 1e-3 / reps
        pts = out.numel()
        touched = harmonic_touched_bytes(plan, 2 * n, H)
        res[f"H{H}"] = {"output_points": pts, "ms": t * 1e3, "points_per_s": pts / t,
                        "GBps": 4 * (H + 1) * pts / t / 1e9, "hbm_frac": 4 * (H + 1) * pts / t / 1e9 / HBM_PEAK_GBS,
                        "touched_bytes": touched, "touched_GBps": touched / t / 1e9,
                        "touched_frac": touched / t / 1e9 / HBM_PEAK_GBS}
        del out
    del plane, bank
    plan.close()
    return res


def cpu_host():
    """Host CPU description and the worker count the CPU legs may use (at most 16)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count(), "affinity": avail, "workers": max(1, min(16, avail))}


def cpu_baseline_templates(n_templates_sample):
    """The templates whose full rows the oracle computes for cpu_baseline (evenly spaced, so
    both ends of the lattice, the widest and the narrowest rows, are in the sample)."""
    import numpy as np
    T = 201 * 61
    return [int(t) for t in np.linspace(0, T - 1, n_templates_sample)]


def cpu_baseline(spec, n_templates_sample):
    """The FP64 oracle, single-threaded, on full rows of a sample of templates. Returns the
    timing record and the oracle rows (FP64), which the headline's error is measured against."""
    import numpy as np
    from oracle import Grid, oracle_plane
    grid = Grid(200.0, 600.0, 2.0, 20.0)
    ts = cpu_baseline_templates(n_templates_sample)
    assert grid.n_templates == 201 * 61
    t0 = time.perf_counter()
    plane = oracle_plane(spec, grid, templates=ts)
    dt = time.perf_counter() - t0
    pts = plane.size
    return {"value": pts / dt, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(ts)} full rows (2^23 points each, templates {ts}) of the 2^22-bin search, "
                      f"FP64 numpy direct correlation incl. template quadrature, {dt:.1f} s"}, ts, plane


def headline_error(gpu_rows, ts, oracle_rows):
    """Floored relative power error (whole rows, row-mean floor) of the timed plan's rows against
    the oracle's rows of the same templates, and whether each row's peak is the oracle's."""
    import numpy as np
    from oracle import error_summary, peak_index
    s = error_summary(gpu_rows, oracle_rows)
    peaks = [peak_index(gpu_rows[i:i + 1]) == peak_index(oracle_rows[i:i + 1]) for i in range(len(ts))]
    return {"max": s["max"], "rms": s["rms"], "row_peaks_match": bool(np.all(peaks)), "templates": ts,
            "points": int(gpu_rows.size), "bar": 1e-4,
            "what": "whole plane rows of the timed plan (same bank, same kernels) against the FP64 oracle's rows"}


_POOL_SPEC = None


def _oracle_row(t):
    from oracle import Grid, oracle_plane
    return oracle_plane(_POOL_SPEC, Grid(200.0, 600.0, 2.0, 20.0), templates=[t]).size


def cpu_oracle_pool(spec, n_rows, workers):
    """The same FP64 oracle over a process pool, one worker per allowed host core."""
    import multiprocessing as mp
    import numpy as np
    from oracle import Grid
    global _POOL_SPEC
    _POOL_SPEC = spec
    grid = Grid(200.0, 600.0, 2.0, 20.0)
    ts = [int(t) for t in np.linspace(0, grid.n_templates - 1, n_rows)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        pts = sum(pool.map(_oracle_row, ts, chunksize=1))
    dt = time.perf_counter() - t0
    _POOL_SPEC = None
    return {"value": pts / dt, "unit": "points/s", "cores": workers, "kind": "oracle_process_pool",
            "sample": f"{len(ts)} full rows of the 2^22-bin search over {workers} processes, {dt:.1f} s"}


def cpu_fft_overlap_save(spec, n_templates, workers):
    """A CPU FFT search of the kind the paper compares with: FP32 overlap-save with scipy.fft on
    all allowed cores, templates made beforehand (untimed). Taps come from the oracle."""
    import numpy as np
    import scipy.fft as sfft
    from oracle import Grid, template_taps
    grid = Grid(200.0, 600.0, 2.0, 20.0)
    x = np.asarray(spec, dtype=np.complex64)
    n = x.shape[0]
    ts = [int(t) for t in np.linspace(0, grid.n_templates - 1, n_templates)]
    total_t = 0.0
    pts = 0
    for t in ts:
        zb, w, h = grid.params(t)
        K = 2 * h
        S = 1024
        while S < 4 * K:
            S *= 2
        U = S - K + 1
        c = np.zeros((2, S), dtype=np.complex128)
        c[0, :K] = template_taps(zb, w, h, 0)
        c[1, :K] = template_taps(zb, w, h, 1)
        H = sfft.ifft(c, norm="forward").astype(np.complex64)
        n_seg = -(-n // U)
        xp = np.zeros(K // 2 - 1 + n_seg * U + S, dtype=np.complex64)
        xp[K // 2 - 1: K // 2 - 1 + n] = x
        idx = np.arange(n_seg)[:, None] * U + np.arange(S)[None, :]
        t0 = time.perf_counter()
        segs = xp[idx]
        f = sfft.fft(segs, workers=workers)
        row = np.empty(2 * n, dtype=np.float32)
        for ph in (0, 1):
            y = sfft.ifft(f * H[ph][None, :], workers=workers)[:, :U].reshape(-1)[:n]
            row[ph::2] = (y.real * y.real + y.imag * y.imag)
        total_t += time.perf_counter() - t0
        pts += row.size
    return {"value": pts / total_t, "unit": "points/s", "cores": workers, "kind": "fft_overlap_save_fp32_scipy",
            "sample": f"{len(ts)} full rows of the 2^22-bin search (segments 1024..8192 >= 4K), {total_t:.1f} s"}


def plane_errors(J, torch):
    """Max/RMS floored relative power error of each path on the full 2^15-bin plane."""
    import numpy as np
    import synth
    from oracle import Grid, error_summary, oracle_plane, peak_index
    cfg = synth.CONFIGS["bins2e15_z20_w60"]
    spec_np = synth.make_spectrum(cfg)
    grid = Grid(cfg.zmax, cfg.wmax, cfg.dz, cfg.dw)
    ora = oracle_plane(spec_np, grid)
    spec = torch.from_numpy(spec_np).cuda()
    res = {}
    for path in ("fft", "split_bf16", "fp16"):
        plan = J.Plan(spec_np.shape[0], cfg.zmax, cfg.wmax, cfg.dz, cfg.dw, path=path)
        bank = plan.new_bank()
        plan.build_templates(bank)
        plane = torch.empty((grid.n_templates, 2 * spec_np.shape[0]), dtype=torch.float32, device="cuda")
        plan.search(bank, spec, plane)
        torch.cuda.synchronize()
        got = plane.cpu().numpy()
        s = error_summary(got, ora)
        res[path] = {"max": s["max"], "rms": s["rms"], "peak_match": peak_index(got) == peak_index(ora)}
        plan.close()
    return res


def serving_leg(J, torch, n_req, load, n_cold=48, top_k=10):
    """Poisson stream of search requests (lengths 2^18..2^23 bins, zmax 50..300, wmax 3 zmax,
    FP32 / split-BF16 half and half) through the request server: n_cold of them all at once with a
    cold template cache (the service rate), then n_req at each offered load with every grid's bank
    resident. Latency is host time from submit to completion, reported over all requests and per
    path; every request also returns its global top-k (k row peaks)."""
    import numpy as np
    import synth
    reqs = synth.serving_requests(max(n_req, n_cold), 1.0)
    # one resident spectrum per length class (seeded), shared by the requests of that length
    specs = {}
    for r in reqs:
        if r["n_samples"] not in specs:
            x = synth.time_series(r["n_samples"], r["seed"], r["tones"])
            specs[r["n_samples"]] = torch.from_numpy(synth.spectrum_from_series(x)).cuda()
    arena = torch.empty(96 << 30, dtype=torch.uint8, device="cuda")
    srv = J.Server(arena, max_active=4, queue_capacity=4 * len(reqs), tiles_per_launch=1 << 16)

    def stats(lat, pts):
        return {"requests": len(lat), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "max_s": float(lat.max()), "request_points_per_s": float(pts.sum() / lat.sum())}

    def run_pass(rs, rate):
        t0 = time.perf_counter()
        tickets = []
        for r in rs:
            due = t0 + r["arrival_s"] / rate
            while True:
                now = time.perf_counter()
                if now >= due:
                    break
                time.sleep(min(0.002, due - now))
            tickets.append(srv.submit(specs[r["n_samples"]], r["zmax"], r["wmax"], r["dz"], r["dw"],
                                      path="split_bf16" if r["split_bf16"] else "fft", top_k=top_k))
            if len(tickets) % 50 == 0:
                print(f"[bench] serving: {len(tickets)} of {len(rs)} submitted", file=sys.stderr, flush=True)
        res = [srv.wait(t, 600.0) for t in tickets]
        wall = time.perf_counter() - t0
        lat = np.array([x["t_done"] - x["t_submit"] for x in res])
        pts = np.array([x["points"] for x in res], dtype=np.float64)
        ok = all(x["status"] == 0 for x in res) and all(x["top_count"] == top_k for x in res)
        split = np.array([r["split_bf16"] for r in rs])
        out = {"requests": len(res), "ok": ok, "p50_s": float(np.percentile(lat, 50)),
               "p99_s": float(np.percentile(lat, 99)), "p99.9_s": float(np.percentile(lat, 99.9)),
               "max_s": float(lat.max()), "wall_s": wall, "points_per_s": float(pts.sum() / wall),
               "points": float(pts.sum())}
        for name, sel in (("fft", ~split), ("split_bf16", split)):
            if sel.any():
                out[name] = stats(lat[sel], pts[sel])
        return out

    st0 = srv.stats()
    cold = run_pass(reqs[:n_cold], 1e9)   # all at once: the service capacity with cold banks
    mu = cold["requests"] / cold["wall_s"]
    print(f"[bench] serving: cold pass {cold['wall_s']:.1f} s, service rate {mu:.2f} requests/s", file=sys.stderr,
          flush=True)
    warm = {}
    for rho in load:
        warm[f"{rho:g}"] = dict(run_pass(reqs[:n_req], rho * mu), load=rho, arrival_rate_hz=rho * mu)
        w = warm[f"{rho:g}"]
        print(f"[bench] serving: load {rho:g}: p50 {w['p50_s']:.2f} s, p99 {w['p99_s']:.2f} s", file=sys.stderr,
              flush=True)
    st = srv.stats()
    srv.close()
    del arena
    return {"loads": list(load), "service_rate_hz": mu, "cold_closed_loop": cold, "warm_poisson": warm,
            "bank_builds": st["bank_builds"], "launches": st["launches"] - st0["launches"],
            "shared_launches": st["shared_launches"] - st0["shared_launches"],
            "max_requests_in_flight": st["max_in_flight"], "top_k": top_k,
            "workload": "synth.serving_requests(seed 191105): lengths 2^18..2^23 bins, zmax even in [50, 300], "
                        "wmax 3 zmax, dz 2, dw 20, 50% tones, 50% split-BF16; per-row peaks and top-k results; "
                        "request_points_per_s = the path's points over its requests' summed latency"}


def batch_leg(J, torch, n_items, cand_items=32):
    """256 uneven de-dispersion-trial spectra (2^20, 2^21, 2^22 bins; zmax 100, wmax 300; 10% with
    one injected jerk tone) through jerk_batch_search: one graph-replayed launch per template slab
    over all spectra. Each time series is made on the GPU (seeded noise plus its tone) and turned
    into its unit-power spectrum by jerk_spectrum_prepare (not timed). Every spectrum writes its own
    plane region (slab rows x 2n floats each, all in HBM at once), so no two spectra share output
    memory. The flat launch (the default) is the headline; the persistent kernel is timed beside it."""
    import synth
    specs_meta = synth.batch_spectra_specs(n_items)
    specs = []
    for n_samp, seed, tones in specs_meta:
        x = synth.time_series_device(n_samp, seed, tones)
        spec, ws_p = J.prepare_spectrum(x)
        torch.cuda.synchronize()
        specs.append(spec)
        del x, ws_p
    n_tones = sum(1 for m in specs_meta if m[2])
    nmax = max(s.shape[0] for s in specs)
    plan = J.Plan(nmax, 100.0, 300.0, 2.0, 20.0, path="fft")
    t0 = time.perf_counter()
    plan.autotune(specs[0], uniform=True)
    t_tune = time.perf_counter() - t0
    bank = plan.new_bank()
    plan.build_templates(bank)
    T = plan.info()["n_templates"]
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    # per-spectrum plane regions: as many rows per slab as fit in 60% of the free memory (<= 64)
    free, _ = torch.cuda.mem_get_info()
    row_bytes_all = sum(2 * s.shape[0] * 4 for s in specs)
    slab_rows = int(max(1, min(64, 0.6 * free // row_bytes_all)))
    planes = [torch.empty((slab_rows, 2 * s.shape[0]), dtype=torch.float32, device="cuda") for s in specs]
    ws = torch.empty(plan.batch_workspace_bytes(n_items), dtype=torch.uint8, device="cuda")
    items = [(s, pl, None) for s, pl in zip(specs, planes)]
    pts = sum(2 * s.shape[0] for s in specs) * T
    out = {"items": n_items, "with_tone": n_tones, "templates": T, "points": pts, "slab_rows": slab_rows,
           "plane_bytes_resident": slab_rows * row_bytes_all}
    for name, flat in (("flat", True), ("persistent", False)):
        # warm-up (captures the graph), then one timed pass over all slabs
        plan.batch_search(bank, items, ws, 0, min(T, slab_rows), graph=True, flat=flat)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t_b in range(0, T, slab_rows):
            plan.batch_search(bank, items, ws, t_b, min(T, t_b + slab_rows), graph=True, flat=flat)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[name] = {"wall_s": wall, "points_per_s": pts / wall}
    out["points_per_s"] = out["flat"]["points_per_s"]
    out["launches"] = -(-T // slab_rows)
    del planes, items
    torch.cuda.empty_cache()
    seg = plan.group(0)["seg_len"]
    # candidates of the first cand_items spectra (k = 6) through jerk_batch_search_candidates: no planes
    cands = None
    if cand_items > 0:
        sub = specs[:cand_items]
        k = 6.0
        cl = []
        for s_ in sub:
            cap = int(1.2e-3 * 2 * s_.shape[0] * T) + 4096
            cl.append((s_, torch.empty((cap, 4), dtype=torch.int32, device="cuda"),
                       torch.zeros(1, dtype=torch.int64, device="cuda"), None))
        cws = plan.batch_search_candidates(bank, cl, k)  # warm-up; allocates the shared workspace
        torch.cuda.synchronize()
        for c in cl:
            c[2].zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.batch_search_candidates(bank, cl, k, ws=cws)
        torch.cuda.synchronize()
        wall_c = time.perf_counter() - t0
        pts_c = sum(2 * s_.shape[0] for s_ in sub) * T
        cands = {"items": len(sub), "k_sigma": k, "points": pts_c, "wall_s": wall_c, "points_per_s": pts_c / wall_c,
                 "candidates": int(sum(int(c[2].item()) for c in cl))}
        del cl, cws
    plan.close()
    out.update({"candidates_no_plane": cands, "seg_len": seg, "autotune_s": t_tune,
                "workload": "synth.batch_spectra_specs(256, seed 191103): lengths 2^20..2^22 bins, 10% with one "
                            "tone; series made on the GPU (synth.time_series_device), spectra by "
                            "jerk_spectrum_prepare; zmax 100, wmax 300"})
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "detail": "sharding by template range, r range or spectrum is described in the "
                                    "design notes; no multi-GPU path is built"}))
        sys.exit(2)
    import numpy as np

    import synth

    # The process-pool CPU leg forks workers, so it runs before anything touches the GPU.
    cfg = synth.CONFIGS["bins2e22_z200_w600"]
    spec_np = synth.make_spectrum(cfg)
    host = cpu_host()
    cpu_pool = None
    if args.cpu_templates > 0:
        cpu_pool = cpu_oracle_pool(spec_np, 2 * host["workers"], host["workers"])

    import torch

    import paper_1911_01353_amd as J

    J.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n = spec_np.shape[0]
    spec = torch.from_numpy(spec_np).cuda()
    print(f"[bench] spectrum {n} bins ready; path {args.path}", file=sys.stderr, flush=True)

    main_res = time_path(J, torch, spec, n, args.path, args.steps, args.warmup, args.slab_gb, True,
                         autotune=bool(args.autotune), load_plan=args.load_plan, save_plan=args.save_plan)
    if args.calib_copy_mib > 0:
        a = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    headline_rows = None
    if args.cpu_templates > 0:
        rowbuf = torch.empty((1, 2 * n), dtype=torch.float32, device="cuda")
        rows = []
        for t in cpu_baseline_templates(args.cpu_templates):
            main_res["plan"].search(main_res["bank"], spec, rowbuf, t, t + 1)
            rows.append(rowbuf.cpu().numpy()[0].copy())
        headline_rows = np.stack(rows)
        del rowbuf
    T = main_res["T"]
    points_per_step = 2 * n * T
    wall = main_res["wall"]
    value = points_per_step * args.steps / wall
    print(f"[bench] {args.path}: {value:.3e} points/s ({wall / args.steps * 1e3:.1f} ms/step)", file=sys.stderr,
          flush=True)

    # dominant kernel roofline: algorithmic bytes (4 B per plane point written + 8 B per spectrum
    # bin read) per launch over the average launch time, against the published HBM peak
    ks = main_res["kernels"]
    dom = max(ks, key=lambda k: ks[k]["time"])
    d = ks[dom]
    avg_t = d["time"] / d["launches"]
    kernel_share = d["time"] / sum(v["time"] for v in ks.values())
    copy = hbm_copy_leg(torch, args.copy_gib) if args.copy_gib > 0 else None
    peaks = peak_probe()
    tflops = d["flops"] / d["launches"] / avg_t / 1e12
    gbps = d["bytes"] / d["launches"] / avg_t / 1e9
    roof = {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBS,
            "traffic": traffic_from_profiles(dom, d["points"] / d["launches"]),
            "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": dom, "kernel_time_share": kernel_share, "avg_launch_ms": avg_t * 1e3,
            "launches": d["launches"], "bytes_per_launch": d["bytes"] / d["launches"],
            "points_per_launch": d["points"] / d["launches"]}
    if copy:
        roof["frac_of_measured_copy"] = gbps / copy["copy_GBps"]
        roof["frac_of_measured_fill"] = gbps / copy["fill_GBps"]
    if d["path"] == 0:
        roof["vector_fp32"] = {
            "achieved_tflops": tflops, "flops_counted": "nominal FFT count 5 S log2 S per transform, 6 S per "
                                                        "spectrum product, 3 per kept lag",
            "peak_tflops": FP32_VECTOR_PUBLISHED_TFLOPS, "frac": tflops / FP32_VECTOR_PUBLISHED_TFLOPS}
        if peaks:
            roof["vector_fp32"]["measured_fma_tflops"] = peaks["fp32_fma"]["TFLOPs"]
            roof["vector_fp32"]["frac_of_measured_fma"] = tflops / peaks["fp32_fma"]["TFLOPs"]
    else:
        roof["mfma"] = {"achieved_tflops": tflops,
                        "peak_tflops": MFMA_BF16_TFLOPS if d["path"] == 1 else MFMA_FP16_TFLOPS,
                        "frac": tflops / (MFMA_BF16_TFLOPS if d["path"] == 1 else MFMA_FP16_TFLOPS)}
        if peaks:
            roof["mfma"]["measured_tflops"] = peaks["mfma_bf16"]["TFLOPs"]
    kernels_out = kernel_table(ks)

    paths = {args.path: value}
    kernels_by_path = {}
    if args.compare_paths:
        for p in ("fft", "split_bf16"):
            if p == args.path:
                continue
            r = time_path(J, torch, spec, n, p, max(1, args.steps // 2), 1, args.slab_gb, True,
                          autotune=bool(args.autotune))
            paths[p] = points_per_step * max(1, args.steps // 2) / r["wall"]
            kernels_by_path[p] = kernel_table(r["kernels"])
            print(f"[bench] {p}: {paths[p]:.3e} points/s", file=sys.stderr, flush=True)
            r["plan"].close()

    rocfft = None
    if args.rocfft_groups > 0:
        rocfft = rocfft_leg(J, torch, main_res["plan"], main_res["bank"], spec, n, args.rocfft_groups,
                            args.rocfft_members)
    cands = None
    if args.cand_rows > 0:
        cands = candidates_leg(J, torch, main_res["plan"], main_res["bank"], spec, n,
                               min(args.cand_rows, T), args.cand_sigma)
        print(f"[bench] candidate selection {cands['points_per_s']:.3e} points/s "
              f"(stats {cands['stats_GBps']:.0f} GB/s, peaks {cands['candidates_GBps']:.0f} GB/s)",
              file=sys.stderr, flush=True)
    fused = None
    if args.fused_reps > 0:
        fused = search_candidates_leg(J, torch, spec, n, args.cand_sigma, args.fused_reps)
        two_step = None
        if cands and "fft" in paths:
            two_step = 1.0 / (1.0 / paths["fft"] + 1.0 / cands["points_per_s"])
            fused["two_step_fft_points_per_s"] = two_step
            fused["speedup_vs_two_step"] = fused["points_per_s"] / two_step
        print(f"[bench] search with fused candidate selection {fused['points_per_s']:.3e} points/s "
              f"({fused['ms']:.1f} ms, {fused['candidates']} candidates)"
              + (f", two-step {two_step:.3e}" if two_step else ""), file=sys.stderr, flush=True)
    harm = harmonics_leg(J, torch, spec, n) if args.harm_templates else None
    prep = spectrum_leg(J, torch, 2 * n) if args.prep else None
    small = small_search_leg(J, torch, args.small_reps) if args.small_reps > 0 else None
    if small:
        print("[bench] 2^15-bin search per graph rep: " + ", ".join(
            f"{p} {small[p]['us_per_search']:.1f} us" for p in ("fft", "split_bf16", "fp16", "auto")), file=sys.stderr,
            flush=True)
    if prep:
        print(f"[bench] spectrum preparation {prep['ms']:.3f} ms for {prep['n_samples']} samples",
              file=sys.stderr, flush=True)
    if harm:
        print(f"[bench] harmonic sums: " + ", ".join(f"H={h[1:]} {v['GBps']:.0f} GB/s" for h, v in harm.items()
                                                       if h.startswith("H")), file=sys.stderr, flush=True)
    errors = plane_errors(J, torch) if args.errors else None
    serving = None
    if args.serve_requests > 0:
        serving = serving_leg(J, torch, args.serve_requests, [float(x) for x in args.serve_load.split(",")],
                              n_cold=args.serve_cold_requests)
        print("[bench] serving warm " + ", ".join(
            f"load {k}: p50 {v['p50_s']:.3f} s p99 {v['p99_s']:.3f} s" for k, v in serving["warm_poisson"].items()),
            file=sys.stderr, flush=True)
    batch = None
    if args.batch_items > 0:
        batch = batch_leg(J, torch, args.batch_items)
        print(f"[bench] batch {batch['flat']['points_per_s']:.3e} points/s (flat launch), "
              f"{batch['persistent']['points_per_s']:.3e} (persistent), {batch['slab_rows']} rows per slab"
              + (f", with candidates {batch['candidates_no_plane']['points_per_s']:.3e} "
                 f"({batch['candidates_no_plane']['items']} spectra)" if batch['candidates_no_plane'] else ""),
              file=sys.stderr, flush=True)
    cpu = None
    err_headline = None
    if args.cpu_templates > 0:
        cpu, ts_ora, rows_ora = cpu_baseline(spec_np, args.cpu_templates)
        err_headline = headline_error(headline_rows, ts_ora, rows_ora)
        print(f"[bench] headline plan against the oracle on {len(ts_ora)} whole rows: max {err_headline['max']:.2e}, "
              f"rms {err_headline['rms']:.2e}, row peaks equal {err_headline['row_peaks_match']}",
              file=sys.stderr, flush=True)
        del rows_ora
    cpu_fft = None
    if args.cpu_templates > 0:
        cpu_fft = cpu_fft_overlap_save(spec_np, 16, host["workers"])
        print(f"[bench] CPU: oracle {cpu['value']:.2e}, oracle pool {cpu_pool['value']:.2e}, "
              f"FFT overlap-save {cpu_fft['value']:.2e} points/s", file=sys.stderr, flush=True)

    latency = None
    if serving:
        top = max(serving["warm_poisson"], key=float)  # the highest offered load
        v = serving["warm_poisson"][top]
        latency = {"load": float(top), "p50_s": v["p50_s"], "p99_s": v["p99_s"], "p99.9_s": v["p99.9_s"],
                   "requests": v["requests"], "source": "serving leg, warm template cache, Poisson arrivals",
                   "by_path": {k: v[k] for k in ("fft", "split_bf16") if k in v}}
    line = {
        "metric": "(r,z,w) plane points/s, FP32 vs split-BF16 @<=1e-4 rel err; p50/p99 latency",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"auto": "f32+bf16x3", "fft": "f32", "split_bf16": "bf16x3", "fp16": "f16"}[args.path],
        "data": "synthetic",
        "config": {"workload": "single search, 2^22 bins (2^23 float32 samples, 4 seeded tones), "
                               "zmax 200, wmax 600, dz 2, dw 20 (201x61=12261 templates), half-bin r, "
                               f"path {args.path}, plane written as slabs of up to {main_res['rows']} rows "
                               "of one width group",
                   "nbins": n, "templates": T, "points_per_step": points_per_step},
        "roofline": roof,
        "cpu_baseline": cpu,
        "cpu_host": host,
        "cpu_oracle_all_cores": cpu_pool,
        "cpu_fft_overlap_save": cpu_fft,
        "paths_points_per_s": paths,
        "vs_unfused_rocfft": rocfft,
        "candidate_selection": cands,
        "search_with_candidates": fused,
        "harmonic_sums": harm,
        "spectrum_preparation": prep,
        "search_2e15_bins_graph": small,
        "plane_error_2e15_bins": errors,
        "error_vs_oracle": err_headline,
        "template_build_s": main_res["t_build"],
        "autotune_s": main_res["t_tune"],
        "kernels": kernels_out,
        "kernels_other_paths": kernels_by_path,
        "hbm_measured": copy,
        "arithmetic_measured": peaks,
        "serving": serving,
        "latency": latency,
        "batched_256_spectra": batch,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
