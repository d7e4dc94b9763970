"""CPU tests of the measurement helpers (bench contract, counter summariser)."""

import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_bench_launch_counts():
    sys.path.insert(0, ROOT)
    import bench
    g = {"path": 0, "seg_len": 512, "taps": 160, "templates_per_block": 16, "fft_ept": 8}
    pts, flops, by = bench.launch_counts(g, 32, 1 << 20)
    assert pts == 32 * 2 * (1 << 20)
    assert by == 4 * pts + 8 * (1 << 20)
    n_seg = -(-(1 << 20) // 353)
    assert abs(flops - n_seg * (2 * 5 * 512 * 9 + 32 * 2 * (6 * 512 + 5 * 512 * 9 + 3 * 353))) < 1
    gm = {"path": 1, "seg_len": 1024, "taps": 64, "templates_per_block": 16, "fft_ept": 16}
    assert bench.launch_counts(gm, 8, 1000)[1] == 8 * 2000 * 8 * 64 * 3


def _write_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, name, v in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_summary_scales_by_the_copy(tmp_path):
    k = "void jerk::fft_correlate_kernel<512, 8, 8, 8, 8, 1, false>(jerk::FftJob)"
    # copy of 256 MiB reads as 128 MiB fetched (scale 2) and 256 MiB written (scale 1)
    _write_csv(tmp_path / "f.csv", "FETCH_SIZE", [(1, "__amd_rocclr_copyBuffer", 131072.0), (2, k, 1000.0),
                                                  (3, k, 1000.0), (4, "gen_taps_kernel", 5.0)])
    _write_csv(tmp_path / "w.csv", "WRITE_SIZE", [(1, "__amd_rocclr_copyBuffer", 262144.0), (2, k, 4000.0),
                                                  (3, k, 4000.0), (4, "gen_taps_kernel", 5.0)])
    out = tmp_path / "hbm.json"
    r = subprocess.run([sys.executable, "-m", "paper_1911_01353_amd.traffic", "--fetch", str(tmp_path / "f.csv"),
                        "--write", str(tmp_path / "w.csv"), "--kernel-regex", r"fft_correlate_kernel<512,",
                        "--bench-name", "fft_correlate_kernel<S=512,E=8>", "--points", "4096000",
                        "--copy-mib", "256", "--out", str(out)], capture_output=True, text=True, cwd=ROOT,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    ent = json.load(open(out))["fft_correlate_kernel<S=512,E=8>"]
    assert abs(ent["fetch_scale"] - 2.0) < 1e-12 and abs(ent["write_scale"] - 1.0) < 1e-12
    assert abs(ent["fetch_bytes_per_point"] - 2000 * 1024 * 2 / 4096000) < 1e-9
    assert abs(ent["write_bytes_per_point"] - 8000 * 1024 / 4096000) < 1e-9
    assert ent["dispatches"] == 2


def test_rocfft_comparator_matches_oracle():
    """The unfused library overlap-save used as the bench's comparator computes the oracle's plane."""
    import numpy as np
    import torch
    from paper_1911_01353_amd.comparator import overlap_save, template_spectra
    from oracle.grid import Grid
    from oracle.plane import oracle_plane
    from oracle.response import template_taps
    rng = np.random.default_rng(5)
    n = 3001
    x = ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2)).astype(np.complex64)
    g = Grid(20.0, 60.0, 2.0, 20.0)
    ts = [3, 77, 146]
    K = max(2 * g.params(t)[2] for t in ts)
    taps = np.zeros((len(ts), 2, K), dtype=np.complex128)
    for i, t in enumerate(ts):
        zb, w, h = g.params(t)
        for ph in (0, 1):
            # a narrower template sits centred in the group's K-tap window
            off = K // 2 - h
            taps[i, ph, off: off + 2 * h] = template_taps(zb, w, h, ph)
    want = oracle_plane(x, g, templates=ts)
    for S in (256, 512):
        spectra = template_spectra(torch.from_numpy(taps), S)
        out = torch.empty((len(ts), 2 * n), dtype=torch.float32)
        overlap_save(torch.from_numpy(x), spectra, K, out)
        err = np.abs(out.numpy() - want) / np.maximum(want, want.mean(axis=1, keepdims=True))
        assert err.max() < 1e-4
