"""The library from a plain C program (tests/c_abi/jerk_demo.c, built with the library): its own
device buffers and stream, no Python in the process. Its plane is checked against the FP64
oracle (1e-4 floored relative power error, peak equal) and its fused candidate search against
the same call made through the Python binding on the same spectrum (equal records)."""

import os
import subprocess

import numpy as np
import pytest

import paper_1911_01353_amd as J
import synth
from oracle import Grid, error_summary, oracle_plane, peak_index

from gpu_helpers import build_bank, device

pytestmark = pytest.mark.gpu

DEMO = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "jerk_demo")


def test_plain_c_caller(tmp_path):
    import torch
    assert os.path.exists(DEMO), "tests/c_abi/jerk_demo is missing: build the library first"
    x = synth.time_series(8192, 191107, (synth.Tone(0.15, 1500.3, 5.0, 30.0, 0.0),))
    spec = synth.spectrum_from_series(x)
    n = spec.shape[0]
    paths = {k: str(tmp_path / f"{k}.bin") for k in ("spec", "plane", "cands")}
    spec.tofile(paths["spec"])
    r = subprocess.run([DEMO, paths["spec"], str(n), "20", "60", paths["plane"], paths["cands"]],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    grid = Grid(20.0, 60.0, 2.0, 20.0)
    T = grid.n_templates
    plane = np.fromfile(paths["plane"], dtype=np.float32).reshape(T, 2 * n)
    ora = oracle_plane(spec, grid)
    assert error_summary(plane, ora)["max"] <= 1e-4
    assert peak_index(plane) == peak_index(ora)
    raw = open(paths["cands"], "rb").read()
    count = int(np.frombuffer(raw[:8], dtype=np.int64)[0])
    got = np.sort(np.frombuffer(raw[8:], dtype=J.CANDIDATE_DTYPE, count=count), order=["t", "p"])
    assert count > 100
    dev = device()
    plan = J.Plan(n, 20.0, 60.0, 2.0, 20.0, path="fft")
    bank = build_bank(plan)
    out = torch.zeros((T * n, 4), dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    plan.search_candidates(bank, torch.from_numpy(spec).to(dev), 3.0, 0.9 * 4.0, out, cnt)
    torch.cuda.synchronize()
    want = J.candidates_numpy(out, cnt)
    assert np.array_equal(got, want)
    plan.close()
