"""GPU parity of the unfused library-FFT (rocFFT via torch.fft) overlap-save comparator.

The comparator is the analogue of the paper's vendor-FFT convolution (section
"Implementation"), timed beside the fused kernels; its speed ratios only mean
something if it computes the same plane. Here it is checked against the FP64
oracle on the whole 2^15-bin plane (all three width groups, two segment
lengths each), to the FP32 bar of 1e-4 floored relative power error, and its
peak against the oracle's.
"""

import numpy as np
import pytest

import paper_1911_01353_amd as J
import synth
from oracle import Grid, error_summary, oracle_plane, peak_index

from gpu_helpers import build_bank, device

pytestmark = pytest.mark.gpu


def test_rocfft_overlap_save_matches_oracle():
    import torch
    from paper_1911_01353_amd.comparator import overlap_save, template_spectra
    dev = device()
    cfg = synth.CONFIGS["bins2e15_z20_w60"]
    spec_np = synth.make_spectrum(cfg)
    n = spec_np.shape[0]
    grid = Grid(cfg.zmax, cfg.wmax, cfg.dz, cfg.dw)
    ora = oracle_plane(spec_np, grid)
    plan = J.Plan(n, cfg.zmax, cfg.wmax, cfg.dz, cfg.dw, path="fft")
    bank = build_bank(plan)
    spec = torch.from_numpy(spec_np).to(dev)
    members = plan.members()
    for seg_len in (1024, 2048):
        plane = np.full((grid.n_templates, 2 * n), np.nan, dtype=np.float32)
        for g, gi in enumerate(plan.groups()):
            K, m = gi["taps"], gi["n_members"]
            taps = bank[gi["taps_offset"]: gi["taps_offset"] + m * 2 * K * 16].view(torch.complex128).view(m, 2, K)
            out = torch.full((m, 2 * n), float("nan"), dtype=torch.float32, device=dev)
            overlap_save(spec, template_spectra(taps, seg_len), K, out)
            torch.cuda.synchronize()
            plane[members[gi["first_member"]: gi["first_member"] + m]] = out.cpu().numpy()
        assert not np.isnan(plane).any(), seg_len
        s = error_summary(plane, ora)
        print(f"rocFFT overlap-save, S = {seg_len}: max {s['max']:.3e} rms {s['rms']:.3e}")
        assert s["max"] <= 1e-4, (seg_len, s)
        assert peak_index(plane) == peak_index(ora) == (102, 16013)
    plan.close()
