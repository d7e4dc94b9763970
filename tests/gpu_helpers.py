"""Helpers for the GPU tests: run the library on numpy inputs and read results back."""

from __future__ import annotations

import numpy as np

import paper_1911_01353_amd as J


def device():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a visible GPU")
    J.load()  # fail loudly if the HIP library is missing
    return torch.device("cuda:0")


def build_bank(plan, stream=None):
    import torch
    bank = plan.new_bank()
    plan.build_templates(bank, stream)
    torch.cuda.synchronize()
    return bank


def gpu_plane(plan, bank, spec_np, t_begin=0, t_end=None, ld=None, poison=True):
    """Run jerk_search on a host spectrum; returns the float32 plane rows [t_begin, t_end)."""
    import torch
    dev = device()
    n = spec_np.shape[0]
    if t_end is None:
        t_end = plan.info()["n_templates"]
    ld = ld or 2 * n
    spec = torch.from_numpy(np.ascontiguousarray(spec_np)).to(dev)
    plane = torch.full((t_end - t_begin, ld), float("nan") if poison else 0.0, dtype=torch.float32, device=dev)
    plan.search(bank, spec, plane, t_begin, t_end)
    torch.cuda.synchronize()
    return plane.cpu().numpy()[:, : 2 * n]


def bank_taps(plan, bank, g):
    """FP64 taps of width group g from the bank: complex128 [n_members][2][taps]."""
    info = plan.group(g)
    nbytes = info["n_members"] * 2 * info["taps"] * 16
    raw = bank[info["taps_offset"]: info["taps_offset"] + nbytes].cpu().numpy()
    return raw.view(np.complex128).reshape(info["n_members"], 2, info["taps"])
