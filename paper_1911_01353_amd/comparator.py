"""Unfused library-FFT overlap-save: the comparator for the fused search kernels.

The paper (section "Implementation") compares its shared-memory overlap-and-save
convolution with a convolution built from vendor FFT library calls, and reports
its own as up to three times faster at jerk-search filter lengths. This module
is that library-built variant on MI355X: every step is a separate torch call
(rocFFT underneath), each a round trip through HBM:

1. cut the zero-extended spectrum into overlapping segments of S bins (stride
   U = S - K + 1) and run one batched forward FFT over all of them;
2. multiply by each template's spectrum (both half-bin phases);
3. one batched inverse FFT per template;
4. power, drop the K - 1 wrapped lags of every segment, interleave the phases.

It is NOT the library's search path (that is ``Plan.search``, which runs the
HIP kernels); it exists to be timed beside it and to cross-check it.
"""

from __future__ import annotations


def template_spectra(taps, seg_len: int):
    """Spectra of zero-padded templates for the correlation form of overlap-save.

    ``taps``: complex128 tensor [m, 2, K] (tap j multiplies bin k0 - K/2 + 1 + j
    of output k0, already conjugated). Returns complex64 [m, 2, seg_len] with
    H[f] = sum_j c_j exp(+2 pi i f j / S), so that IFFT(FFT(segment) * H) at lag
    l is sum_j segment[l + j] c_j.
    """
    import torch
    m, _, K = taps.shape
    if seg_len < K:
        raise ValueError("segment shorter than the template")
    c = torch.zeros((m, 2, seg_len), dtype=torch.complex128, device=taps.device)
    c[..., :K] = taps
    return torch.fft.ifft(c, norm="forward").to(torch.complex64)


def overlap_save(spec, spectra, taps: int, out) -> None:
    """Rows of ``out`` (float32 [m, >= 2n], both phases interleaved along r) from the
    template spectra [m, 2, S] of K-tap templates, by unfused library calls."""
    import torch
    n = spec.shape[0]
    m, _, S = spectra.shape
    K = taps
    U = S - K + 1
    if U < 1:
        raise ValueError("segment shorter than the template")
    n_seg = -(-n // U)
    xp = torch.zeros(K // 2 - 1 + n_seg * U + S, dtype=torch.complex64, device=spec.device)
    xp[K // 2 - 1: K // 2 - 1 + n] = spec
    segs = xp.unfold(0, S, U)[:n_seg]
    f = torch.fft.fft(segs)
    for i in range(m):
        y = torch.fft.ifft(f[None] * spectra[i][:, None, :])[..., :U]
        pw = (y.real * y.real + y.imag * y.imag).reshape(2, n_seg * U)[:, :n]
        out[i, : 2 * n].view(n, 2).copy_(pw.t())
