"""Spectrum preparation: real time series -> normalised complex spectrum.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's search works on the Fourier transform of a time series (section
"Introduction": periodicity searches Fourier-transform the series; the matched
filters then act on its spectrum). It does not say how the spectrum is scaled.
Reading used here (the same one the synthetic inputs follow):

1. the DFT ``X[k] = sum_j x[j] exp(-2 pi i j k / N)`` of the ``N`` samples, in
   FP64 (``N`` even, ``N >= 4``);
2. keep bins ``0 .. N/2 - 1`` (the Nyquist bin ``N/2`` is dropped);
3. set the DC bin ``X[0]`` to zero;
4. divide by ``sqrt(mean_{1 <= k < N/2} |X[k]|^2)`` so that the mean power of
   the kept bins above DC is 1; a spectrum that is zero above DC stays zero;
5. round once to complex64.
"""

from __future__ import annotations

import numpy as np


def prepare_spectrum(series: np.ndarray) -> np.ndarray:
    """complex64 spectrum of ``N/2`` bins from ``N`` real samples (steps 1-5)."""
    x = np.asarray(series, dtype=np.float64)
    n = x.shape[0]
    if x.ndim != 1 or n < 4 or n % 2:
        raise ValueError("series must be 1-D with an even length >= 4")
    spec = np.fft.fft(x)[: n // 2]
    spec[0] = 0.0
    mean_power = float(np.mean(np.abs(spec[1:]) ** 2))
    if mean_power > 0.0:
        spec = spec / np.sqrt(mean_power)
    return spec.astype(np.complex64)
