"""Direct correlation of a spectrum with the template bank: the (r, z, w) power plane.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition (paper, section "Implementation": each matched filter fits the
response for one (z, w); Figure 1: the filtering is a convolution that
overlap-and-save evaluates segment by segment). For template ``t`` with
half-width ``h`` and output ``p = 2 k0 + phase`` (two outputs per bin, at
``r = p / 2``):

    Y[t][p] = sum_{k = k0-h+1}^{k0+h} X[k] * conj(T(k0 + phase/2 - k; zbar_t, w_t))
    P[t][p] = |Y[t][p]|^2

with ``X[k] = 0`` outside ``[0, n)``. Raw power, no per-template scaling. This
is the plain direct sum; overlap-and-save reaches the same numbers in exact
arithmetic, so the direct sum is the oracle for both GPU paths.
"""

from __future__ import annotations

import numpy as np

from .grid import Grid
from .response import template_taps


def correlate_row(spectrum: np.ndarray, taps: np.ndarray, half_width: int,
                  k_lo: int, k_hi: int) -> np.ndarray:
    """Complex outputs ``Y[k0]`` for ``k0`` in ``[k_lo, k_hi)`` of one template/phase.

    ``taps[j]`` (already conjugated) multiplies bin ``k0 - half_width + 1 + j``.
    """
    x = np.asarray(spectrum, dtype=np.complex128)
    n = x.shape[0]
    ntap = taps.shape[0]
    if ntap != 2 * half_width:
        raise ValueError("taps must have 2*half_width entries")
    first = k_lo - half_width + 1          # first bin touched
    last = (k_hi - 1) + half_width         # last bin touched (inclusive)
    window = np.zeros(last - first + 1, dtype=np.complex128)
    a, b = max(first, 0), min(last + 1, n)
    if a < b:
        window[a - first:b - first] = x[a:b]
    # np.correlate(a, v)[m] = sum_j a[m + j] * conj(v[j]): a direct (non-FFT) sum.
    return np.correlate(window, np.conj(taps), mode="valid")


def oracle_plane(spectrum: np.ndarray, grid: Grid, templates=None, p_lo: int = 0,
                 p_hi: int | None = None) -> np.ndarray:
    """FP64 power plane ``P[t][p]`` for the given templates and ``p`` in ``[p_lo, p_hi)``.

    ``templates``: iterable of template indices (default: all, in order).
    ``p`` indexes the half-bin r grid, ``r = p / 2``; default range ``[0, 2n)``.
    Returns a float64 array of shape ``(len(templates), p_hi - p_lo)``.
    """
    n = int(np.asarray(spectrum).shape[0])
    if p_hi is None:
        p_hi = 2 * n
    if templates is None:
        templates = range(grid.n_templates)
    templates = list(templates)
    if not (0 <= p_lo <= p_hi <= 2 * n):
        raise ValueError("p range outside [0, 2n)")
    out = np.zeros((len(templates), p_hi - p_lo), dtype=np.float64)
    if p_hi == p_lo:
        return out
    k_lo = p_lo // 2
    k_hi = (p_hi + 1) // 2
    for row, t in enumerate(templates):
        zbar, w, h = grid.params(t)
        for phase in (0, 1):
            y = correlate_row(spectrum, template_taps(zbar, w, h, phase), h, k_lo, k_hi)
            pw = y.real * y.real + y.imag * y.imag
            p = 2 * np.arange(k_lo, k_hi) + phase
            keep = (p >= p_lo) & (p < p_hi)
            out[row, p[keep] - p_lo] = pw[keep]
    return out
