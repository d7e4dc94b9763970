"""Fourier response of a tone with constant fdot (z) and fddot (w), in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definitions (paper, section "Implementation": ``z = fdot T^2``, ``w = fddot T^3``)
------------------------------------------------------------------------------

Let ``u = t / T`` run over the unit observation ``[0, 1)``. A unit tone whose
frequency, fdot and fddot at the start of the observation are
``r0 / T``, ``z0 / T^2`` and ``w0 / T^3`` has phase (in cycles)

    phi(u) = r0 u + z0 u^2 / 2 + w0 u^3 / 6.

Bin ``k`` of its Fourier transform (normalised by the number of samples) is,
in the continuum limit,

    R(r0 - k; z0, w0),    R(q; z, w) = integral_0^1 exp(2 pi i (q u + z u^2/2 + w u^3/6)) du.

Templates are labelled by the observation-average frequency and fdot:
``rbar = r0 + z0/2 + w0/6`` and ``zbar = z0 + w0/2`` (``w`` is constant).
Substituting gives the template as a function of the offset
``qbar = rbar - k`` of bin ``k`` from the trial frequency:

    T(qbar; zbar, w) = R(qbar - zbar/2 + w/12; zbar - w/2, w).

Quadrature
----------

``R`` is evaluated by composite 32-point Gauss-Legendre quadrature on
``[0, 1]`` split into ``P`` equal panels, with
``P = 2 * ceil(|q| + |z| + |w|/2 + 1) + 2``: the integrand's phase turns at
most ``|q| + |z| + |w|/2`` cycles over the interval, so every panel spans at
most half a cycle and 32 nodes integrate it to FP64 rounding. Each tap is
integrated on its own (its panel count depends only on its own arguments).
"""

from __future__ import annotations

import math

import numpy as np

_GL_NODES = 32
_GL_X, _GL_W = np.polynomial.legendre.leggauss(_GL_NODES)  # on [-1, 1]


def _panel_count(q: float, z: float, w: float) -> int:
    """Panels for one evaluation of R: two per cycle of the phase plus two."""
    return 2 * int(math.ceil(abs(q) + abs(z) + abs(w) / 2.0 + 1.0)) + 2


def _response_one(q: float, z: float, w: float) -> complex:
    """R(q; z, w) for scalar arguments by composite Gauss-Legendre quadrature."""
    p = _panel_count(q, z, w)
    h = 1.0 / p
    left = np.arange(p, dtype=np.float64)[:, None] * h
    u = left + (0.5 * h) * (_GL_X[None, :] + 1.0)  # (p, 32) nodes in [0, 1]
    phase = q * u + z * u * u / 2.0 + w * u * u * u / 6.0  # cycles
    phase = phase - np.rint(phase)  # exp(2 pi i phase) only needs phase mod 1
    vals = np.exp(2j * np.pi * phase)
    return complex((0.5 * h) * np.sum(vals * _GL_W[None, :]))


def response(q, z: float, w: float) -> np.ndarray:
    """R(q; z, w) for an array of ``q`` (complex128, same shape as ``q``).

    Start-of-observation convention: the response at offset ``q = r0 - k`` of
    a tone with start values ``(r0, z0=z, w0=w)``.
    """
    q = np.asarray(q, dtype=np.float64)
    out = np.empty(q.shape, dtype=np.complex128)
    flat_q = q.reshape(-1)
    flat_o = out.reshape(-1)
    for i, qi in enumerate(flat_q):
        flat_o[i] = _response_one(float(qi), float(z), float(w))
    return out


def template_response(qbar, zbar: float, w: float) -> np.ndarray:
    """T(qbar; zbar, w) = R(qbar - zbar/2 + w/12; zbar - w/2, w).

    Average-value convention: ``qbar = rbar - k`` with ``rbar`` and ``zbar``
    the observation averages of the frequency and fdot.
    """
    qbar = np.asarray(qbar, dtype=np.float64)
    return response(qbar - zbar / 2.0 + w / 12.0, zbar - w / 2.0, w)


def template_taps(zbar: float, w: float, half_width: int, phase: int) -> np.ndarray:
    """Correlation taps of one template for output phase ``phase`` (0 or 1).

    The output at ``r = k0 + phase/2`` sums ``X[k] * conj(T(r - k))`` over the
    ``2*half_width`` bins ``k = k0 - half_width + 1 ... k0 + half_width``.
    Tap ``j`` multiplies bin ``k = k0 - half_width + 1 + j``, so its offset is
    ``qbar_j = half_width - 1 - j + phase/2``. Returned taps are already
    conjugated: ``c_j = conj(T(qbar_j; zbar, w))``.
    """
    if phase not in (0, 1):
        raise ValueError("phase must be 0 or 1 (two outputs per bin)")
    j = np.arange(2 * half_width, dtype=np.float64)
    qbar = (half_width - 1) - j + phase / 2.0
    return np.conj(template_response(qbar, zbar, w))
