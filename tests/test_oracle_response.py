"""Pins of the oracle's response and template functions.

Each check compares the oracle's Gauss-Legendre quadrature with something it
does not use: a closed form (sinc, Fresnel), 30-digit mpmath quadrature on a
different rule, the DFT of a sampled tone, Parseval's identity, or symmetry.
"""

import math

import mpmath
import numpy as np
import pytest
from scipy.special import fresnel

from oracle.grid import half_width
from oracle.response import response, template_response, template_taps


def test_zero_fdot_fddot_is_fourier_interpolation():
    # R(q; 0, 0) = integral_0^1 e^{2 pi i q u} du = e^{i pi q} sin(pi q) / (pi q).
    rng = np.random.default_rng(1)
    q = np.concatenate([rng.uniform(-60, 60, 40), np.arange(-5, 6), np.arange(-5, 6) + 0.5])
    got = response(q, 0.0, 0.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        want = np.exp(1j * np.pi * q) * np.where(q == 0, 1.0, np.sin(np.pi * q) / (np.pi * q))
    want[q == 0] = 1.0
    assert np.max(np.abs(got - want)) < 1e-14


def _fresnel_response(q, z):
    """R(q; z, 0) from the Fresnel integrals (z != 0)."""
    if z < 0:
        return np.conj(_fresnel_response(-q, -z))
    s = math.sqrt(2.0 / z)
    t1, t2 = q * s, (q + z) * s
    s1, c1 = fresnel(t1)
    s2, c2 = fresnel(t2)
    return np.exp(-1j * np.pi * q * q / z) / math.sqrt(2.0 * z) * ((c2 - c1) + 1j * (s2 - s1))


@pytest.mark.parametrize("z", [0.5, 3.0, 17.3, 150.0, -40.0, -299.0])
def test_constant_fdot_matches_fresnel(z):
    rng = np.random.default_rng(int(abs(z) * 10))
    q = rng.uniform(-abs(z) - 30, 30, 25)
    got = response(q, z, 0.0)
    want = _fresnel_response(q, z)
    assert np.max(np.abs(got - want)) < 1e-12


def _mp_response(q, z, w):
    mpmath.mp.dps = 30
    q, z, w = mpmath.mpf(q), mpmath.mpf(z), mpmath.mpf(w)
    f = lambda u: mpmath.expjpi(2 * (q * u + z * u * u / 2 + w * u ** 3 / 6))  # noqa: E731
    m = int(math.ceil(abs(q) + abs(z) + abs(w) / 2 + 1)) + 1
    return complex(mpmath.quad(f, [mpmath.mpf(i) / m for i in range(m + 1)]))


@pytest.mark.parametrize("q,z,w", [
    (0.3, 1.2, -2.5),
    (12.7, -35.0, 80.0),
    (-3.5, 20.0, 60.0),
    (40.25, -7.0, -120.0),
    (-150.25, 300.0, -900.0),
])
def test_general_response_matches_mpmath(q, z, w):
    got = response([q], z, w)[0]
    assert abs(got - _mp_response(q, z, w)) < 1e-13


def test_average_value_convention_against_sampled_tone():
    """DFT of a sampled complex tone equals T(rbar - k; zbar, w) (Euler-Maclaurin corrected).

    The tone has start values (r0, z0, w0); its observation-average frequency
    and fdot are rbar = r0 + z0/2 + w0/6 and zbar = z0 + w0/2. The DFT is a
    left Riemann sum of R's integral; adding the end-point (trapezoid) and
    first Euler-Maclaurin terms leaves an O(N^-4) error.
    """
    n = 2 ** 14
    r0, z0, w0 = 3000.37, -23.4, 71.3
    u = np.arange(n) / n
    cyc = r0 * u + z0 * u * u / 2 + w0 * u ** 3 / 6
    x = np.exp(2j * np.pi * (cyc - np.floor(cyc)))
    dft = np.fft.fft(x) / n
    rbar, zbar = r0 + z0 / 2 + w0 / 6, z0 + w0 / 2
    ks = np.arange(int(rbar) - 40, int(rbar) + 41)
    q = r0 - ks
    g1 = np.exp(2j * np.pi * (r0 + z0 / 2 + w0 / 6 - ks))     # g(1); g(0) = 1
    dg0 = 2j * np.pi * q                                        # g'(0)
    dg1 = 2j * np.pi * (q + z0 + w0 / 2) * g1                   # g'(1)
    em = dft[ks] + (g1 - 1.0) / (2 * n) - (dg1 - dg0) / (12.0 * n * n)
    want = template_response(rbar - ks, zbar, w0)
    assert np.max(np.abs(em - want)) < 1e-10
    # Without the average-value shift the match fails badly (guards the convention).
    wrong = template_response(r0 - ks, z0, w0)
    assert np.max(np.abs(em - wrong)) > 1e-2


def test_template_symmetry():
    rng = np.random.default_rng(5)
    for _ in range(5):
        zb, w = rng.uniform(-100, 100), rng.uniform(-300, 300)
        qb = rng.uniform(-50, 50, 7)
        a = template_response(qb, zb, w)
        b = np.conj(template_response(-qb, -zb, w * -1.0))
        assert np.max(np.abs(a - b)) < 1e-13


@pytest.mark.parametrize("zb,w", [(0.0, 0.0), (16.0, 20.0), (-20.0, 60.0), (100.0, -300.0)])
def test_parseval_and_captured_energy(zb, w):
    """sum_k |T(qbar - k)|^2 = 1 over all integers k (Fourier coefficients of a unit-modulus function)."""
    qb0 = 0.37
    L = 700
    k = np.arange(-L, L + 1)
    tot = np.sum(np.abs(template_response(qb0 - k, zb, w)) ** 2)
    h = half_width(zb, w)
    fmax = h - 16
    # Tail beyond L is bounded by sum_{|q| > L - fmax} 1 / (pi q)^2 <= 2 / (pi^2 (L - fmax - 1)).
    assert 0.0 <= 1.0 - tot <= 2.0 / (np.pi ** 2 * (L - fmax - 1)) + 1e-12
    # The 2h taps of the correlation capture at least 98.5% of the energy (the
    # worst case is the half-bin sinc at zbar = w = 0, whose tail beyond 16 bins
    # holds about 2 / (16 pi^2) = 1.3%).
    for phase in (0, 1):
        cap = np.sum(np.abs(template_taps(zb, w, h, phase)) ** 2)
        assert 0.985 <= cap <= 1.0 + 1e-12


def test_taps_layout():
    # Tap j multiplies bin k0 - h + 1 + j; at zbar = w = 0 and integer r the only
    # non-zero tap is the one on bin k0, i.e. j = h - 1.
    h = half_width(0.0, 0.0)
    c0 = template_taps(0.0, 0.0, h, 0)
    assert c0.shape == (2 * h,)
    assert abs(c0[h - 1] - 1.0) < 1e-14
    assert np.max(np.abs(np.delete(c0, h - 1))) < 1e-14
    # Half-bin phase: tap j sits at offset qbar = h - 1 - j + 1/2.
    c1 = template_taps(0.0, 0.0, h, 1)
    qb = (h - 1) - np.arange(2 * h) + 0.5
    want = np.conj(np.exp(1j * np.pi * qb) * np.sin(np.pi * qb) / (np.pi * qb))
    assert np.max(np.abs(c1 - want)) < 1e-14
