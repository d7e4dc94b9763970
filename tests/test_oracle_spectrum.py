"""Pins of the oracle's spectrum preparation.

Brute-force DFT sums on tiny series, the closed form of a cosine at an integer
bin, Parseval's identity for the kept half spectrum, DC removal, the unit mean
power invariant, and agreement with the synthetic-input recipe.
"""

import math

import numpy as np
import pytest

import synth
from oracle.spectrum import prepare_spectrum


@pytest.mark.parametrize("n", [4, 6, 16, 30])
def test_tiny_series_against_direct_dft(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n).astype(np.float32)
    want = np.zeros(n // 2, dtype=np.complex128)
    for k in range(1, n // 2):
        want[k] = sum(float(x[j]) * complex(math.cos(2 * math.pi * j * k / n), -math.sin(2 * math.pi * j * k / n))
                      for j in range(n))
    want /= math.sqrt(np.mean(np.abs(want[1:]) ** 2))
    got = prepare_spectrum(x)
    assert got.dtype == np.complex64 and got.shape == (n // 2,)
    assert np.max(np.abs(got - want)) < 1e-6


def test_cosine_at_integer_bin_closed_form():
    """a cos(2 pi k0 j / N + phi) has X[k0] = a N/2 e^{i phi} and nothing else above DC, so the
    normalised bin has power M - 1 (M = N/2 kept bins) and phase phi."""
    n, k0, a, phi = 4096, 300, 0.7, 0.4
    j = np.arange(n)
    x = a * np.cos(2 * np.pi * k0 * j / n + phi) + 3.0       # the offset lands in DC only
    got = prepare_spectrum(x).astype(np.complex128)
    m = n // 2
    assert abs(abs(got[k0]) ** 2 - (m - 1)) < 1e-4 * m
    assert abs(np.angle(got[k0]) - phi) < 1e-6
    rest = np.delete(got, k0)
    assert np.max(np.abs(rest)) < 1e-5


def test_parseval_half_spectrum_and_unit_mean_power():
    rng = np.random.default_rng(2)
    n = 1 << 14
    x = rng.standard_normal(n)
    raw = np.fft.fft(x)
    m = n // 2
    # sum over 1..M-1 of |X_k|^2 is half of N sum x^2 less the DC and Nyquist terms
    half = (n * np.sum(x * x) - abs(raw[0]) ** 2 - abs(raw[m]) ** 2) / 2
    got = prepare_spectrum(x).astype(np.complex128)
    assert got[0] == 0
    assert abs(np.mean(np.abs(got[1:]) ** 2) - 1.0) < 1e-6
    scale = math.sqrt(half / (m - 1))
    assert np.max(np.abs(got[1:] * scale - raw[1:m])) < 1e-5 * scale


def test_zero_above_dc_stays_zero():
    got = prepare_spectrum(np.full(64, 2.5, dtype=np.float32))
    assert np.all(got == 0)


def test_synthetic_recipe_agrees():
    x = synth.time_series(1 << 12, 77, (synth.Tone(0.1, 500.2, 3.0, 5.0),))
    a = prepare_spectrum(x)
    b = synth.spectrum_from_series(x)
    d = np.abs(a.astype(np.complex128) - b.astype(np.complex128))
    assert np.max(d) <= 2.0 ** -22 * max(1.0, float(np.max(np.abs(b))))


def test_rejects_bad_lengths():
    for n in (2, 5):
        with pytest.raises(ValueError):
            prepare_spectrum(np.zeros(n))
