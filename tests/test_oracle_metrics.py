"""Pins of the comparison rules and of the synthetic input recipe."""

import numpy as np

import synth
from oracle.metrics import error_summary, peak_index, relative_power_error, top2_margin


def test_relative_error_floor():
    ora = np.array([[0.0, 1.0, 2.0, 5.0]])          # row mean 2
    test = np.array([[0.1, 1.1, 2.0, 4.0]])
    e = relative_power_error(test, ora)
    assert np.allclose(e, [[0.05, 0.05, 0.0, 0.2]])
    s = error_summary(test, ora)
    assert abs(s["max"] - 0.2) < 1e-15
    assert abs(s["rms"] - np.sqrt((0.05 ** 2 * 2 + 0.04) / 4)) < 1e-15


def test_relative_error_zero_row():
    z = np.zeros((2, 3))
    assert np.all(relative_power_error(z, z) == 0)


def test_peak_tie_goes_to_lowest_linear_index():
    p = np.zeros((3, 4), dtype=np.float32)
    p[1, 2] = 5
    p[2, 0] = 5
    assert peak_index(p) == (1, 2)
    # values equal in float32 are ties even if float64 differs in the last bits
    q = np.zeros((2, 2))
    q[0, 1] = 1.0
    q[1, 0] = 1.0 + 1e-12
    assert peak_index(q) == (0, 1)
    assert top2_margin(np.array([[1.0, 4.0, 2.0]])) == 0.5


def test_spectrum_recipe_is_deterministic_and_normalised():
    a = synth.spectrum_from_series(synth.time_series(4096, 5, ()))
    b = synth.spectrum_from_series(synth.time_series(4096, 5, ()))
    assert a.dtype == np.complex64 and a.shape == (2048,)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    assert a[0] == 0
    p = np.abs(a[1:].astype(np.complex128)) ** 2
    assert abs(p.mean() - 1.0) < 1e-6


def test_request_stream_ranges():
    reqs = synth.serving_requests(200, 10.0)
    assert all(2 ** 19 <= r["n_samples"] <= 2 ** 24 for r in reqs)
    assert all(50 <= r["zmax"] <= 300 and r["zmax"] % 2 == 0 for r in reqs)
    assert all(r["wmax"] == 3 * r["zmax"] for r in reqs)
    t = [r["arrival_s"] for r in reqs]
    assert all(b >= a for a, b in zip(t, t[1:]))
    specs = synth.batch_spectra_specs(256)
    assert {s[0] // 2 for s in specs} <= {2 ** 20, 2 ** 21, 2 ** 22}
    assert 10 <= sum(1 for s in specs if s[2]) <= 45


def test_relative_error_whole_row_floor_for_windows():
    """A window of a row is floored at the whole row's mean, not at the window's own mean."""
    row = np.array([1.0, 1.0, 1.0, 1.0, 0.0, 10.0, 6.0, 0.0])   # whole-row mean 2.5
    test = row + np.array([0, 0, 0, 0, 0.5, 0, 0, 0.5])
    win = slice(4, 8)                                           # window mean 4
    e_row = relative_power_error(test[None, :], row[None, :])[0, win]
    e_win = relative_power_error(test[None, win], row[None, win], floor=row.mean())[0]
    assert np.array_equal(e_row, e_win)
    assert np.allclose(e_win, [0.2, 0.0, 0.0, 0.2])
    # the window's own mean would have given a looser 0.125
    assert np.allclose(relative_power_error(test[None, win], row[None, win])[0], [0.125, 0, 0, 0.125])
    # one floor per row
    two = np.stack([row[win], row[win]])
    e2 = relative_power_error(two + 0.5, two, floor=[2.5, 5.0])
    assert np.allclose(e2[:, 0], [0.2, 0.1])
    assert error_summary(test[None, win], row[None, win], floor=2.5)["max"] == 0.2
