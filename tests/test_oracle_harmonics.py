"""Pins of the oracle's harmonic summing.

Closed forms on planes built from the lattice coordinates (each harmonic's
index scaling in r, zbar and w shows up in a different sum), the H = 1
identity, the fundamental domain, and a periodic jerked signal whose harmonic
sum peaks at its fundamental.
"""

import numpy as np
import pytest

import synth
from oracle import Grid, oracle_plane
from oracle.harmonics import fundamental_params, fundamental_shape, harmonic_sum, zero_index


def _coord_plane(grid, n_r, f):
    T = grid.n_templates
    out = np.zeros((T, n_r))
    p = np.arange(n_r)
    for t in range(T):
        out[t] = f(grid.zbar(t), grid.w(t), p)
    return out


@pytest.mark.parametrize("H", [1, 2, 3, 4, 8])
def test_closed_forms_on_coordinate_planes(H):
    g = Grid(16.0, 80.0, 2.0, 20.0)
    n_r = 101
    tri = H * (H + 1) / 2
    n_zf, n_wf, n_pf = fundamental_shape(g, n_r, H)
    s = harmonic_sum(_coord_plane(g, n_r, lambda z, w, p: np.ones_like(p, dtype=float)), g, H)
    assert s.shape == (n_zf * n_wf, n_pf) and np.all(s == H)
    s = harmonic_sum(_coord_plane(g, n_r, lambda z, w, p: p.astype(float)), g, H)
    assert np.all(s == np.arange(n_pf) * tri)
    sz = harmonic_sum(_coord_plane(g, n_r, lambda z, w, p: (z + 1000.0) + 0 * p), g, H)
    sw = harmonic_sum(_coord_plane(g, n_r, lambda z, w, p: (w + 5000.0) + 0 * p), g, H)
    for row in range(n_zf * n_wf):
        zf, wf = fundamental_params(g, H, row)
        assert np.all(sz[row] == zf * tri + 1000.0 * H)
        assert np.all(sw[row] == wf * tri + 5000.0 * H)


def test_single_harmonic_is_the_plane():
    g = Grid(6.0, 40.0, 2.0, 20.0)
    rng = np.random.default_rng(1)
    plane = rng.exponential(size=(g.n_templates, 50))
    assert np.array_equal(harmonic_sum(plane, g, 1), plane)


def test_fundamental_domain():
    g = Grid(200.0, 600.0, 2.0, 20.0)
    assert zero_index(g) == 100
    assert fundamental_shape(g, 2 * 4096, 2) == (101, 31, 4096)
    assert fundamental_shape(g, 2 * 4096, 3) == (67, 21, 2731)
    assert fundamental_shape(g, 7, 8) == (25, 7, 1)
    with pytest.raises(ValueError):
        zero_index(Grid(21.0, 60.0, 2.0, 20.0))


def test_periodic_jerked_signal_sums_at_its_fundamental():
    """Four harmonics of a signal with fundamental (rbar, zbar, w) = (400, 6, 20)."""
    n_t = 1 << 13
    rbar, zb, w = 400.0, 6.0, 20.0
    z0 = zb - w / 2
    r0 = rbar - z0 / 2 - w / 6
    tones = tuple(synth.Tone(0.15, h * r0, h * z0, h * w, 0.3 * h) for h in range(1, 5))
    spec = synth.make_spectrum(synth.SearchConfig("four harmonics", n_t, 5, 24.0, 80.0, 2.0, 20.0, tones))
    g = Grid(24.0, 80.0, 2.0, 20.0)
    plane = oracle_plane(spec, g)
    s = harmonic_sum(plane, g, 4)
    row, p = np.unravel_index(int(np.argmax(s)), s.shape)
    assert fundamental_params(g, 4, int(row)) == (zb, w)
    assert p == int(2 * rbar)
    # the sum at the fundamental collects each harmonic's own peak
    peaks = []
    for h in range(1, 5):
        t = (g.J + h * 1) * g.n_z + (zero_index(g) + h * 3)
        peaks.append(plane[t, h * p])
        assert plane[t, h * p] > 0.8 * plane[t, h * p - 2: h * p + 3].max()
    assert abs(s[row, p] - sum(peaks)) < 1e-9 * s[row, p]
    assert s[row, p] > 3 * plane.mean() * 4 + 10
