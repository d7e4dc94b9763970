"""Pins of the oracle's template lattice and half-width rule."""

import math

import numpy as np
import pytest

from oracle.grid import Grid, half_width


@pytest.mark.parametrize("zmax,wmax,n_z,n_w", [
    (20, 60, 21, 7),        # 2^15-bin single search
    (200, 600, 201, 61),    # 2^22-bin realistic search
    (100, 300, 101, 31),    # batched de-dispersion trials
    (50, 150, 51, 15),      # smallest serving grid (wmax not a multiple of dw)
    (300, 900, 301, 91),    # largest serving grid
])
def test_grid_counts(zmax, wmax, n_z, n_w):
    g = Grid(zmax, wmax, 2.0, 20.0)
    assert (g.n_z, g.n_w, g.n_templates) == (n_z, n_w, n_z * n_w)
    # w-major order, ends of the lattice
    assert g.zbar(0) == -zmax and g.w(0) == -g.J * 20.0
    assert g.zbar(g.n_templates - 1) == zmax and g.w(g.n_templates - 1) == g.J * 20.0
    assert g.zbar(n_z) == -zmax and g.w(n_z) == g.w(0) + 20.0


@pytest.mark.parametrize("zb,w,K", [(0, 0, 32), (20, 60, 62), (100, 300, 182),
                                    (200, 600, 332), (300, 900, 482), (-20, 60, 62)])
def test_half_width_examples(zb, w, K):
    assert 2 * half_width(float(zb), float(w)) == K


def test_half_width_against_sampled_sweep():
    """ceil(max |f(s)|) from the analytic extremum equals the brute-force maximum.

    f(s) is the instantaneous frequency offset of the template's tone from the
    trial frequency: d/du of the phase (q u + z u^2/2 + w u^3/6) with the
    average-value substitution, at u = s + 1/2.
    """
    rng = np.random.default_rng(11)
    s = np.linspace(-0.5, 0.5, 200001)
    for _ in range(300):
        zb = rng.uniform(-300, 300)
        w = rng.uniform(-900, 900)
        q0 = -zb / 2 + w / 12        # offset at u = 0 for qbar = 0
        z0 = zb - w / 2
        u = s + 0.5
        f = q0 + z0 * u + w * u * u / 2
        fmax = np.max(np.abs(f))
        # the dense sampling underestimates the max by < 1e-6; skip near-integer cases
        if abs(fmax - round(fmax)) < 1e-4:
            continue
        assert half_width(zb, w, 0) == math.ceil(fmax)


def test_grid_half_widths_small_search():
    g = Grid(20, 60, 2, 20)
    hs = g.half_widths()
    assert hs.min() == 16 and 2 * hs.max() == 62
    # template t = 102 is (zbar, w) = (16, 20)
    assert g.params(102)[:2] == (16.0, 20.0)
