"""Incoherent harmonic summing over the (r, z, w) power plane.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper (section "Results") names the harmonic sum as the stage that follows
matched filtering and improves the sensitivity of Fourier searches, costing at
least as much as the filtering, and leaves it out of its timings; it gives no
definition. Reading used here: a periodic signal with fundamental (r, z, w)
has its h-th harmonic at (h r, h z, h w) (frequency and its derivatives all
scale with h), and the harmonic sum of H harmonics is the plain sum of the
plane's powers at those points,

    S_H(r, z, w) = sum_{h=1}^{H} P(h r, h zbar, h w).

With two outputs per bin (``p = 2 r``) and a lattice that contains ``zbar = 0``
(``zmax`` a multiple of ``dz``; ``w = 0`` is always on it), every harmonic of a
lattice point is itself a lattice point, so no interpolation is involved:
fundamental ``(i, j, p)`` reads template ``(i0 + h (i - i0), J + h (j - J))``
at ``h p``, with ``i0 = zmax / dz`` the index of ``zbar = 0``. Fundamentals are
kept when all H harmonics lie on the plane: ``|i - i0| <= floor(i0 / H)``,
``|j - J| <= floor(J / H)`` and ``H p <= n_r - 1``. The output rows are those
fundamentals in the lattice's own order (w-major), row
``(j - J + floor(J/H)) * n_zf + (i - i0 + floor(i0/H))``, ``n_zf = 2 floor(i0/H) + 1``.
"""

from __future__ import annotations

import numpy as np

from .grid import Grid


def zero_index(grid: Grid) -> int:
    """Index ``i0`` of ``zbar = 0``; ValueError when the lattice does not contain it."""
    q = grid.zmax / grid.dz
    if abs(q - round(q)) > 1e-9:
        raise ValueError("harmonic sums need zmax to be a multiple of dz")
    return int(round(q))


def fundamental_shape(grid: Grid, n_r: int, n_harm: int) -> tuple[int, int, int]:
    """(n_zf, n_wf, n_pf): fundamentals whose n_harm harmonics all lie on the plane."""
    if n_harm < 1 or n_r < 1:
        raise ValueError("n_harm and n_r must be >= 1")
    i0 = zero_index(grid)
    return 2 * (i0 // n_harm) + 1, 2 * (grid.J // n_harm) + 1, (n_r - 1) // n_harm + 1


def harmonic_sum(plane: np.ndarray, grid: Grid, n_harm: int) -> np.ndarray:
    """``S_H`` of a full plane ``[T][n_r]`` (rows in template order), in FP64."""
    a = np.asarray(plane, dtype=np.float64)
    if a.shape[0] != grid.n_templates:
        raise ValueError("plane must hold every template of the grid")
    n_r = a.shape[1]
    n_zf, n_wf, n_pf = fundamental_shape(grid, n_r, n_harm)
    i0, J = zero_index(grid), grid.J
    dzf, dwf = n_zf // 2, n_wf // 2
    out = np.zeros((n_zf * n_wf, n_pf), dtype=np.float64)
    p = np.arange(n_pf)
    for jf in range(n_wf):
        for izf in range(n_zf):
            i = i0 - dzf + izf
            j = J - dwf + jf
            acc = np.zeros(n_pf, dtype=np.float64)
            for h in range(1, n_harm + 1):
                t = (J + h * (j - J)) * grid.n_z + (i0 + h * (i - i0))
                acc += a[t, h * p]
            out[jf * n_zf + izf] = acc
    return out


def fundamental_params(grid: Grid, n_harm: int, row: int) -> tuple[float, float]:
    """(zbar, w) of output row ``row`` of a harmonic sum."""
    n_zf = 2 * (zero_index(grid) // n_harm) + 1
    n_wf = 2 * (grid.J // n_harm) + 1
    jf, izf = divmod(row, n_zf)
    return (izf - n_zf // 2) * grid.dz, (jf - n_wf // 2) * grid.dw
