"""The (zbar, w) template lattice and the per-template half-width, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Lattice (paper, section "Implementation" and Figure 2: one fdot filter set per
fddot value searched):

    zbar_i = -zmax + i * dz,   i = 0 .. n_z - 1,   n_z = floor(2 zmax / dz) + 1
    w_j    = -J dw + j * dw,   j = 0 .. n_w - 1,   J = floor(wmax / dw), n_w = 2J + 1
    template index t = j * n_z + i   (w-major)

Half-width rule (the paper states none). In centred time ``s = u - 1/2`` on
``[-1/2, 1/2]``, the instantaneous frequency of the template's tone minus the
trial frequency ``rbar`` is

    f(s) = -w/24 + zbar s + w s^2 / 2.

Its end-point values are ``+-zbar/2 + w/12``; the interior extremum (at
``s = -zbar / w`` when ``|zbar / w| <= 1/2``) has magnitude
``w/24 + zbar^2 / (2 |w|)``, which never exceeds ``|zbar|/2 + |w|/12``. So

    f_max = |zbar| / 2 + |w| / 12,

the half-width is ``h = ceil(f_max) + margin`` bins and the template has
``K = 2 h`` taps.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def half_width(zbar: float, w: float, margin: int = 16) -> int:
    """Half-width ``h`` (bins) of the template ``(zbar, w)``; ``K = 2h`` taps."""
    fmax = abs(zbar) / 2.0 + abs(w) / 12.0
    return int(math.ceil(fmax)) + int(margin)


@dataclass(frozen=True)
class Grid:
    """The template lattice of one search."""

    zmax: float
    wmax: float
    dz: float
    dw: float
    margin: int = 16

    @property
    def n_z(self) -> int:
        return int(math.floor(2.0 * self.zmax / self.dz + 1e-9)) + 1

    @property
    def n_w(self) -> int:
        return 2 * self.J + 1

    @property
    def J(self) -> int:
        return int(math.floor(self.wmax / self.dw + 1e-9)) if self.dw > 0 else 0

    @property
    def n_templates(self) -> int:
        return self.n_z * self.n_w

    def zbar(self, t: int) -> float:
        return -self.zmax + (t % self.n_z) * self.dz

    def w(self, t: int) -> float:
        return (-self.J + t // self.n_z) * self.dw

    def params(self, t: int) -> tuple[float, float, int]:
        """(zbar, w, half_width) of template ``t``."""
        zb, ww = self.zbar(t), self.w(t)
        return zb, ww, half_width(zb, ww, self.margin)

    def half_widths(self) -> np.ndarray:
        return np.array([self.params(t)[2] for t in range(self.n_templates)], dtype=np.int64)
