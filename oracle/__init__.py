"""FP64 CPU oracle for the Fourier-domain jerk search matched filter.

TEST INFRASTRUCTURE ONLY. This package is the slow, plainly written
reference that the GPU library is checked against. Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it. The product path (``paper_1911_01353_amd``) never imports, links
or calls anything here, and nothing here imports the product path.

What the oracle computes, and where it comes from
-------------------------------------------------

The paper (Adamek, Novotny, Dimoudi, Armour, "Searching for pulsars in
extreme orbits - GPU acceleration of the Fourier domain 'jerk' search",
arXiv:1911.01353) defines the search only in prose:

* section "Implementation": every matched filter fits the Fourier response of
  a signal with a given first frequency derivative ``z = fdot T^2`` and second
  frequency derivative ``w = fddot T^3``; the jerk search applies one
  acceleration (z) filter set for every w value searched (Figure 2);
* section "Implementation", Figure 1: the correlation of the spectrum with
  each filter is an overlap-and-save convolution (any correct convolution
  gives the same numbers; the oracle uses the plain direct sum, which is what
  overlap-and-save reproduces exactly in exact arithmetic).

The paper prints no response formula, width rule, grid or precision. The
readings used here (each listed in the design notes of the repository) are:

* ``response.py`` - the response is the Fourier transform over the unit
  observation of a unit tone with cubic phase ``r u + z u^2/2 + w u^3/6``
  (this is what ``z = fdot T^2`` and ``w = fddot T^3`` imply); templates are
  parameterised by the observation-average frequency and fdot.
* ``grid.py`` - the (z, w) lattice and the per-template half-width rule.
* ``plane.py`` - the direct correlation and the power plane.
* ``metrics.py`` - the relative power error floored at the row mean and the
  peak rule used to compare planes.

Parity pins: every function here is pinned by ``tests/test_oracle_*.py`` to
closed forms (sinc, Fresnel), to 30-digit ``mpmath`` quadrature, to the DFT
of a sampled tone, to Parseval's identity, to symmetry, and to brute force on
tiny inputs. None is "parity unpinned".
"""

from .response import response, template_taps, template_response
from .grid import Grid, half_width
from .plane import correlate_row, oracle_plane
from .metrics import relative_power_error, error_summary, peak_index, top2_margin

__all__ = [
    "response",
    "template_response",
    "template_taps",
    "Grid",
    "half_width",
    "correlate_row",
    "oracle_plane",
    "relative_power_error",
    "error_summary",
    "top2_margin",
    "peak_index",
]
