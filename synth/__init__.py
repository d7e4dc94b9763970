"""Seeded synthetic inputs shared by the GPU library's tests, the oracle's tests and the bench.

This module makes spectra and request streams only. It holds none of the
search's arithmetic (no response, template, correlation or power code), so
that the oracle and the GPU path see bit-identical inputs while sharing no
code with each other.
"""

from .spectra import (
    Tone,
    SearchConfig,
    CONFIGS,
    time_series,
    time_series_device,
    spectrum_from_series,
    make_spectrum,
    draw_tones,
    batch_spectra_specs,
    serving_requests,
)

__all__ = [
    "Tone",
    "SearchConfig",
    "CONFIGS",
    "time_series",
    "time_series_device",
    "spectrum_from_series",
    "make_spectrum",
    "draw_tones",
    "batch_spectra_specs",
    "serving_requests",
]
