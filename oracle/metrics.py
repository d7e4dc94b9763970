"""Comparison rules for power planes: floored relative error and the peak rule.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Relative error. Plain ``|dP| / P`` is ill-posed where the power is near zero,
so the denominator is floored at the row mean of the oracle plane:

    e[t][p] = |P_test[t][p] - P_oracle[t][p]| / max(P_oracle[t][p], mean_p P_oracle[t][:])

For unit-mean-power noise the row mean is the template's captured energy
(about 1), so the floor only matters well below the typical power.

The floor is the mean of the WHOLE row. When only a window of a row is
compared (full-size planes are checked on sampled windows), the window's own
mean is not that floor: a window centred on a strong signal has a larger mean
and would loosen the bar exactly there. Such callers pass the whole-row mean
of the oracle as ``floor``.

Peak rule. The global peak is the largest power; equal values resolve to the
lowest linear index ``t * width + p``. The decision is taken in FP32 (the
precision of the GPU plane) on both sides.
"""

from __future__ import annotations

import numpy as np


def relative_power_error(test: np.ndarray, oracle: np.ndarray, floor=None) -> np.ndarray:
    """Per-point floored relative power error, shape of the inputs.

    ``floor``: the oracle's mean power over each whole row (scalar, or one value
    per row), for inputs that hold only part of each row. Default: the mean of
    the rows given, which is the whole-row mean when whole rows are given.
    """
    test = np.asarray(test, dtype=np.float64)
    oracle = np.asarray(oracle, dtype=np.float64)
    if test.shape != oracle.shape:
        raise ValueError(f"shape mismatch {test.shape} vs {oracle.shape}")
    if oracle.ndim == 1:
        oracle2, test2 = oracle[None, :], test[None, :]
    else:
        oracle2, test2 = oracle, test
    if floor is None:
        floor = oracle2.mean(axis=1, keepdims=True)
    else:
        floor = np.asarray(floor, dtype=np.float64).reshape(-1, 1)
        if floor.shape[0] not in (1, oracle2.shape[0]):
            raise ValueError("floor needs one value per row")
    denom = np.maximum(oracle2, floor)
    # An all-zero row (empty input) compares exactly.
    denom = np.where(denom > 0.0, denom, 1.0)
    e = np.abs(test2 - oracle2) / denom
    return e.reshape(test.shape)


def error_summary(test: np.ndarray, oracle: np.ndarray, floor=None) -> dict:
    """Max and RMS of the floored relative error (``floor`` as in ``relative_power_error``)."""
    e = relative_power_error(test, oracle, floor)
    if e.size == 0:
        return {"max": 0.0, "rms": 0.0}
    return {"max": float(e.max()), "rms": float(np.sqrt(np.mean(e * e)))}


def peak_index(plane: np.ndarray) -> tuple[int, int]:
    """(row, column) of the largest FP32 power; ties go to the lowest linear index."""
    p32 = np.asarray(plane, dtype=np.float32)
    flat = int(np.argmax(p32.reshape(-1)))  # argmax returns the first maximum
    return divmod(flat, p32.shape[1])


def top2_margin(plane: np.ndarray) -> float:
    """Relative gap between the largest and second-largest value of a plane."""
    v = np.sort(np.asarray(plane, dtype=np.float64).reshape(-1))
    if v.size < 2 or v[-1] <= 0:
        return 0.0
    return float((v[-1] - v[-2]) / v[-1])
