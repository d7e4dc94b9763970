"""Candidate selection over the power plane: statistics, threshold, peaks.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper (section "Results") times the matched filter together with
candidate selection, which it describes as computing the mean and standard
deviation and then keeping only the peaks that lie above a threshold the user
chooses. It gives neither the domain of the statistics nor the peak rule.
Readings used here:

* statistics are per plane row (one template): the population mean ``mu_t``
  and standard deviation ``sigma_t`` (divisor ``n_r``, not ``n_r - 1``) of the
  ``n_r`` powers of the row, accumulated in FP64;
* the threshold is ``mu_t + k sigma_t`` for a user-given ``k``;
* a peak is a local maximum along ``r`` inside its row: strictly greater than
  its left neighbour and not less than its right one (the row's ends count as
  having no neighbour on that side), so a flat top of equal powers gives one
  candidate, at its leftmost point;
* a candidate is a point that is a peak and whose power, widened to FP64, is
  strictly above the threshold. Its significance is ``(P - mu_t) / sigma_t``.

A row of constant power has ``sigma_t = 0``: no point lies strictly above
``mu_t``, so the row has no candidates.
"""

from __future__ import annotations

import numpy as np


def row_statistics(plane: np.ndarray) -> np.ndarray:
    """``[rows, 2]`` FP64 array of (mean, population standard deviation) per row."""
    a = np.asarray(plane, dtype=np.float64)
    if a.ndim != 2:
        raise ValueError("plane must be 2-D")
    out = np.zeros((a.shape[0], 2), dtype=np.float64)
    if a.shape[1] == 0:
        return out
    mean = a.mean(axis=1)
    var = ((a - mean[:, None]) ** 2).mean(axis=1)
    out[:, 0] = mean
    out[:, 1] = np.sqrt(var)
    return out


def is_peak(row: np.ndarray) -> np.ndarray:
    """Boolean mask of the local maxima of one row (see the module docstring)."""
    r = np.asarray(row)
    m = np.ones(r.shape[0], dtype=bool)
    if r.shape[0] > 1:
        m[1:] &= r[1:] > r[:-1]
        m[:-1] &= r[:-1] >= r[1:]
    return m


def find_candidates(plane: np.ndarray, k_sigma: float, stats: np.ndarray | None = None,
                    row_template=None) -> np.ndarray:
    """Candidates of a plane slab, ordered by (template, p).

    ``row_template[i]`` is the template index of row ``i`` (default ``i``).
    Returns a structured array with fields ``t``, ``p``, ``power`` (FP32, the
    plane's value) and ``sigma`` (FP64 significance).
    """
    a = np.asarray(plane, dtype=np.float32)
    rows = a.shape[0]
    st = row_statistics(a) if stats is None else np.asarray(stats, dtype=np.float64)
    tmpl = np.arange(rows) if row_template is None else np.asarray(row_template)
    recs = []
    for i in range(rows):
        mu, sd = st[i]
        thr = mu + k_sigma * sd
        row = a[i]
        hit = is_peak(row) & (row.astype(np.float64) > thr)
        for p in np.nonzero(hit)[0]:
            recs.append((int(tmpl[i]), int(p), row[p], (float(row[p]) - mu) / sd))
    dt = np.dtype([("t", np.int64), ("p", np.int64), ("power", np.float32), ("sigma", np.float64)])
    out = np.array(recs, dtype=dt)
    return np.sort(out, order=["t", "p"])
