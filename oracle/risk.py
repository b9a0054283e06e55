"""Failure frequencies and the Risk Index (Section II.C, eq. (1)-(3)).

  lambda_i = 1 / MTTF_i
  F_i  = lambda_i               (eq. 1, N-1 frequency)
  F_ij = lambda_i lambda_j      (eq. 2, N-2 frequency, independent failures)
  R_i  = F_i S_i + sum_{j != i} F_ij S_ij    (eq. 3)

R_i sums the frequency-weighted severity of every scenario in the given list
in which component i takes part, in list order.  With an unordered pair list
each pair appears once; with the paper's ordered list every pair appears
twice.
"""
from __future__ import annotations

import numpy as np


def failure_rate_from_mttf(mttf_years):
    return 1.0 / np.asarray(mttf_years, dtype=float)


def scenario_frequency(outages, lam):
    """F_c for every row of the outage list (eq. 1 and eq. 2)."""
    out = np.asarray(outages)
    F = np.empty(len(out))
    for c, (i, j) in enumerate(out):
        if i < 0:
            F[c] = 0.0              # the base case (-1, -1): nothing fails
        else:
            F[c] = lam[i] if j < 0 else lam[i] * lam[j]
    return F


def risk_index(outages, severe, lam, n_comp):
    """R_i of eq. (3), summed over the list in scenario order."""
    F = scenario_frequency(outages, lam)
    R = np.zeros(n_comp)
    for c, (i, j) in enumerate(np.asarray(outages)):
        if severe[c] and i >= 0:    # the base case involves no component
            R[i] += F[c]
            if j >= 0:
                R[j] += F[c]
    return R
