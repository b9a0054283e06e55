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
    """F_c for every row of the outage list: the product of the outaged
    components' rates (eq. 1 for N-1, eq. 2 for N-2, and the same
    independence for rows of three); -1 entries pad a row."""
    out = np.asarray(outages)
    F = np.empty(len(out))
    for c, row in enumerate(out):
        ids = [int(v) for v in row if v >= 0]
        if not ids:
            F[c] = 0.0              # the base case: nothing fails
            continue
        f = lam[ids[0]]
        for k in ids[1:]:
            f = f * lam[k]
        F[c] = f
    return F


def risk_index(outages, severe, lam, n_comp):
    """R_i of eq. (3), summed over the list in scenario order."""
    F = scenario_frequency(outages, lam)
    R = np.zeros(n_comp)
    for c, row in enumerate(np.asarray(outages)):
        if not severe[c]:
            continue
        for k in row:               # the base case involves no component
            if k >= 0:
                R[k] += F[c]
    return R


# --- extensions listed as future work in Section V.C -------------------------
#
# Non-binary severity.  The paper suggests a continuous severity built, for
# instance, from damping ratios.  Reading taken here: a scenario severe by any
# Section II.B criterion keeps S = 1; a secure scenario gets
#     S = clip((zeta_ref - zeta_min) / zeta_ref, 0, 1),
# so S falls linearly from 1 at zero damping to 0 at the reference damping
# zeta_ref (default 5%) and stays 0 above it.
#
# Common-cause failures.  The paper's N-2 frequency assumes independent
# failures; a pair (i, j) that can fail together from one cause (two lines on
# one tower) has in addition that cause's frequency, so
#     F_ij = lambda_i lambda_j + lambda_cc(i, j),
# with lambda_cc given per tagged pair (both orders of the pair share it).
#
# Monte-Carlo on the failure rates.  For M sampled rate vectors (the samples
# are an input) R_i is evaluated once per sample with eq. (3); the spread of
# R_i and of each component's rank (0 = the largest R) over the samples give
# the confidence intervals on the ranking that the paper asks for.

SEV_BINARY, SEV_DAMPING = 0, 1


def severity_weights(severe, min_damping, mode=SEV_BINARY, zeta_ref=0.05):
    """Per-scenario severity S_c: the binary record, or the damping-based
    continuous severity above."""
    severe = np.asarray(severe)
    out = np.empty(len(severe))
    for c in range(len(severe)):
        if severe[c] or mode == SEV_BINARY:
            out[c] = 1.0 if severe[c] else 0.0
        else:
            z = float(min_damping[c])
            if not np.isfinite(z):
                out[c] = 0.0        # no state matrix: nothing to grade
            else:
                out[c] = min(max((zeta_ref - z) / zeta_ref, 0.0), 1.0)
    return out


def common_cause_table(pairs, rates, n_comp):
    """lambda_cc(i, j) as a symmetric table (0 where no pair is tagged; a pair
    listed twice adds its rates)."""
    T = np.zeros((n_comp, n_comp))
    for (i, j), r in zip(np.asarray(pairs).reshape(-1, 2), np.asarray(rates, float)):
        T[i, j] += r
        if i != j:
            T[j, i] += r
    return T


def risk_index_weighted(outages, weight, lam, n_comp, cc=None):
    """R_i = sum over the list of F_c S_c for the scenarios containing i, with
    a real-valued severity S_c and, optionally, the common-cause table cc
    added to every N-2 frequency; summed in scenario order."""
    R = np.zeros(n_comp)
    for c, (i, j) in enumerate(np.asarray(outages)):
        if i < 0 or weight[c] == 0.0:
            continue
        if j < 0:
            f = lam[i]
        else:
            f = lam[i] * lam[j] + (cc[i, j] if cc is not None else 0.0)
        R[i] += f * weight[c]
        if j >= 0:
            R[j] += f * weight[c]
    return R


RANK_QUANTILES = (5, 50, 95)     # percent


def risk_monte_carlo(outages, weight, lam_samples, n_comp, cc=None):
    """R for every sampled rate vector (eq. (3) per sample), then per
    component: mean and sample standard deviation of R, the histogram of its
    rank over the samples (rank 0 = largest R; equal R ranked by component
    id), and the rank quantiles of RANK_QUANTILES: the smallest rank r whose
    cumulative count reaches ceil(q M / 100)."""
    lam_samples = np.atleast_2d(np.asarray(lam_samples, float))
    M = lam_samples.shape[0]
    R = np.stack([risk_index_weighted(outages, weight, lam_samples[m], n_comp, cc)
                  for m in range(M)])
    mean = R.mean(axis=0)
    std = R.std(axis=0, ddof=1) if M > 1 else np.zeros(n_comp)
    hist = np.zeros((n_comp, n_comp), np.int64)
    ids = np.arange(n_comp)
    for m in range(M):
        order = np.lexsort((ids, -R[m]))        # descending R, then ascending id
        rank = np.empty(n_comp, np.int64)
        rank[order] = ids
        hist[ids, rank] += 1
    cum = np.cumsum(hist, axis=1)
    quant = np.zeros((n_comp, len(RANK_QUANTILES)), np.int64)
    for k, q in enumerate(RANK_QUANTILES):
        need = max(1, -(-q * M // 100))
        quant[:, k] = np.argmax(cum >= need, axis=1)
    return R, mean, std, hist, quant
