"""Pins for eq. (1)-(3): the paper's printed Risk Index values.

With the paper's inventory and Table I rates, a component k whose every N-1
and ordered N-2 scenario is severe has R_k = lam_k + 2 lam_k (Lambda - lam_k)
(each unordered pair appears twice in the ordered list).  For a line this is
the printed maximum 1.472; for a transformer the top of the printed
0.56-0.59 range.  The scenario count 57,122 = 1 base + 239 N-1 + 239*238
ordered N-2 also follows from the inventory.
"""
import json
import os

import numpy as np

from oracle import risk
from inputs import contingencies

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_risk.json")))


def _paper_inventory():
    lam = np.concatenate([np.full(GOLD["n_lines"], GOLD["lambda_line"]),
                          np.full(GOLD["n_transformers"], GOLD["lambda_transformer"]),
                          np.full(GOLD["n_generators"], GOLD["lambda_generator"])])
    return lam


def test_scenario_count_matches_paper():
    lam = _paper_inventory()
    lst = contingencies.n1_n2(np.arange(len(lam)), ordered=True)
    assert 1 + len(lst) == GOLD["scenario_count"]


def test_printed_top_risk_values():
    lam = _paper_inventory()
    n = len(lam)
    lst = contingencies.n1_n2(np.arange(n), ordered=True)
    line, trafo = 0, GOLD["n_lines"]
    for k, printed in [(line, GOLD["max_line_risk"]),
                       (trafo, GOLD["transformer_risk_range"][1])]:
        severe = ((lst[:, 0] == k) | (lst[:, 1] == k)).astype(np.uint8)
        R = risk.risk_index(lst, severe, lam, n)
        assert round(R[k], 3) == printed
    # with each pair counted once the printed line value is unreachable
    ulst = contingencies.n1_n2(np.arange(n), ordered=False)
    severe = ((ulst[:, 0] == 0) | (ulst[:, 1] == 0)).astype(np.uint8)
    assert risk.risk_index(ulst, severe, lam, n)[0] < 0.8


def test_total_risk_identity_and_ordered_doubling():
    rng = np.random.default_rng(5)
    n = 12
    lam = rng.uniform(0.001, 0.1, n)
    ul = contingencies.n1_n2(np.arange(n))
    s = rng.integers(0, 2, len(ul)).astype(np.uint8)
    R = risk.risk_index(ul, s, lam, n)
    F = risk.scenario_frequency(ul, lam)
    size = np.where(ul[:, 1] < 0, 1, 2)
    assert np.isclose(R.sum(), np.sum(size * F * s), rtol=1e-13)
    # ordered list with symmetric severities: N-2 part doubles
    ol = contingencies.n1_n2(np.arange(n), ordered=True)
    key = {(min(a, b), max(a, b)) if b >= 0 else (a, -1): v for (a, b), v in zip(ul, s)}
    so = np.array([key[(min(a, b), max(a, b)) if b >= 0 else (a, -1)] for a, b in ol], np.uint8)
    Ro = risk.risk_index(ol, so, lam, n)
    n1 = ul[:, 1] < 0
    R1 = risk.risk_index(ul[n1], s[n1], lam, n)
    assert np.allclose(Ro, R1 + 2 * (R - R1), rtol=1e-13)


def test_mttf_conversion():
    assert np.allclose(risk.failure_rate_from_mttf([20, 50, 10]), [0.05, 0.02, 0.10])


def test_base_case_row_adds_no_risk():
    """Eq. (3) sums over scenarios in which component i fails; the base case
    (-1, -1) has none, so it adds nothing whatever its severity."""
    from oracle import risk
    lam = np.array([0.1, 0.2, 0.3])
    lst = np.array([[0, -1], [1, 2], [-1, -1]])
    R1 = risk.risk_index(lst, np.array([1, 1, 1]), lam, 3)
    R0 = risk.risk_index(lst[:2], np.array([1, 1]), lam, 3)
    assert np.array_equal(R1, R0)
    assert risk.scenario_frequency(lst, lam)[2] == 0.0
