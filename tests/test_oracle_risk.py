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


# --- extensions: non-binary severity, common cause, Monte-Carlo on lambda ---

def test_damping_severity_values():
    from oracle.risk import severity_weights, SEV_DAMPING, SEV_BINARY
    severe = np.array([1, 0, 0, 0, 0, 0, 0, 1])
    zeta = np.array([0.3, 0.0, 0.05, 0.025, 0.2, np.nan, 0.0125, np.nan])
    w = severity_weights(severe, zeta, SEV_DAMPING, zeta_ref=0.05)
    assert np.allclose(w, [1.0, 1.0, 0.0, 0.5, 0.0, 0.0, 0.75, 1.0], rtol=1e-15, atol=1e-15)
    assert severity_weights(severe, zeta, SEV_BINARY).tolist() == severe.tolist()
    # another reference damping
    assert severity_weights([0], [0.05], SEV_DAMPING, zeta_ref=0.1)[0] == 0.5


def _all_severe(n=12, seed=0):
    rng = np.random.default_rng(seed)
    lam = rng.uniform(0.001, 0.1, n)
    lst = contingencies.n1_n2(np.arange(n))
    return lam, lst


def test_weighted_risk_closed_form_all_severe():
    """Every N-1 and unordered N-2 scenario severe: R_k = lam_k (1 + Lambda -
    lam_k); a tagged common-cause pair adds its rate to both members; a
    half-weight severity halves everything."""
    lam, lst = _all_severe()
    n = len(lam)
    L = lam.sum()
    ones = np.ones(len(lst))
    R = risk.risk_index_weighted(lst, ones, lam, n)
    assert np.allclose(R, lam * (1 + L - lam), rtol=1e-14)
    cc = risk.common_cause_table([[2, 5], [5, 7], [2, 5]], [0.01, 0.003, 0.002], n)
    Rc = risk.risk_index_weighted(lst, ones, lam, n, cc)
    extra = np.zeros(n)
    extra[[2, 5]] += 0.012
    extra[[5, 7]] += 0.003
    assert np.allclose(Rc, lam * (1 + L - lam) + extra, rtol=1e-14)
    assert np.allclose(risk.risk_index_weighted(lst, 0.5 * ones, lam, n), 0.5 * R, rtol=1e-15)


def test_monte_carlo_closed_form_ranks():
    """All scenarios severe: R_k = lam_k (1 + Lambda - lam_k) is increasing in
    lam_k (every rate is below (1 + Lambda) / 2), so in every sample the rank
    order of R is that of the sampled rates."""
    from inputs.rate_samples import lognormal_rates
    lam, lst = _all_severe(10, 3)
    n = len(lam)
    S = lognormal_rates(lam, 40, seed=9)
    R, mean, std, hist, quant = risk.risk_monte_carlo(lst, np.ones(len(lst)), S, n)
    L = S.sum(axis=1, keepdims=True)
    assert np.allclose(R, S * (1 + L - S), rtol=1e-13)
    assert np.allclose(mean, (S * (1 + L - S)).mean(axis=0), rtol=1e-13)
    assert np.allclose(std, (S * (1 + L - S)).std(axis=0, ddof=1), rtol=1e-12)
    want = np.zeros((n, n), np.int64)
    for m in range(len(S)):
        order = np.argsort(-S[m], kind="stable")
        want[order, np.arange(n)] += 1
    assert np.array_equal(hist, want)
    assert np.all(hist.sum(axis=1) == len(S)) and np.all(hist.sum(axis=0) == len(S))


def test_monte_carlo_one_sample_is_eq3():
    lam, lst = _all_severe(9, 5)
    rng = np.random.default_rng(1)
    severe = rng.integers(0, 2, len(lst))
    R, *_ = risk.risk_monte_carlo(lst, severe.astype(float), lam[None, :], len(lam))
    ref = np.zeros(len(lam))
    for (i, j), s in zip(lst, severe):       # eq. (3) written out
        if s:
            f = lam[i] if j < 0 else lam[i] * lam[j]
            ref[i] += f
            if j >= 0:
                ref[j] += f
    assert np.allclose(R[0], ref, rtol=1e-14)


def test_rank_quantile_definition():
    """20 samples with ranks 0 (once), 1 (9 times), 2 (10 times): the 5%
    quantile needs 1 sample (rank 0), the median 10 (rank 1), the 95% 19
    (rank 2)."""
    n = 3
    lst = np.array([[0, -1], [1, -1], [2, -1]])
    # component 0's rank set through its rate relative to the others
    S = []
    for r in [0] + [1] * 9 + [2] * 10:
        v = {0: [0.9, 0.5, 0.1], 1: [0.5, 0.9, 0.1], 2: [0.1, 0.5, 0.9]}[r]
        S.append(v)
    _, _, _, hist, quant = risk.risk_monte_carlo(lst, np.ones(3), np.array(S), n)
    assert hist[0].tolist() == [1, 9, 10]
    assert quant[0].tolist() == [0, 1, 2]


def test_n3_risk_closed_form():
    """Every row of an N-1 + N-2 + N-3 list severe: R_k = lam_k (1 + e1 + e2)
    with e1, e2 the first and second elementary symmetric sums of the other
    components' rates."""
    lam, _ = _all_severe(8, 2)
    n = len(lam)
    lst2 = contingencies.n1_n2(np.arange(n))
    lst = np.concatenate([np.concatenate([lst2, np.full((len(lst2), 1), -1)], axis=1),
                          contingencies.n3(np.arange(n))])
    R = risk.risk_index(lst, np.ones(len(lst), bool), lam, n)
    for k in range(n):
        o = np.delete(lam, k)
        e1 = o.sum()
        e2 = (e1 * e1 - (o * o).sum()) / 2
        assert abs(R[k] - lam[k] * (1 + e1 + e2)) < 1e-14
