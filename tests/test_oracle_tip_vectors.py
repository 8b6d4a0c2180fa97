"""Oracle pins for general tip partial vectors (the pruning recursion's tip
vector in its general form, as phg_set_tip_partials takes it).

* Brute force: the plain sum over internal states with those tips' states
  summed out under their vectors (tests/brute.py, no oracle code), for
  log-likelihoods and every branch derivative.
* Codes as vectors: one-hot and all-ones vectors reproduce the code path
  bit for bit.
* Linearity: a site likelihood is linear in any one tip's vector.
"""
import numpy as np
import pytest

import oracle
from paper_2303_04390_amd import synth
from tests import brute
from tests.test_oracle_pins import small_problem


def code_vectors(codes_row, S):
    C = codes_row.shape[0]
    v = np.zeros((C, S))
    obs = codes_row < S
    v[np.nonzero(obs)[0], codes_row[obs]] = 1.0
    v[~obs] = 1.0
    return v


def random_vectors(rng, C, S, zero_frac=0.3):
    v = rng.uniform(0.0, 1.0, (C, S))
    v[rng.uniform(size=(C, S)) < zero_frac] = 0.0
    v[np.arange(C), rng.integers(0, S, C)] = rng.uniform(0.5, 1.0, C)   # never all-zero
    return v


@pytest.mark.parametrize("S,N,seed", [(4, 5, 1), (4, 6, 2), (3, 4, 3), (20, 3, 4)])
def test_brute_force_with_tip_vectors(S, N, seed):
    prob = small_problem(N, S=S, C=7, seed=seed, R=2, stationary=False)
    rng = np.random.default_rng(100 + seed)
    prob.tip_vectors = {0: random_vectors(rng, 7, S), N - 1: random_vectors(rng, 7, S)}
    out = oracle.evaluate_problem(prob)
    P, dP = brute.expm_P(prob.Q, prob.rates, prob.b)
    L = brute.brute_site_likelihood(prob.parent, P, prob.codes, prob.pi, prob.weights,
                                    tip_vectors=prob.tip_vectors)
    assert np.allclose(out["site_ll"], np.log(L), rtol=1e-12, atol=1e-12)
    for x in range(2 * N - 2):
        dL = brute.brute_site_likelihood(prob.parent, P, prob.codes, prob.pi, prob.weights, deriv_branch=x,
                                         dP=dP, tip_vectors=prob.tip_vectors)
        ref = float(np.sum(prob.pattern_weights * dL / L))
        scale = float(np.sum(prob.pattern_weights * np.abs(dL / L)))
        assert abs(out["grad"][x] - ref) <= 1e-11 * scale + 1e-13, (x, out["grad"][x], ref)


@pytest.mark.parametrize("S", [4, 20])
def test_code_vectors_reproduce_codes_exactly(S):
    prob = small_problem(12, S=S, C=30, seed=5, ambiguous=0.2)
    base = oracle.evaluate_problem(prob)
    prob.tip_vectors = {t: code_vectors(prob.codes[t], S) for t in (0, 3, 7, 11)}
    out = oracle.evaluate_problem(prob)
    assert out["logl"] == base["logl"]
    assert np.array_equal(out["grad"], base["grad"])


def test_site_likelihood_linear_in_one_tip_vector():
    """L_c(v) = sum_t v[c, t] L_c(e_t) for one tip, and the same for dL_c/db."""
    S, C = 4, 9
    prob = small_problem(7, S=S, C=C, seed=8, R=3, stationary=False)
    prob.pattern_weights = np.ones(C)
    rng = np.random.default_rng(3)
    v = random_vectors(rng, C, S, zero_frac=0.0)
    tip = 2
    prob.tip_vectors = {tip: v}
    out = oracle.evaluate_problem(prob)
    Lv = np.exp(out["site_ll"])
    Lsum = np.zeros(C)
    for t in range(S):
        e = np.zeros((C, S))
        e[:, t] = 1.0
        prob.tip_vectors = {tip: e}
        Lsum += v[:, t] * np.exp(oracle.evaluate_problem(prob)["site_ll"])
    assert np.allclose(Lv, Lsum, rtol=1e-12, atol=0)
