"""Pins of the oracle with a separate substitution model per rate category
(Q^(r) = gamma_r Q_r, the general case the gradient-kernel section allows):
brute-force summation with scipy's expm of each category's own generator,
central differences of the log-likelihood, and the two reductions to a
shared model."""
import numpy as np
import pytest

import oracle
from paper_2303_04390_amd import synth
from tests import brute


def cat_problem(N, C, seed, R=3, S=4, ambiguous=0.1):
    rng = np.random.default_rng(seed)
    parent = synth.yule_topology(N, rng)
    b = synth.exponential_branch_lengths(N, 0.3, rng)
    Qs, V, Vinv, lam = synth.category_models(S, R, rng)
    pi = rng.dirichlet([3.0] * S)
    rates = rng.gamma(2.0, 0.5, R)
    w = rng.dirichlet([3.0] * R)
    codes = rng.integers(0, S, (N, C))
    codes[rng.random((N, C)) < ambiguous] = S
    prob = synth.Problem(parent=parent, b=b, V=V, Vinv=Vinv, lam=lam, pi=pi, rates=rates, weights=w,
                         codes=codes.astype(np.int32), pattern_weights=1.0 + rng.poisson(1.0, C), Q=Qs)
    return prob


@pytest.mark.parametrize("N,seed", [(3, 0), (4, 1), (5, 2)])
def test_brute_force_logl_and_every_derivative(N, seed):
    prob = cat_problem(N, 6, seed)
    P, dP = brute.expm_P(prob.Q, prob.rates, prob.b)
    out = oracle.evaluate_problem(prob)
    L = brute.brute_site_likelihood(prob.parent, P, prob.codes, prob.pi, prob.weights)
    assert abs(out["logl"] - np.sum(prob.pattern_weights * np.log(L))) <= 1e-12 * abs(out["logl"])
    for x in range(2 * N - 2):
        dL = brute.brute_site_likelihood(prob.parent, P, prob.codes, prob.pi, prob.weights,
                                         deriv_branch=x, dP=dP)
        g = np.sum(prob.pattern_weights * dL / L)
        assert abs(out["grad"][x] - g) <= 1e-10 * max(abs(g), out["absgrad"][x] * 1e-2) + 1e-13, (x, out["grad"][x], g)


def test_central_differences_per_category_models():
    prob = cat_problem(12, 150, 5, R=4)
    out = oracle.evaluate_problem(prob)
    for x in range(22):
        h = 1e-4 * max(prob.b[x], 1e-2)

        def ll(bx):
            bb = prob.b.copy()
            bb[x] = bx
            return oracle.evaluate(prob.parent, bb, prob.V, prob.Vinv, prob.lam, prob.pi, prob.rates,
                                   prob.weights, prob.codes, prob.pattern_weights)["logl"]

        d = lambda hh: (ll(prob.b[x] + hh) - ll(prob.b[x] - hh)) / (2 * hh)  # noqa: E731
        rich = (4 * d(h / 2) - d(h)) / 3
        assert abs(out["grad"][x] - rich) <= 1e-6 * max(abs(rich), out["absgrad"][x] * 1e-2) + 1e-8, \
            (x, out["grad"][x], rich)


def test_identical_categories_reduce_to_the_shared_model():
    prob = synth.config_problem("hky16", seed=2, n_patterns=200)
    R = prob.n_categories
    shared = oracle.evaluate_problem(prob)
    stack = synth.Problem(**{**prob.__dict__, "V": np.stack([prob.V] * R),
                             "Vinv": np.stack([prob.Vinv] * R), "lam": np.stack([prob.lam] * R)})
    per = oracle.evaluate_problem(stack)
    assert per["logl"] == shared["logl"] and np.array_equal(per["grad"], shared["grad"])


def test_scaled_generators_equal_category_rates():
    """Q_r = gamma_r Q with unit rates is the shared model with rates gamma_r."""
    prob = synth.config_problem("hky16", seed=3, n_patterns=200)
    R = prob.n_categories
    shared = oracle.evaluate_problem(prob)
    stack = synth.Problem(**{**prob.__dict__, "V": np.stack([prob.V] * R),
                             "Vinv": np.stack([prob.Vinv] * R),
                             "lam": np.stack([prob.rates[r] * prob.lam for r in range(R)]),
                             "rates": np.ones(R)})
    per = oracle.evaluate_problem(stack)
    assert abs(per["logl"] - shared["logl"]) <= 1e-12 * abs(shared["logl"])
    assert np.max(np.abs(per["grad"] - shared["grad"]) / np.maximum(np.abs(shared["grad"]),
                                                                   1e-2 * shared["absgrad"])) <= 1e-10
