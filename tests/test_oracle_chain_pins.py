"""Pins of the oracle's chain rules (node heights, branch rate scalars,
branch-set sums) against central finite differences of the oracle's own
log-likelihood written as a function of heights and rates -- a route that
does not use the chain-rule formulas -- and against the translation
invariance of a dated tree (moving every height by the same amount leaves
every branch length unchanged)."""
import numpy as np

import oracle
from paper_2303_04390_amd import synth


def dated_problem(N=12, C=200, seed=0):
    rng = np.random.default_rng(seed)
    parent = synth.yule_topology(N, rng)
    heights, rates = synth.time_tree(parent, rng, mean_interval=0.05, rate_sigma=0.4)
    b = oracle.branch_lengths_from_time_tree(parent, heights, rates)
    pi = rng.dirichlet([3.0] * 4)
    Q = synth.hky_model(2.5, pi)
    cr, cw = synth.discrete_gamma(0.6, 4)
    prob = synth.make_problem(parent, b, Q, pi, cr, rng.dirichlet([4.0] * 4), C, rng,
                              pattern_weights=1.0 + rng.poisson(2.0, C), ambiguous_fraction=0.05)
    return prob, heights, rates


def logl_dated(prob, heights, rates):
    b = oracle.branch_lengths_from_time_tree(prob.parent, heights, rates)
    return oracle.evaluate(prob.parent, b, prob.V, prob.Vinv, prob.lam, prob.pi, prob.rates,
                           prob.weights, prob.codes, prob.pattern_weights)["logl"]


def richardson(f, h):
    d = lambda hh: (f(hh) - f(-hh)) / (2 * hh)  # noqa: E731
    return (4 * d(h / 2) - d(h)) / 3


def test_branch_lengths_from_time_tree_definition():
    prob, heights, rates = dated_problem(N=5, C=10, seed=3)
    for i in range(2 * 5 - 2):
        k = prob.parent[i]
        assert heights[k] > heights[i]
        assert prob.b[i] == (heights[k] - heights[i]) * rates[i]


def test_height_and_rate_gradients_match_finite_differences():
    prob, heights, rates = dated_problem()
    ref = oracle.evaluate_problem(prob)
    dh, dr = oracle.time_tree_gradients(prob.parent, heights, rates, ref["grad"])
    n = 2 * 12 - 1
    for k in range(n):
        def f(e):
            h = heights.copy()
            h[k] += e
            return logl_dated(prob, h, rates)
        fd = richardson(f, 1e-5)
        assert abs(dh[k] - fd) <= 1e-6 * max(abs(fd), 1.0), (k, dh[k], fd)
    for i in range(n - 1):
        def f(e):
            r = rates.copy()
            r[i] += e
            return logl_dated(prob, heights, r)
        fd = richardson(f, 1e-5 * rates[i])
        assert abs(dr[i] - fd) <= 1e-6 * max(abs(fd), 1.0), (i, dr[i], fd)


def test_height_gradient_is_translation_invariant():
    prob, heights, rates = dated_problem(seed=5)
    ref = oracle.evaluate_problem(prob)
    dh, _ = oracle.time_tree_gradients(prob.parent, heights, rates, ref["grad"])
    scale = np.sum(np.abs(dh))
    assert abs(np.sum(dh)) <= 1e-12 * scale
    shift = lambda e: logl_dated(prob, heights + e, rates)  # noqa: E731
    assert abs(richardson(shift, 1e-3)) <= 1e-9 * scale


def test_strict_and_local_clock_rates_match_finite_differences():
    """Branches in a set share one rate mu_j (rate scalar = mu_j); the set
    sums of d/d rate_i are d logL / d mu_j."""
    prob, heights, _ = dated_problem(seed=7)
    n = 2 * 12 - 1
    rng = np.random.default_rng(1)
    set_of = rng.integers(-1, 3, n - 1)            # three local clocks, some branches fixed
    mu = np.array([0.8, 1.3, 0.6])
    base = np.full(n - 1, 1.1)                     # rate of branches in no set

    def rates_for(m):
        r = base.copy()
        r[set_of >= 0] = m[set_of[set_of >= 0]]
        return r

    rates = rates_for(mu)
    prob.b = oracle.branch_lengths_from_time_tree(prob.parent, heights, rates)
    ref = oracle.evaluate_problem(prob)
    _, dr = oracle.time_tree_gradients(prob.parent, heights, rates, ref["grad"])
    d_mu = oracle.branch_set_sums(dr, set_of, 3)
    for j in range(3):
        def f(e):
            m = mu.copy()
            m[j] += e
            return logl_dated(prob, heights, rates_for(m))
        fd = richardson(f, 1e-5)
        assert abs(d_mu[j] - fd) <= 1e-6 * max(abs(fd), 1.0), (j, d_mu[j], fd)
    # a strict clock is one set holding every branch (all rates = mu = 1)
    r1 = np.ones(n - 1)
    prob.b = oracle.branch_lengths_from_time_tree(prob.parent, heights, r1)
    ref1 = oracle.evaluate_problem(prob)
    _, dr1 = oracle.time_tree_gradients(prob.parent, heights, r1, ref1["grad"])
    strict = oracle.branch_set_sums(dr1, np.zeros(n - 1, int), 1)[0]
    fd = richardson(lambda e: logl_dated(prob, heights, r1 * (1 + e)), 1e-5)
    assert abs(strict - fd) <= 1e-6 * max(abs(fd), 1.0), (strict, fd)


def test_branch_set_sums_brute_force():
    vals = np.arange(1.0, 11.0)
    set_of = np.array([0, 2, -1, 2, 0, 1, 1, -1, 0, 2])
    out = oracle.branch_set_sums(vals, set_of, 4)
    assert list(out) == [1 + 5 + 9, 6 + 7, 2 + 4 + 10, 0.0]
