"""The FP32 precision guard (host logic) and the conditioning fact it rests on.

The guard's statistic is checked against a restatement of its definition on
small trees.  The conditioning fact is shown with the oracle's own
recursions run in float64 except that every stored partial (post-order p,
pre-order q) is rounded once to float32: on a 1000-deep caterpillar with
branch lengths ~Exp(1) that rounding alone moves some derivative beyond the
1e-4 bar, while on a tree shaped like the 1000-taxon benchmark workload it
stays an order of magnitude inside; the statistic separates the two.  No kernel runs here.
"""
import numpy as np
import pytest

import oracle
from oracle.likelihood import tip_partials, transition_matrices, tree_structure, rate_matrix
from paper_2303_04390_amd import binding as B
from paper_2303_04390_amd import synth


def _saturation(prob):
    """max over internal k and children x' of min(L_k, L_x'),
    L_v = b_v * max_r gamma_r mu_r, mu_r the smallest non-zero |lambda|."""
    lam = np.abs(np.atleast_2d(prob.lam))
    if lam.shape[0] == 1:
        lam = np.repeat(lam, len(prob.rates), axis=0)
    mus = []
    for row in lam:
        i0 = int(np.argmin(row))
        keep = np.ones(len(row), bool)
        if row[i0] <= 1e-9 * row.max():
            keep[i0] = False
        mus.append(row[keep].min())
    rate = max(g * m for g, m in zip(prob.rates, mus))
    n = len(prob.parent)
    L = np.append(np.asarray(prob.b) * rate, np.inf)
    best = 0.0
    for x in range(n - 1):
        k = prob.parent[x]
        best = max(best, min(L[k], L[x]))
    return best


def _ctx_for(prob):
    ctx = B.Context(prob.n_tips, prob.n_patterns, prob.n_states, prob.n_categories, B.PHG_FP32_SCALED)
    ctx.set_problem(prob)
    return ctx


@pytest.mark.parametrize("which", ["hky16", "aa500", "codon128"])
def test_saturation_statistic_matches_definition(which):
    prob = synth.config_problem(which, seed=1, n_patterns=8)
    with _ctx_for(prob) as ctx:
        got = B.phg_fp32_saturation(ctx.handle)
    assert got == pytest.approx(_saturation(prob), rel=1e-12)


def test_saturation_per_category_models_and_root():
    rng = np.random.default_rng(5)
    prob = synth.config_problem("hky16", seed=3, n_patterns=8)
    prob.Q, prob.V, prob.Vinv, prob.lam = synth.category_models(4, 4, rng)
    # the root's children: L_root counts as infinite, so a long root child
    # alone sets the statistic
    root = 2 * prob.n_tips - 2
    child = int(np.nonzero(prob.parent == root)[0][0])
    prob.b = prob.b.copy()
    prob.b[child] = 50.0
    with _ctx_for(prob) as ctx:
        got = B.phg_fp32_saturation(ctx.handle)
    assert got == pytest.approx(_saturation(prob), rel=1e-12)
    assert got > 10


def test_guard_calls_validate():
    prob = synth.config_problem("hky16", seed=0, n_patterns=8)
    ctx = B.Context(prob.n_tips, prob.n_patterns, 4, 4, B.PHG_FP32_SCALED)
    try:
        with pytest.raises(B.PhgError) as e:
            B.phg_fp32_saturation(ctx.handle)
        assert e.value.status == B.PHG_ERR_STATE
        with pytest.raises(B.PhgError) as e:
            B.phg_set_fp32_guard(ctx.handle, -1.0)
        assert e.value.status == B.PHG_ERR_ARG
        with pytest.raises(B.PhgError):
            B.phg_set_fp32_guard(ctx.handle, float("nan"))
        B.phg_set_fp32_guard(ctx.handle, 0.0)
        B.phg_set_fp32_guard(ctx.handle, 2.5)
        assert B.phg_last_precision(ctx.handle) == -1
    finally:
        ctx.close()


def _storage_rounded_gradient(prob):
    """The pre-order and gradient of eq:preorder and eq:gradient in the form
    the kernels take for branch x below node k with sibling x':
    u = q_k o (P_x' p_x'), d = sum_r w_r u.(dP_x p_x) / sum_r w_r u.(P_x p_x)
    with dP = gamma_r Q P (equal to eq:gradient because q_x = P_x^T u).
    Arithmetic in float64; each stored partial (p at internal nodes, q at
    internal nodes) rounded once to float32 after an exact power-of-two
    normalisation, which cancels in the ratio."""
    S, R = prob.lam.shape[-1], len(prob.rates)
    P = transition_matrices(prob.V, prob.Vinv, prob.lam, prob.rates, prob.b)
    Q = rate_matrix(prob.V, prob.Vinv, prob.lam)
    dP = np.asarray(prob.rates)[None, :, None, None] * np.matmul(Q, P)
    kids, post, pre = tree_structure(prob.parent)
    n = len(kids)
    N = (n + 1) // 2
    C = prob.codes.shape[1]

    def store(x):
        mx = x.max(axis=(0, 2))
        _, e = np.frexp(mx)
        return np.ldexp(x, -e[None, :, None]).astype(np.float32).astype(np.float64)

    def mv(M, x):                    # (M x)_s = sum_t M_st x_t per (r, c)
        return x @ np.swapaxes(M, -1, -2)

    p = [np.broadcast_to(tip_partials(prob.codes[v], S), (R, C, S)) if v < N else None for v in range(n)]
    for k in post:
        if k >= N:
            i, j = kids[k]
            p[k] = store(mv(P[i], p[i]) * mv(P[j], p[j]))
    q = [None] * n
    q[n - 1] = np.broadcast_to(prob.pi, (R, C, S)).astype(np.float64)
    w = np.asarray(prob.weights)
    grad = np.zeros(n - 1)
    for k in pre:
        for x in kids[k]:
            xs = [c for c in kids[k] if c != x][0]
            u = q[k] * mv(P[xs], p[xs])
            num = np.einsum("r,rcs,rcs->c", w, u, mv(dP[x], p[x]))
            den = np.einsum("r,rcs,rcs->c", w, u, mv(P[x], p[x]))
            grad[x] = np.sum(prob.pattern_weights * num / den)
            if kids[x]:
                q[x] = store(u @ P[x])
    return grad


def _caterpillar(N, C, mean_b, seed):
    rng = np.random.default_rng(seed)
    pi = np.array([0.2, 0.3, 0.1, 0.4])
    Q = synth.hky_model(3.0, pi)
    rates, w = synth.discrete_gamma(0.8, 4)
    V, Vinv, lam = synth.eigensystem(Q, pi)
    parent = synth.caterpillar_topology(N)
    return synth.Problem(parent=parent, b=rng.exponential(mean_b, 2 * N - 2), V=V, Vinv=Vinv, lam=lam,
                         pi=pi, rates=rates, weights=w, codes=rng.integers(0, 4, (N, C)).astype(np.int32),
                         pattern_weights=np.ones(C), Q=Q)


def _scaled_err(prob):
    ref = oracle.evaluate_problem(prob)
    bar = np.maximum(np.abs(ref["grad"]), 1e-2 * ref["absgrad"])
    return float(np.max(np.abs(_storage_rounded_gradient(prob) - ref["grad"]) / bar))


def test_float32_storage_alone_reaches_the_bar_on_saturated_trees():
    sat_prob = _caterpillar(1000, 48, 1.0, 30)
    calm_prob = synth.config_problem("hky1000", seed=0, n_patterns=200)
    e_sat, e_calm = _scaled_err(sat_prob), _scaled_err(calm_prob)
    s_sat, s_calm = _saturation(sat_prob), _saturation(calm_prob)
    print(f"storage-rounding error: saturated {e_sat:.2e} (statistic {s_sat:.2f}); "
          f"1000-taxon HKY {e_calm:.2e} (statistic {s_calm:.2f})")
    # beyond the 1e-4 bar from storage rounding alone; the calm tree an
    # order of magnitude inside it
    assert e_sat > 1e-4 and e_calm < 1e-5
    assert s_sat > B_GUARD > s_calm


B_GUARD = 1.5
