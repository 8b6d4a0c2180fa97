"""One substitution model per rate category on the GPU (phg_set_category_eigen)
against the oracle, at the standard bars, for 4 states (both schedules, both
precisions) and for 20 states (MFMA and vector-ALU kernels)."""
import numpy as np
import pytest

import oracle
from paper_2303_04390_amd import binding as B
from paper_2303_04390_amd import synth
from tests.parity import check

pytestmark = pytest.mark.gpu

TOL = {B.PHG_FP64: (1e-12, 1e-9), B.PHG_FP32_SCALED: (1e-6, 1e-4)}


def cat_problem(N, C, S, R, seed, mean_b=0.05):
    rng = np.random.default_rng(seed)
    parent = synth.yule_topology(N, rng)
    b = synth.exponential_branch_lengths(N, mean_b, rng)
    Qs, V, Vinv, lam = synth.category_models(S, R, rng)
    pi = rng.dirichlet([3.0] * S)
    rates, _ = synth.discrete_gamma(0.7, R)
    w = rng.dirichlet([3.0] * R)
    codes = rng.integers(0, S, (N, C))
    codes[rng.random((N, C)) < 0.05] = S
    return synth.Problem(parent=parent, b=b, V=V, Vinv=Vinv, lam=lam, pi=pi, rates=rates, weights=w,
                         codes=codes.astype(np.int32), pattern_weights=1.0 + rng.poisson(2.0, C), Q=Qs)


@pytest.mark.parametrize("prec", [B.PHG_FP32_SCALED, B.PHG_FP64])
@pytest.mark.parametrize("schedule", [B.PHG_SCHEDULE_AUTO, B.PHG_SCHEDULE_LEVELS])
def test_four_states_per_category_models(prec, schedule):
    prob = cat_problem(200, 1500, 4, 4, seed=1)
    ref = oracle.evaluate_problem(prob)
    print(f"[case] per-category S=4 prec={prec} schedule={schedule}", flush=True)
    with B.Context.for_problem(prob, prec, schedule=schedule) as ctx:
        logl, grad = ctx.gradient()
    check(f"cat-models-S4/{prec}/{schedule}", logl, grad, ref, *TOL[prec])


@pytest.mark.parametrize("R", [3, 4])     # MFMA kernels, vector-ALU kernels
@pytest.mark.parametrize("prec", [B.PHG_FP32_SCALED, B.PHG_FP64])
def test_twenty_states_per_category_models(prec, R):
    prob = cat_problem(40, 230, 20, R, seed=2)
    ref = oracle.evaluate_problem(prob)
    print(f"[case] per-category S=20 R={R} prec={prec}", flush=True)
    with B.Context.for_problem(prob, prec) as ctx:
        logl, grad = ctx.gradient()
    check(f"cat-models-S20-R{R}/{prec}", logl, grad, ref, *TOL[prec])


def test_identical_category_models_match_the_shared_model_bitwise():
    prob = synth.config_problem("hky16", seed=6, n_patterns=700)
    R = prob.n_categories
    stack = synth.Problem(**{**prob.__dict__, "V": np.stack([prob.V] * R),
                             "Vinv": np.stack([prob.Vinv] * R), "lam": np.stack([prob.lam] * R)})
    for prec in (B.PHG_FP32_SCALED, B.PHG_FP64):
        print(f"[case] identical categories prec={prec}", flush=True)
        with B.Context.for_problem(prob, prec) as ctx:
            l0, g0 = ctx.gradient()
        with B.Context.for_problem(stack, prec) as ctx:
            l1, g1 = ctx.gradient()
            # back to one shared model on the same context
            B.phg_set_eigen(ctx.handle, prob.V, prob.Vinv, prob.lam)
            l2, g2 = ctx.gradient()
        assert l0 == l1 and np.array_equal(g0, g1)
        assert l0 == l2 and np.array_equal(g0, g2)


@pytest.mark.parametrize("S,R", [(4, 24), (4, 64), (20, 32)])
def test_many_rate_categories(S, R):
    """More categories than the 4-state kernels hold (they run one category at
    a time on the MFMA kernels), with per-category models."""
    prob = cat_problem(24, 150, S, R, seed=R + S)
    ref = oracle.evaluate_problem(prob)
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        print(f"[case] S={S} R={R} prec={prec}", flush=True)
        with B.Context.for_problem(prob, prec) as ctx:
            logl, grad = ctx.gradient()
        check(f"many-categories-S{S}-R{R}/{prec}", logl, grad, ref, *TOL[prec])
