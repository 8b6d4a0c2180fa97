"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64 path: logL within 1e-12 relative, gradients within 1e-9 (scaled rule of
tests/parity.py).  FP32-with-rescaling path: logL within 1e-6 relative,
gradients within 1e-4 (same rule) -- the accuracy targets of the
1000-taxon HKY+Gamma4 workload.
"""
import numpy as np
import pytest

import oracle
from paper_2303_04390_amd import binding as B
from paper_2303_04390_amd import synth
from tests.parity import check

pytestmark = pytest.mark.gpu

TOL = {B.PHG_FP64: (1e-12, 1e-9), B.PHG_FP32_SCALED: (1e-6, 1e-4)}
PREC_NAME = {B.PHG_FP64: "fp64", B.PHG_FP32_SCALED: "fp32"}


SCHED_NAME = {B.PHG_SCHEDULE_AUTO: "auto", B.PHG_SCHEDULE_LEVELS: "levels",
              B.PHG_SCHEDULE_BLOCKS: "blocks"}


def gpu_eval(prob, prec, schedule=B.PHG_SCHEDULE_AUTO):
    with B.Context.for_problem(prob, prec, schedule=schedule) as ctx:
        return ctx.gradient()


def compare(name, prob, prec, ref=None, schedule=B.PHG_SCHEDULE_AUTO):
    print(f"[case] {name} {PREC_NAME[prec]} {SCHED_NAME[schedule]} N={prob.n_tips} C={prob.n_patterns} "
          f"S={prob.n_states} R={prob.n_categories}", flush=True)
    ref = ref if ref is not None else oracle.evaluate_problem(prob)
    logl, grad = gpu_eval(prob, prec, schedule)
    check(f"{name}/{PREC_NAME[prec]}/{SCHED_NAME[schedule]}", logl, grad, ref, *TOL[prec])
    return logl, grad, ref


@pytest.fixture(scope="module")
def hky16():
    prob = synth.config_problem("hky16", seed=0)
    return prob, oracle.evaluate_problem(prob)


@pytest.fixture(scope="module")
def hky1000():
    prob = synth.config_problem("hky1000", seed=0)
    return prob, oracle.evaluate_problem(prob)


@pytest.mark.parametrize("prec", [B.PHG_FP64, B.PHG_FP32_SCALED])
def test_hky16(hky16, prec):
    compare("hky16", hky16[0], prec, hky16[1])


@pytest.mark.parametrize("prec", [B.PHG_FP32_SCALED, B.PHG_FP64])
def test_hky1000_full(hky1000, prec):
    compare("hky1000", hky1000[0], prec, hky1000[1])


@pytest.mark.parametrize("C", [1, 63, 64, 65, 130])
def test_ragged_pattern_counts(C):
    prob = synth.config_problem("hky1000", seed=3, n_tips=12, n_patterns=C)
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        compare(f"ragged-C{C}", prob, prec)


@pytest.mark.parametrize("R", [1, 2, 8])
def test_category_counts(R):
    rng = np.random.default_rng(R)
    parent = synth.yule_topology(20, rng)
    b = rng.exponential(0.1, 38)
    pi = rng.dirichlet([5.0] * 4)
    Q = synth.hky_model(3.0, pi)
    rates, w = synth.discrete_gamma(0.6, R)
    if R > 1:
        w = rng.dirichlet([3.0] * R)
    prob = synth.make_problem(parent, b, Q, pi, rates, w, 200, rng,
                              pattern_weights=1.0 + rng.poisson(2.0, 200), ambiguous_fraction=0.1)
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        compare(f"R{R}", prob, prec)


def test_two_tips():
    prob = synth.config_problem("hky16", seed=5, n_tips=2, n_patterns=100)
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        compare("N2", prob, prec)


def test_zero_branches_and_ambiguous_columns():
    prob = synth.config_problem("hky16", seed=6, n_patterns=200)
    prob.b[[2, 7, 11]] = 0.0
    prob.codes[:, 17] = 4                     # one fully ambiguous column
    prob.codes[3, :50] = 4                    # an ambiguous stretch on one tip
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        _, grad, ref = compare("zero-b+ambig", prob, prec)


def test_nonstationary_root_and_unit_weights():
    prob = synth.config_problem("hky16", seed=7, n_patterns=300)
    prob.pi = np.array([0.7, 0.1, 0.1, 0.1])
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        compare("nonstationary-pi", prob, prec)


def _caterpillar(N, C, mean_b, seed):
    rng = np.random.default_rng(seed)
    parent = synth.caterpillar_topology(N)
    b = rng.exponential(mean_b, 2 * N - 2)
    pi = np.array([0.2, 0.3, 0.1, 0.4])
    Q = synth.hky_model(3.0, pi)
    rates, w = synth.discrete_gamma(0.8, 4)
    V, Vinv, lam = synth.eigensystem(Q, pi)
    return synth.Problem(parent=parent, b=b, V=V, Vinv=Vinv, lam=lam, pi=pi, rates=rates,
                         weights=w, codes=rng.integers(0, 4, (N, C)).astype(np.int32),
                         pattern_weights=np.ones(C), Q=Q)


def test_deep_caterpillar_needs_rescaling():
    """999 levels, random tip states: site likelihoods far below FP64's
    range, so only the power-of-two rescaling keeps them."""
    prob = _caterpillar(1000, 96, 0.1, 12)
    ref = oracle.evaluate_problem(prob)
    assert np.max(ref["site_ll"]) < -800
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        compare("caterpillar1000-b0.1", prob, prec, ref)


@pytest.mark.fp32_routed
def test_saturated_branches_fp32_guard():
    """Branches ~Exp(1) on a 1000-deep caterpillar.  Nearly stationary
    pre-order vectors meet nearly flat sibling vectors, and one float32
    rounding of the stored partials already moves some derivatives by ~1e-4
    of themselves, so no float32-partials arithmetic holds the bar here.  The
    FP32 precision guard sees the saturation (statistic far above its 1.5
    threshold) and evaluates in FP64: the FP32 request meets the FP32 bar."""
    prob = _caterpillar(1000, 96, 1.0, 11)
    ref = oracle.evaluate_problem(prob)
    compare("caterpillar1000-b1", prob, B.PHG_FP64, ref)
    print("[case] caterpillar1000-b1 fp32 guarded", flush=True)
    with B.Context.for_problem(prob, B.PHG_FP32_SCALED) as ctx:
        sat = B.phg_fp32_saturation(ctx.handle)
        assert sat > 5.0, sat
        logl, grad = ctx.gradient()
        assert B.phg_last_precision(ctx.handle) == B.PHG_FP64
        assert B.phg_log_likelihood(ctx.handle) == logl
    check("caterpillar1000-b1/fp32-guarded", logl, grad, ref, *TOL[B.PHG_FP32_SCALED])


def test_saturated_branches_fp32_unguarded_limit():
    """The same tree with the guard off runs the float32 kernels.  This
    characterises the conditioning limit the guard exists for (measured
    ~1.4e-3 scaled error, beyond the 1e-4 bar): log P(Y) still meets 1e-6 and
    the gradient stays within 1e-2."""
    prob = _caterpillar(1000, 96, 1.0, 11)
    ref = oracle.evaluate_problem(prob)
    print("[case] caterpillar1000-b1 fp32 unguarded", flush=True)
    with B.Context.for_problem(prob, B.PHG_FP32_SCALED) as ctx:
        B.phg_set_fp32_guard(ctx.handle, 0.0)
        logl, grad = ctx.gradient()
        assert B.phg_last_precision(ctx.handle) == B.PHG_FP32_SCALED
    check("caterpillar1000-b1/fp32-unguarded", logl, grad, ref, 1e-6, 1e-2)


@pytest.mark.parametrize("schedule", [B.PHG_SCHEDULE_AUTO, B.PHG_SCHEDULE_LEVELS])
@pytest.mark.parametrize("prec", [B.PHG_FP64, B.PHG_FP32_SCALED])
def test_log_likelihood_only_path(hky1000, prec, schedule):
    """phg_log_likelihood runs P(t), the post-order pass and the final sum
    only; its value is bitwise the log-likelihood of the full evaluation."""
    prob, ref = hky1000
    print(f"[case] logL-only {PREC_NAME[prec]} {SCHED_NAME[schedule]}", flush=True)
    with B.Context.for_problem(prob, prec, schedule=schedule) as ctx:
        ll_only = ctx.log_likelihood()
        logl, grad = ctx.gradient()
        assert ll_only == logl
        assert ctx.log_likelihood() == logl
    assert abs(ll_only - ref["logl"]) / abs(ref["logl"]) <= TOL[prec][0]


def test_zero_site_likelihood_is_numeric_error():
    pi = np.full(4, 0.25)
    Q = synth.hky_model(2.0, pi)
    V, Vinv, lam = synth.eigensystem(Q, pi)
    prob = synth.Problem(parent=np.array([2, 2, -1], np.int32), b=np.zeros(2), V=V, Vinv=Vinv,
                         lam=lam, pi=pi, rates=np.ones(1), weights=np.ones(1),
                         codes=np.array([[0, 1], [1, 1]], np.int32), pattern_weights=np.ones(2), Q=Q)
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        print(f"[case] zero-likelihood {PREC_NAME[prec]}", flush=True)
        with B.Context.for_problem(prob, prec) as ctx:
            with pytest.raises(B.PhgError) as e:
                ctx.gradient()
            assert e.value.status == B.PHG_ERR_NUMERIC
            # the same pattern with weight 0 is ignored
            B.phg_set_pattern_weights(ctx.handle, np.array([0.0, 1.0]))
            logl, grad = ctx.gradient()
            assert np.isfinite(logl) and np.all(np.isfinite(grad))


def test_repeatable_and_branch_updates(hky16):
    prob, _ = hky16
    print("[case] repeatability + branch updates", flush=True)
    with B.Context.for_problem(prob, B.PHG_FP32_SCALED) as ctx:
        l1, g1 = ctx.gradient()
        l2, g2 = ctx.gradient()
        assert l1 == l2 and np.array_equal(g1, g2)
        rng = np.random.default_rng(1)
        for step in range(3):
            b = prob.b * np.exp(rng.normal(0, 0.05, prob.b.shape))
            B.phg_set_branch_lengths(ctx.handle, b)
            logl, grad = ctx.gradient()
            p2 = synth.Problem(**{**prob.__dict__, "b": b})
            ref = oracle.evaluate_problem(p2)
            check(f"hmc-step{step}", logl, grad, ref, *TOL[B.PHG_FP32_SCALED])


def test_async_with_torch_memory_and_stream(hky16):
    import torch
    prob, ref = hky16
    print("[case] async + bound workspace/stream", flush=True)
    dev = torch.device("cuda:0")
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        nbytes = B.phg_workspace_size(prob.n_tips, prob.n_patterns, 4, 4, prec)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = (ws.data_ptr() + 255) // 256 * 256
        out = torch.full((1 + 30,), float("nan"), dtype=torch.float64, device=dev)
        stream = torch.cuda.Stream(device=dev)
        h = B.phg_create(prob.n_tips, prob.n_patterns, 4, 4, prec, 0)
        try:
            B.phg_bind_workspace(h, base, nbytes)
            B.phg_bind_stream(h, stream.cuda_stream)
            B.set_problem(h, prob)
            B.phg_gradient_async(h, out.data_ptr(), out.data_ptr() + 8)
            stream.synchronize()
            res = out.cpu().numpy()
            logl_sync, g_sync = B.phg_gradient(h, 30)
            assert res[0] == logl_sync and np.array_equal(res[1:], g_sync)
            check(f"async/{PREC_NAME[prec]}", res[0], res[1:], ref, *TOL[prec])
        finally:
            B.phg_destroy(h)
        del ws


@pytest.mark.parametrize("prec", [B.PHG_FP32_SCALED, B.PHG_FP64])
def test_level_schedule_hky1000(hky1000, prec):
    compare("hky1000", hky1000[0], prec, hky1000[1], schedule=B.PHG_SCHEDULE_LEVELS)


@pytest.mark.parametrize("N,C,seed", [(2, 70, 1), (3, 64, 2), (7, 130, 3), (40, 65, 4), (300, 200, 5)])
def test_blocked_and_level_schedules_agree(N, C, seed):
    """Small and odd trees (down to two tips, block shapes with tips at every
    heap position) under both schedules, both precisions."""
    prob = synth.config_problem("hky1000", seed=seed, n_tips=N, n_patterns=C)
    ref = oracle.evaluate_problem(prob)
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        lb, gb, _ = compare(f"sched-N{N}", prob, prec, ref, schedule=B.PHG_SCHEDULE_BLOCKS)
        ll, gl, _ = compare(f"sched-N{N}", prob, prec, ref, schedule=B.PHG_SCHEDULE_LEVELS)
        print(f"[schedules] N={N} {PREC_NAME[prec]} bitwise-equal={lb == ll and np.array_equal(gb, gl)}",
              flush=True)


def test_blocked_caterpillar_levels():
    """A caterpillar has one block per three levels and a tip at every
    second heap position: stresses frontier and in-block tip handling."""
    N, C = 200, 64
    rng = np.random.default_rng(13)
    parent = synth.caterpillar_topology(N)
    b = rng.exponential(0.1, 2 * N - 2)
    pi = np.array([0.2, 0.3, 0.1, 0.4])
    Q = synth.hky_model(3.0, pi)
    rates, w = synth.discrete_gamma(0.8, 4)
    prob = synth.make_problem(parent, b, Q, pi, rates, w, C, rng, ambiguous_fraction=0.1)
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        compare("caterpillar200", prob, prec, schedule=B.PHG_SCHEDULE_BLOCKS)


@pytest.fixture(scope="module")
def hky20k():
    prob = synth.config_problem("hky1000", seed=7, n_tips=20000, n_patterns=130)
    return prob, oracle.evaluate_problem(prob)


@pytest.mark.parametrize("prec,schedule", [(B.PHG_FP32_SCALED, B.PHG_SCHEDULE_BLOCKS),
                                           (B.PHG_FP32_SCALED, B.PHG_SCHEDULE_LEVELS),
                                           (B.PHG_FP64, B.PHG_SCHEDULE_AUTO)])
def test_large_tree(hky20k, prec, schedule):
    """20,000 taxa (39,998 branches, the paper's largest branch count) with a
    ragged pattern count: many block levels and node levels, wide launches."""
    compare("hky20k", hky20k[0], prec, hky20k[1], schedule=schedule)


def test_large_tree_twenty_states():
    from tests.test_gpu_parity_states import generic_problem
    prob = generic_problem(5000, 20, 70, seed=3, R=2)
    ref = oracle.evaluate_problem(prob)
    for prec in (B.PHG_FP32_SCALED, B.PHG_FP64):
        compare("aa5000", prob, prec, ref)
