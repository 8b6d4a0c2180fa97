"""The work-queue traversal (PHG_SCHEDULE_QUEUE) through the C ABI.

It runs the blocked schedule's arithmetic in one launch per pass (or one for
both), items waiting on per-(block, tile) completion marks instead of level
launches, so its results must equal the level-launched blocked schedule's
bit for bit -- which the oracle parity tests hold to the FP32 bar -- on every
tree shape, category count, both launch modes, repeated evaluations (the
marks' epochs), library-owned graph replays and the log-likelihood-only
path.  One case is also checked against the oracle directly.
"""
import numpy as np
import pytest

import oracle
from paper_2303_04390_amd import binding as B
from paper_2303_04390_amd import synth
from tests.parity import check

pytestmark = pytest.mark.gpu

F32 = B.PHG_FP32_SCALED


def _run(prob, schedule, launches=0, graphs=True, repeats=2):
    """(logL, gradient) of `repeats` synchronous evaluations and a
    log-likelihood-only one."""
    B.phg_set_tuning(4, 0, F32, B.PHG_TUNE_QUEUE_LAUNCHES, launches)
    try:
        with B.Context.for_problem(prob, F32, schedule=schedule) as ctx:
            B.phg_set_fp32_guard(ctx.handle, 0.0)
            B.phg_set_graphs(ctx.handle, graphs)
            got = B.phg_get_schedule(ctx.handle)
            assert got == schedule, (got, schedule)
            outs = [ctx.gradient() for _ in range(repeats)]
            ll_only = ctx.log_likelihood()
    finally:
        B.phg_set_tuning(4, 0, F32, B.PHG_TUNE_QUEUE_LAUNCHES, 0)
    return outs, ll_only


def _same(name, prob):
    print(f"[case] queue {name} N={prob.n_tips} C={prob.n_patterns} R={prob.n_categories}", flush=True)
    (ref, *_), ref_ll = _run(prob, B.PHG_SCHEDULE_BLOCKS, repeats=1)
    for launches in (1, 2):
        for graphs in (True, False):
            outs, ll_only = _run(prob, B.PHG_SCHEDULE_QUEUE, launches, graphs)
            for logl, grad in outs:
                assert logl == ref[0], (name, launches, graphs, logl, ref[0])
                assert np.array_equal(grad, ref[1]), (name, launches, graphs)
            assert ll_only == ref_ll, (name, launches, graphs, ll_only, ref_ll)
    return ref


def _problem(N, C, R, seed, caterpillar=False, mean_b=0.05):
    rng = np.random.default_rng(seed)
    parent = synth.caterpillar_topology(N) if caterpillar else synth.yule_topology(N, rng)
    b = rng.exponential(mean_b, 2 * N - 2)
    pi = rng.dirichlet([5.0] * 4)
    rates, w = synth.discrete_gamma(0.6, R)
    if R > 1:
        w = rng.dirichlet([3.0] * R)
    return synth.make_problem(parent, b, synth.hky_model(3.0, pi), pi, rates, w, C, rng,
                              pattern_weights=1.0 + rng.poisson(2.0, C), ambiguous_fraction=0.05)


@pytest.mark.parametrize("N,C,R,seed", [(2, 70, 4, 1), (3, 1, 4, 2), (9, 64, 4, 3), (40, 130, 1, 4),
                                        (40, 130, 2, 5), (150, 200, 8, 6), (300, 65, 4, 7)])
def test_queue_equals_blocks(N, C, R, seed):
    _same(f"yule-N{N}-C{C}-R{R}", _problem(N, C, R, seed))


def test_queue_deep_caterpillar():
    # 400 levels: every block is a chain, each item waits on the one before
    _same("caterpillar400", _problem(400, 130, 4, 8, caterpillar=True, mean_b=0.02))


def test_queue_hky1000_against_oracle():
    prob = synth.config_problem("hky1000", seed=0, n_patterns=2000)
    ref = _same("hky1000-C2000", prob)
    check("queue/hky1000-C2000", ref[0], ref[1], oracle.evaluate_problem(prob), 1e-6, 1e-4)


def test_queue_branch_updates_between_evaluations():
    # the marks of one evaluation must not satisfy the next: new branch
    # lengths through the same context give the blocked schedule's results
    prob = synth.config_problem("hky1000", seed=11, n_tips=200, n_patterns=300)
    rng = np.random.default_rng(11)
    with B.Context.for_problem(prob, F32, schedule=B.PHG_SCHEDULE_QUEUE) as q, \
            B.Context.for_problem(prob, F32, schedule=B.PHG_SCHEDULE_BLOCKS) as b:
        for ctx in (q, b):
            B.phg_set_fp32_guard(ctx.handle, 0.0)
        for _ in range(4):
            bl = prob.b * np.exp(rng.normal(0.0, 0.3, prob.b.shape))
            B.phg_set_branch_lengths(q.handle, bl)
            B.phg_set_branch_lengths(b.handle, bl)
            lq, gq = q.gradient()
            lb, gb = b.gradient()
            assert lq == lb and np.array_equal(gq, gb)
