"""The work-queue traversals (PHG_SCHEDULE_QUEUE) through the C ABI.

4 states (FP32): the blocked schedule's arithmetic in one launch per pass
(or one for both), items waiting on per-(block, tile) completion marks
instead of level launches.  17..256 states on the vector-ALU and MFMA
kernels: the level schedule's records as items, one launch per pass.  Results must equal the level-launched schedule's bit for bit --
which the oracle parity tests hold to their bars -- on every tree shape,
category count, launch mode, repeated evaluations (the marks' epochs),
library-owned graph replays and the log-likelihood-only path.  Some cases
are also checked against the oracle directly.
"""
import numpy as np
import pytest

import oracle
from paper_2303_04390_amd import binding as B
from paper_2303_04390_amd import synth
from tests.parity import check

pytestmark = pytest.mark.gpu

F32 = B.PHG_FP32_SCALED


def _run(prob, schedule, launches=0, graphs=True, repeats=2, prec=F32):
    """(logL, gradient) of `repeats` synchronous evaluations and a
    log-likelihood-only one."""
    B.phg_set_tuning(4, 0, F32, B.PHG_TUNE_QUEUE_LAUNCHES, launches)
    try:
        with B.Context.for_problem(prob, prec, schedule=schedule) as ctx:
            B.phg_set_fp32_guard(ctx.handle, 0.0)
            B.phg_set_graphs(ctx.handle, graphs)
            got = B.phg_get_schedule(ctx.handle)
            assert got == schedule, (got, schedule)
            outs = [ctx.gradient() for _ in range(repeats)]
            ll_only = ctx.log_likelihood()
    finally:
        B.phg_set_tuning(4, 0, F32, B.PHG_TUNE_QUEUE_LAUNCHES, 0)
    return outs, ll_only


def _same(name, prob, prec=F32):
    print(f"[case] queue {name} N={prob.n_tips} C={prob.n_patterns} S={prob.n_states} R={prob.n_categories} "
          f"{'fp32' if prec == F32 else 'fp64'}", flush=True)
    four = prob.n_states == 4
    ref_sched = B.PHG_SCHEDULE_BLOCKS if four else B.PHG_SCHEDULE_LEVELS
    (ref, *_), ref_ll = _run(prob, ref_sched, repeats=1, prec=prec)
    for launches in ((1, 2) if four else (0,)):
        for graphs in (True, False):
            outs, ll_only = _run(prob, B.PHG_SCHEDULE_QUEUE, launches, graphs, prec=prec)
            for logl, grad in outs:
                assert logl == ref[0], (name, launches, graphs, logl, ref[0])
                assert np.array_equal(grad, ref[1]), (name, launches, graphs)
            assert ll_only == ref_ll, (name, launches, graphs, ll_only, ref_ll)
    return ref


def _problem(N, C, R, seed, caterpillar=False, mean_b=0.05, S=4):
    rng = np.random.default_rng(seed)
    parent = synth.caterpillar_topology(N) if caterpillar else synth.yule_topology(N, rng)
    b = rng.exponential(mean_b, 2 * N - 2)
    pi = rng.dirichlet([5.0] * S)
    if S == 4:
        Q = synth.hky_model(3.0, pi)
    else:
        ex = np.triu(rng.gamma(1.0, 1.0, (S, S)), 1)
        Q = synth.reversible_q(ex + ex.T, pi)
    rates, w = synth.discrete_gamma(0.6, R)
    if R > 1:
        w = rng.dirichlet([3.0] * R)
    return synth.make_problem(parent, b, Q, pi, rates, w, C, rng,
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


# vector-ALU kernels: 17..20 states FP32 (DPP kernels), 24 and 32 states
# FP32, 20 and 24 states FP64; tip-tip nodes are folded on these shapes
@pytest.mark.parametrize("N,C,S,R,prec,seed", [(2, 70, 20, 4, F32, 21), (9, 64, 20, 4, F32, 22),
                                               (60, 130, 20, 1, F32, 23), (60, 130, 20, 8, F32, 24),
                                               (120, 65, 17, 4, F32, 25), (80, 100, 24, 2, F32, 26),
                                               (50, 70, 32, 4, F32, 27), (60, 130, 20, 4, B.PHG_FP64, 28),
                                               (40, 70, 24, 2, B.PHG_FP64, 29)])
def test_queue_vector_alu_equals_levels(N, C, S, R, prec, seed):
    _same(f"valu-N{N}-C{C}", _problem(N, C, R, seed, S=S, mean_b=0.1), prec)


def test_queue_vector_alu_caterpillar():
    # 149 post-order and pre-order levels of one node each
    _same("valu-caterpillar150", _problem(150, 70, 4, 30, caterpillar=True, mean_b=0.05, S=20))


def test_queue_vector_alu_against_oracle():
    prob = _problem(90, 200, 4, 32, S=20, mean_b=0.1)
    ref = _same("valu-N90-C200", prob)
    check("queue/valu-N90-C200", ref[0], ref[1], oracle.evaluate_problem(prob), 1e-6, 1e-4)


def test_queue_vector_alu_tip_vectors():
    # general tip vectors are inputs the items read as they are (no marks)
    prob = _problem(40, 70, 4, 31, S=20, mean_b=0.1)
    rng = np.random.default_rng(31)
    vec = rng.uniform(0.0, 1.0, (prob.n_patterns, 20))
    outs = []
    for schedule in (B.PHG_SCHEDULE_LEVELS, B.PHG_SCHEDULE_QUEUE):
        with B.Context.for_problem(prob, F32, schedule=schedule) as ctx:
            B.phg_set_fp32_guard(ctx.handle, 0.0)
            B.phg_set_tip_partials(ctx.handle, 3, vec)
            assert B.phg_get_schedule(ctx.handle) == schedule
            outs.append(ctx.gradient())
    assert outs[0][0] == outs[1][0] and np.array_equal(outs[0][1], outs[1][1])


# MFMA kernels (17..256 states outside the vector-ALU shapes): one and two
# row blocks, FP32 and FP64, folded tip-tip nodes above 32 states, R = 3
@pytest.mark.parametrize("N,C,S,R,prec,seed", [(9, 64, 61, 4, F32, 41), (70, 130, 61, 4, F32, 42),
                                               (70, 130, 61, 4, B.PHG_FP64, 43), (40, 90, 33, 3, F32, 44),
                                               (50, 70, 20, 3, F32, 45), (30, 40, 122, 2, F32, 46),
                                               (20, 33, 200, 2, B.PHG_FP64, 47), (2, 20, 61, 1, F32, 48)])
def test_queue_mfma_equals_levels(N, C, S, R, prec, seed):
    _same(f"mfma-N{N}-C{C}", _problem(N, C, R, seed, S=S, mean_b=0.1), prec)


def test_queue_mfma_caterpillar_and_oracle():
    _same("mfma-caterpillar80", _problem(80, 50, 2, 49, caterpillar=True, mean_b=0.05, S=61))
    prob = _problem(60, 100, 4, 50, S=61, mean_b=0.1)
    ref = _same("mfma-N60-C100", prob)
    check("queue/mfma-N60-C100", ref[0], ref[1], oracle.evaluate_problem(prob), 1e-6, 1e-4)


@pytest.mark.parametrize("S", [4, 20])
def test_queue_wait_bound_fault_path(S):
    # a work item that waits past the bound abandons the evaluation: the final
    # sums turn to NaN and the synchronous call reports PHG_ERR_NUMERIC; with
    # the default bound the next evaluation through the same context is exact
    # again (its P(t) launch clears the fault word).  A caterpillar makes every
    # item wait on the one before, so a 1 us bound is always exceeded; the
    # kernels exit normally either way.
    prob = _problem(300 if S == 4 else 120, 64, 4, 60, caterpillar=True, mean_b=0.02, S=S)
    (ref, *_), _ = _run(prob, B.PHG_SCHEDULE_BLOCKS if S == 4 else B.PHG_SCHEDULE_LEVELS, repeats=1)
    with B.Context.for_problem(prob, F32, schedule=B.PHG_SCHEDULE_QUEUE) as ctx:
        B.phg_set_fp32_guard(ctx.handle, 0.0)
        B.phg_set_graphs(ctx.handle, False)
        B.phg_set_tuning(S, 0, F32, B.PHG_TUNE_QUEUE_WAIT_US, 1)
        try:
            with pytest.raises(B.PhgError) as e:
                ctx.gradient()
            assert e.value.status == B.PHG_ERR_NUMERIC
        finally:
            B.phg_set_tuning(S, 0, F32, B.PHG_TUNE_QUEUE_WAIT_US, 0)
        logl, grad = ctx.gradient()
        assert logl == ref[0] and np.array_equal(grad, ref[1])
