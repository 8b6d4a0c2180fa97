"""General tip partial vectors (phg_set_tip_partials) on the GPU, against the
oracle: every level-kernel family they run on (4 states; up to 16 states or
R > 8; 17..32 states on the vector ALUs; above 16 states on the MFMA kernels
with and without LDS-staged inputs), both precisions,
ragged tiles, cherries of two such tips."""
import numpy as np
import pytest

import oracle
from paper_2303_04390_amd import binding as B
from tests.parity import check
from tests.test_gpu_parity_states import NAME, TOL, compare, generic_problem
from tests.test_oracle_tip_vectors import code_vectors, random_vectors

pytestmark = pytest.mark.gpu


def with_vectors(prob, frac, seed):
    rng = np.random.default_rng(seed)
    N, C, S = prob.n_tips, prob.n_patterns, prob.n_states
    tips = [t for t in range(N) if rng.uniform() < frac]
    # both children of some cherry, so a node with two vector tips occurs
    for k in range(N, 2 * N - 1):
        kids = np.nonzero(prob.parent[:N] == k)[0]
        if len(kids) == 2:
            tips += [int(kids[0]), int(kids[1])]
            break
    prob.tip_vectors = {int(t): random_vectors(rng, C, S) for t in sorted(set(tips))}
    return prob


@pytest.mark.parametrize("S,N,C,R", [(4, 40, 150, 4), (4, 30, 70, 16), (8, 25, 90, 3), (20, 20, 80, 4),
                                     (20, 12, 50, 3), (28, 15, 70, 2), (61, 10, 45, 2), (122, 8, 33, 2)])
@pytest.mark.parametrize("prec", [B.PHG_FP32_SCALED, B.PHG_FP64])
def test_tip_vectors_match_oracle(S, N, C, R, prec):
    prob = with_vectors(generic_problem(N, S, C, seed=S * 7 + C, R=R, mean_b=0.1), 0.35, seed=S + N)
    compare(f"vectors S{S} N{N} C{C} R{R} ({len(prob.tip_vectors)} tips)", prob, prec)


@pytest.mark.parametrize("prec", [B.PHG_FP32_SCALED, B.PHG_FP64])
def test_code_vectors_on_levels_match_codes_on_blocks(prec):
    """One-hot / all-ones vectors for some tips (level kernels) give the
    codes-only result of the blocked kernels, and reverting restores it."""
    prob = generic_problem(60, 4, 200, seed=11, R=4, ambiguous=0.1)
    ref = oracle.evaluate_problem(prob)
    with B.Context.for_problem(prob, prec) as ctx:
        l0, g0 = ctx.gradient()
        for t in range(0, 60, 3):
            B.phg_set_tip_partials(ctx.handle, t, code_vectors(prob.codes[t], 4))
        assert B.phg_get_schedule(ctx.handle) == B.PHG_SCHEDULE_LEVELS
        l1, g1 = ctx.gradient()
        for t in range(0, 60, 3):
            B.phg_set_tip_partials(ctx.handle, t, None)
        l2, g2 = ctx.gradient()
    for name, (l, g) in (("codes", (l0, g0)), ("code vectors", (l1, g1)), ("reverted", (l2, g2))):
        check(f"{name}/{NAME[prec]}", l, g, ref, *TOL[prec])
    assert l2 == l0 and np.array_equal(g2, g0)
