"""Parity of the MFMA kernels for state counts other than 4 (amino acids,
codons, and small generic spaces) with the FP64 oracle, through the C ABI.

Bars as for 4 states: FP64 logL 1e-12 relative and gradients 1e-9 (scaled
rule); FP32-with-rescaling logL 1e-6 and gradients 1e-4.
"""
import numpy as np
import pytest

import oracle
from paper_2303_04390_amd import binding as B
from paper_2303_04390_amd import synth
from tests.parity import check

pytestmark = pytest.mark.gpu

TOL = {B.PHG_FP64: (1e-12, 1e-9), B.PHG_FP32_SCALED: (1e-6, 1e-4)}
NAME = {B.PHG_FP64: "fp64", B.PHG_FP32_SCALED: "fp32"}


def compare(name, prob, prec, ref=None, tol=None):
    print(f"[case] {name} {NAME[prec]} N={prob.n_tips} C={prob.n_patterns} S={prob.n_states} "
          f"R={prob.n_categories}", flush=True)
    ref = ref if ref is not None else oracle.evaluate_problem(prob)
    with B.Context.for_problem(prob, prec) as ctx:
        logl, grad = ctx.gradient()
    check(f"{name}/{NAME[prec]}", logl, grad, ref, *(tol or TOL[prec]))
    return ref


def generic_problem(N, S, C, seed, R=4, ambiguous=0.05, mean_b=0.1):
    rng = np.random.default_rng(seed)
    parent = synth.yule_topology(N, rng)
    b = rng.exponential(mean_b, 2 * N - 2)
    pi = rng.dirichlet([2.0] * S)
    pi = np.maximum(pi, 1e-3)
    pi /= pi.sum()
    Q = synth.gtr_model(rng.gamma(1.0, 1.0, S * (S - 1) // 2), pi)
    rates, w = synth.discrete_gamma(0.6, R)
    if R > 1:
        w = rng.dirichlet([3.0] * R)
    return synth.make_problem(parent, b, Q, pi, rates, w, C, rng,
                              pattern_weights=1.0 + rng.poisson(2.0, C), ambiguous_fraction=ambiguous)


@pytest.fixture(scope="module")
def aa500():
    prob = synth.config_problem("aa500", seed=0)
    return prob, oracle.evaluate_problem(prob)


@pytest.fixture(scope="module")
def codon128():
    prob = synth.config_problem("codon128", seed=0)
    return prob, oracle.evaluate_problem(prob)


@pytest.mark.parametrize("prec", [B.PHG_FP32_SCALED, B.PHG_FP64])
def test_aa500_full(aa500, prec):
    compare("aa500", aa500[0], prec, aa500[1])


@pytest.mark.parametrize("prec", [B.PHG_FP32_SCALED, B.PHG_FP64])
def test_codon128_full(codon128, prec):
    compare("codon128", codon128[0], prec, codon128[1])


@pytest.mark.parametrize("S,N,C", [(20, 9, 1), (20, 9, 37), (20, 9, 100), (61, 6, 33), (61, 6, 70),
                                   (2, 12, 50), (3, 12, 50), (5, 12, 50), (16, 12, 50), (17, 12, 50),
                                   (21, 10, 70), (24, 9, 130), (25, 8, 65), (32, 7, 129),
                                   (33, 8, 50), (40, 7, 31), (48, 9, 97), (49, 7, 65), (64, 6, 40)])
def test_state_counts_and_ragged_tiles(S, N, C):
    prob = generic_problem(N, S, C, seed=S * 100 + C)
    ref = oracle.evaluate_problem(prob)
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        compare(f"S{S}-N{N}-C{C}", prob, prec, ref)


@pytest.mark.parametrize("R", [1, 2, 3, 8, 16])
def test_categories_generic(R):
    prob = generic_problem(10, 20, 80, seed=R, R=R)
    ref = oracle.evaluate_problem(prob)
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        compare(f"S20-R{R}", prob, prec, ref)


def test_four_states_sixteen_categories_use_generic_kernels():
    prob = synth.config_problem("hky16", seed=9, n_patterns=150)
    rng = np.random.default_rng(4)
    rates, _ = synth.discrete_gamma(0.5, 16)
    prob.rates, prob.weights = rates, rng.dirichlet([2.0] * 16)
    ref = oracle.evaluate_problem(prob)
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        compare("S4-R16", prob, prec, ref)


def test_codon_deep_caterpillar_rescaling():
    """61 states on a 300-deep caterpillar with random codons: site
    likelihoods far below the FP64 range, so only rescaling keeps them.

    The likelihood of random codons rests on tiny multi-substitution entries
    of P(t) (down to 1e-31).  Built from the 61-state eigensystem, those
    entries carry an absolute error of ~5e-15 (relative up to 1e-3), and two
    FP64 evaluations of the same formula in different summation orders (GPU
    vs oracle) legitimately differ: replacing the eigen route by scipy's expm
    moves this case's logL by 5e-9 relative.  The FP64 bar here is therefore
    1e-9 (logL) and 1e-6 (gradients); FP32 keeps the standard bar."""
    N, C = 300, 40
    rng = np.random.default_rng(5)
    parent = synth.caterpillar_topology(N)
    b = rng.exponential(0.1, 2 * N - 2)
    pos = np.stack([rng.dirichlet([10.0] * 4) for _ in range(3)])
    Q, pi = synth.gy94_model(0.3, 2.0, pos)
    rates, w = synth.discrete_gamma(0.5, 4)
    V, Vinv, lam = synth.eigensystem(Q, pi)
    prob = synth.Problem(parent=parent, b=b, V=V, Vinv=Vinv, lam=lam, pi=pi, rates=rates, weights=w,
                         codes=rng.integers(0, 61, (N, C)).astype(np.int32), pattern_weights=np.ones(C),
                         Q=Q)
    ref = oracle.evaluate_problem(prob)
    assert np.max(ref["site_ll"]) < -800
    compare("codon-caterpillar300", prob, B.PHG_FP64, ref, tol=(1e-9, 1e-6))
    compare("codon-caterpillar300", prob, B.PHG_FP32_SCALED, ref)


def test_generic_repeatable_and_async(codon128):
    import torch
    prob, ref = codon128
    print("[case] codon128 repeatability + async", flush=True)
    with B.Context.for_problem(prob, B.PHG_FP32_SCALED) as ctx:
        l1, g1 = ctx.gradient()
        l2, g2 = ctx.gradient()
        assert l1 == l2 and np.array_equal(g1, g2)
        E = 2 * prob.n_tips - 2
        out = torch.full((1 + E,), float("nan"), dtype=torch.float64, device="cuda:0")
        stream = torch.cuda.Stream()
        B.phg_bind_stream(ctx.handle, stream.cuda_stream)
        B.phg_gradient_async(ctx.handle, out.data_ptr(), out.data_ptr() + 8)
        stream.synchronize()
        res = out.cpu().numpy()
        assert res[0] == l1 and np.array_equal(res[1:], g1)


@pytest.mark.parametrize("S,N,C,R", [(65, 10, 37, 2), (122, 12, 40, 4), (128, 8, 16, 1), (129, 8, 33, 3),
                                     (200, 6, 20, 2), (255, 6, 17, 2), (256, 7, 23, 2), (256, 12, 40, 4)])
def test_large_state_spaces(S, N, C, R):
    """65..256 states (Markov-modulated and phylogeographic state spaces) on
    the large-state MFMA kernels, ragged 16-pattern tiles; 256 states take
    16-bit tip codes (code 256 = fully ambiguous)."""
    prob = generic_problem(N, S, C, seed=S + C, R=R, mean_b=0.05)
    ref = oracle.evaluate_problem(prob)
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        compare(f"S{S}-N{N}-C{C}-R{R}", prob, prec, ref)


@pytest.mark.parametrize("which", ["s122", "s240"])
def test_bench_shapes_large_states(which):
    """The 128-taxon 122- and 240-state workloads of the benchmark, at their
    full size (2000 and 1000 patterns), both precisions."""
    prob = synth.config_problem(which, seed=0)
    ref = oracle.evaluate_problem(prob)
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        compare(which, prob, prec, ref)


def _table_bytes_per_branch(S, R, prec):
    """The unit the table budget is counted in: P, dP and their backward
    copies for one branch.  Vector-ALU kernels (phg_kernel_family_of):
    [SP][SP] forward and [SP + 1][SP] backward tables, SP
    the state count padded to 20, 24 or 32.  MFMA kernels: gl_mat_rows rows
    of the operand-order row length, backward copies one row more."""
    fp32 = prec == B.PHG_FP32_SCALED
    tsz = 4 if fp32 else 8
    if B.phg_kernel_family_of(S, R, prec) == B.PHG_KERNELS_VECTOR_ALU:
        SP = 20 if S <= 20 else (24 if S <= 24 else 32)
        return R * (2 * SP * SP + 2 * (SP + 1) * SP) * tsz
    G = 2 if S <= 32 else 4
    row = 4 * (((S + 3) // 4 + G - 1) // G * G)
    rows = (S + 15) // 16 * 16 if S <= 64 else (S + 63) // 64 * 64
    return R * (2 * rows + 2 * (rows + 1)) * row * tsz


@pytest.mark.parametrize("S,N,C,R", [(20, 30, 70, 2), (20, 30, 70, 3), (61, 12, 40, 2), (256, 10, 20, 2)])
def test_per_chunk_tables_match_full_tables(S, N, C, R):
    """Under a small table budget the context holds a pool of branch tables
    and rebuilds them per launch chunk; its results are bitwise those of the
    full tables, and both meet the oracle bar."""
    prob = generic_problem(N, S, C, seed=S + 7, R=R, mean_b=0.05)
    ref = oracle.evaluate_problem(prob)
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        print(f"[case] per-chunk tables S={S} N={N} C={C} R={R} {NAME[prec]}", flush=True)
        with B.Context.for_problem(prob, prec) as full:
            assert B.phg_table_slots(full.handle) == 0
            lf, gf = full.gradient()
        check(f"S{S}-full/{NAME[prec]}", lf, gf, ref, *TOL[prec])
        per = _table_bytes_per_branch(S, prob.n_categories, prec)
        for budget, slots in ((1, 2), (7 * per, 6)):
            ctx = B.Context(prob.n_tips, prob.n_patterns, S, prob.n_categories, prec)
            try:
                B.phg_set_table_budget(ctx.handle, budget)
                ctx.set_problem(prob)
                assert B.phg_table_slots(ctx.handle) == slots
                lc, gc = ctx.gradient()
                assert B.phg_table_slots(ctx.handle) == slots
                assert ctx.log_likelihood() == lc
                n_post, n_pre, launches = B.phg_schedule_info(ctx.handle)
            finally:
                ctx.close()
            assert lc == lf and np.array_equal(gc, gf), (budget, np.max(np.abs(gc - gf)))
            # a P(t) launch before every chunk of every level
            assert launches > n_post + n_pre + 2
            if slots == 2:
                assert launches == 4 * (N - 1) + 1
