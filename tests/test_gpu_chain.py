"""Chain rules on the device (node heights, branch rate scalars, branch-set
sums) against the oracle's chain rules applied to the oracle's gradient.

Bars: the chain rules are sums of a few gradient components times rates or
time spans, so each output is held to the gradient's own rule propagated
through it: |x - x*| <= tol * sum over its terms of |c_t| max(|g*_t|, 1e-2 A_t)
(c_t the coefficient of g_t), tol = 1e-9 for FP64 and 1e-4 for FP32.
"""
import numpy as np
import pytest

import oracle
from paper_2303_04390_amd import binding as B
from paper_2303_04390_amd import synth

pytestmark = pytest.mark.gpu

TOL = {B.PHG_FP64: 1e-9, B.PHG_FP32_SCALED: 1e-4}


def dated(config, seed, n_tips=None, n_patterns=None, mean_interval=0.005, tip_spread=0.01):
    prob = synth.config_problem(config, seed=seed, n_tips=n_tips, n_patterns=n_patterns)
    rng = np.random.default_rng(seed + 100)
    heights, rates = synth.time_tree(prob.parent, rng, mean_interval=mean_interval, tip_spread=tip_spread)
    prob.b = oracle.branch_lengths_from_time_tree(prob.parent, heights, rates)
    return prob, heights, rates


def bounds(prob, heights, rates, ref, set_of, n_sets):
    """Propagated per-output bars (without tol) for d_heights, d_rates, d_sets."""
    unit = np.maximum(np.abs(ref["grad"]), 1e-2 * ref["absgrad"])
    t = np.array([heights[prob.parent[i]] - heights[i] for i in range(len(rates))])
    bh = np.zeros(len(heights))
    for i, k in enumerate(prob.parent[:-1]):
        bh[k] += rates[i] * unit[i]
        bh[i] += rates[i] * unit[i]
    br = t * unit
    bs = oracle.branch_set_sums(br, set_of, n_sets) if n_sets else None
    return bh, br, bs


def expect_close(name, got, want, bar, tol):
    err = np.abs(np.asarray(got) - want)
    ratio = np.where(bar > 0, err / np.where(bar > 0, bar, 1.0), np.where(err == 0, 0.0, np.inf))
    worst = int(np.argmax(ratio))
    print(f"[parity] {name}: max err / bar {ratio.max():.3e} (tol {tol:.0e}) at {worst}", flush=True)
    assert ratio.max() <= tol, (name, worst, got[worst], want[worst], bar[worst])


def run_case(name, prob, heights, rates, prec, set_of, n_sets):
    print(f"[case] {name} prec={prec} N={prob.n_tips} C={prob.n_patterns} sets={n_sets}", flush=True)
    ref = oracle.evaluate_problem(prob)
    dh_ref, dr_ref = oracle.time_tree_gradients(prob.parent, heights, rates, ref["grad"])
    ds_ref = oracle.branch_set_sums(dr_ref, set_of, n_sets)
    bh, br, bs = bounds(prob, heights, rates, ref, set_of, n_sets)
    with B.Context.for_problem(prob, prec) as ctx:
        B.phg_set_time_tree(ctx.handle, heights, rates)
        B.phg_set_branch_sets(ctx.handle, set_of, n_sets)
        logl, dh, dr, ds = B.phg_time_tree_gradient(ctx.handle, prob.n_tips, n_sets)
        # the time tree's branch lengths are the ones the plain gradient sees
        l2, g2 = ctx.gradient()
    tol = TOL[prec]
    assert abs(logl - ref["logl"]) <= (1e-12 if prec == B.PHG_FP64 else 1e-6) * abs(ref["logl"])
    assert logl == l2
    expect_close(f"{name}/d_heights", dh, dh_ref, bh, tol)
    expect_close(f"{name}/d_rates", dr, dr_ref, br, tol)
    expect_close(f"{name}/d_sets", ds, ds_ref, bs, tol)
    # d_rates is exactly (h_pa - h) * g on the device's own gradient
    t = np.array([heights[prob.parent[i]] - heights[i] for i in range(len(rates))])
    assert np.array_equal(dr, t * g2)


@pytest.mark.parametrize("prec", [B.PHG_FP64, B.PHG_FP32_SCALED])
def test_time_tree_hky16_local_clocks(prec):
    prob, h, r = dated("hky16", 0, n_patterns=500, mean_interval=0.05, tip_spread=0.1)
    set_of = np.random.default_rng(3).integers(-1, 3, 2 * prob.n_tips - 2)
    run_case("hky16-dated", prob, h, r, prec, set_of, 3)


@pytest.mark.parametrize("prec", [B.PHG_FP32_SCALED, B.PHG_FP64])
def test_time_tree_hky1000_strict_clock(prec):
    prob, h, r = dated("hky1000", 1)
    run_case("hky1000-dated", prob, h, r, prec, np.zeros(2 * prob.n_tips - 2, np.int32), 1)


def test_time_tree_amino_acids_ragged():
    prob, h, r = dated("aa500", 2, n_tips=40, n_patterns=77, mean_interval=0.03)
    set_of = np.arange(2 * 40 - 2) % 5 - 1
    run_case("aa40-dated", prob, h, r, B.PHG_FP32_SCALED, set_of, 4)


def test_branch_length_sets_match_oracle():
    prob = synth.config_problem("hky16", seed=5, n_patterns=300)
    set_of = np.random.default_rng(8).integers(-1, 4, 30).astype(np.int32)
    ref = oracle.evaluate_problem(prob)
    want = oracle.branch_set_sums(ref["grad"], set_of, 4)
    unit = np.maximum(np.abs(ref["grad"]), 1e-2 * ref["absgrad"])
    bar = oracle.branch_set_sums(unit, set_of, 4)
    for prec in (B.PHG_FP64, B.PHG_FP32_SCALED):
        print(f"[case] branch-length sets prec={prec}", flush=True)
        with B.Context.for_problem(prob, prec) as ctx:
            B.phg_set_branch_sets(ctx.handle, set_of, 4)
            logl, ds = B.phg_gradient_branch_sets(ctx.handle, 4)
            l2, g2 = ctx.gradient()
        assert logl == l2
        expect_close(f"length-sets/{prec}", ds, want, bar, TOL[prec])
        # the set kernel sums the device's own gradient in increasing index
        for j in range(4):
            acc = 0.0
            for i in np.nonzero(set_of == j)[0]:
                acc += g2[i]
            assert abs(ds[j] - acc) <= 1e-15 * np.sum(np.abs(g2))


def test_time_tree_then_new_lengths_and_topology():
    prob, h, r = dated("hky16", 7, n_patterns=200, mean_interval=0.05)
    with B.Context.for_problem(prob, B.PHG_FP64) as ctx:
        B.phg_set_time_tree(ctx.handle, h, r)
        B.phg_time_tree_gradient(ctx.handle, prob.n_tips)
        B.phg_set_branch_lengths(ctx.handle, prob.b * 1.1)
        with pytest.raises(B.PhgError) as e:
            B.phg_time_tree_gradient(ctx.handle, prob.n_tips)
        assert e.value.status == B.PHG_ERR_STATE
        B.phg_set_time_tree(ctx.handle, h * 1.5, r)      # new heights, same topology
        logl, dh, dr, _ = B.phg_time_tree_gradient(ctx.handle, prob.n_tips)
    prob.b = oracle.branch_lengths_from_time_tree(prob.parent, h * 1.5, r)
    ref = oracle.evaluate_problem(prob)
    dh_ref, _ = oracle.time_tree_gradients(prob.parent, h * 1.5, r, ref["grad"])
    assert abs(logl - ref["logl"]) <= 1e-12 * abs(ref["logl"])
    assert np.max(np.abs(dh - dh_ref)) <= 1e-9 * np.max(np.abs(dh_ref))
