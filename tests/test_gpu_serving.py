"""Serving engine: continuous batching of requests for many trees.

Every work unit's arithmetic is independent of what else shares its launch,
so a request's result must be bitwise identical alone and in a mix; results
are also checked against the single-context path (bitwise) and the oracle.
"""
import threading

import numpy as np
import pytest

import oracle
from paper_2303_04390_amd import binding as B
from paper_2303_04390_amd import synth
from tests.parity import check

pytestmark = pytest.mark.gpu

GiB = 1 << 30


def states122_problem(seed, N=12, C=150):
    rng = np.random.default_rng(seed)
    pi = rng.dirichlet([2.0] * 122)
    Q = synth.gtr_model(rng.gamma(1.0, 1.0, 122 * 121 // 2), pi)
    rates, w = synth.discrete_gamma(0.5, 4)
    return synth.make_problem(synth.yule_topology(N, rng), synth.exponential_branch_lengths(N, 0.05, rng), Q,
                              pi, rates, w, C, rng)


def trees_mix(seed=0):
    """Trees of uneven taxon and pattern counts, 4, 20, 61 and 122 states,
    both precisions.  The 122-state trees' P(t) tables span 2 x 2 output
    tiles of the P(t) kernel and the 20- and 61-state ones a single tile, so
    their P(t) work must not share a launch."""
    out = []
    for k, (N, C) in enumerate([(64, 500), (300, 2000), (1000, 3000), (20, 7000), (500, 1200)]):
        out.append((synth.config_problem("hky1000", seed=seed + k, n_tips=N, n_patterns=C),
                    B.PHG_FP32_SCALED))
    out.append((synth.config_problem("hky1000", seed=seed + 9, n_tips=200, n_patterns=900), B.PHG_FP64))
    out.append((synth.config_problem("aa500", seed=seed + 3, n_tips=60, n_patterns=400), B.PHG_FP32_SCALED))
    out.append((synth.config_problem("codon128", seed=seed + 4, n_tips=24, n_patterns=300), B.PHG_FP64))
    out.append((states122_problem(seed + 5), B.PHG_FP32_SCALED))
    out.append((states122_problem(seed + 6, N=9, C=70), B.PHG_FP64))
    return out


def single_context(prob, prec, b=None):
    with B.Context.for_problem(prob, prec) as ctx:
        if b is not None:
            B.phg_set_branch_lengths(ctx.handle, b)
        return ctx.gradient()


def test_single_request_matches_context_and_oracle():
    prob = synth.config_problem("hky1000", seed=1, n_tips=300, n_patterns=2500)
    print("[case] server single request", flush=True)
    srv = B.phg_server_create(0, 4 * GiB, 8)
    try:
        tid = B.phg_server_register_tree(srv, prob, B.PHG_FP32_SCALED)
        rid = B.phg_server_submit(srv, tid, prob.b)
        logl, grad = B.phg_server_wait(srv, rid, 2 * prob.n_tips - 2)
    finally:
        B.phg_server_destroy(srv)
    l0, g0 = single_context(prob, B.PHG_FP32_SCALED)
    assert logl == l0 and np.array_equal(grad, g0)
    check("server-single", logl, grad, oracle.evaluate_problem(prob), 1e-6, 1e-4)


def test_alone_vs_mix_bitwise():
    mix = trees_mix()
    rng = np.random.default_rng(7)
    bs = [p.b * np.exp(rng.normal(0, 0.05, p.b.shape)) for p, _ in mix]
    alone = []
    print("[case] alone", flush=True)
    srv = B.phg_server_create(0, 8 * GiB, 16)
    try:
        for (p, prec), b in zip(mix, bs):
            tid = B.phg_server_register_tree(srv, p, prec)
            rid = B.phg_server_submit(srv, tid, b)
            alone.append(B.phg_server_wait(srv, rid, 2 * p.n_tips - 2))
    finally:
        B.phg_server_destroy(srv)
    print("[case] mix: all trees at once, 3 requests each, interleaved", flush=True)
    srv = B.phg_server_create(0, 8 * GiB, 16)
    try:
        tids = [B.phg_server_register_tree(srv, p, prec) for p, prec in mix]
        rids = []
        for rep in range(3):
            for k, ((p, _), tid) in enumerate(zip(mix, tids)):
                b = bs[k] if rep == 1 else p.b * np.exp(rng.normal(0, 0.05, p.b.shape))
                rids.append((k, rep, B.phg_server_submit(srv, tid, b)))
        res = {}
        for k, rep, rid in rids:
            res[(k, rep)] = B.phg_server_wait(srv, rid, 2 * mix[k][0].n_tips - 2)
        stats = B.phg_server_stats(srv)
    finally:
        B.phg_server_destroy(srv)
    print(f"[serving] mix stats {stats}", flush=True)
    for k in range(len(mix)):
        la, ga = alone[k]
        lm, gm = res[(k, 1)]
        assert la == lm and np.array_equal(ga, gm), k
    # the same results as the single-context path
    for k, ((p, prec), b) in enumerate(zip(mix, bs)):
        l0, g0 = single_context(p, prec, b)
        assert alone[k][0] == l0 and np.array_equal(alone[k][1], g0), k
    assert stats["completed"] == 3 * len(mix)
    # requests share launches: fewer than the same requests issue one
    # context at a time
    alone_launches = 0
    for p, prec in mix:
        with B.Context.for_problem(p, prec) as ctx:
            alone_launches += 3 * B.phg_schedule_info(ctx.handle)[2]
    print(f"[serving] launches {stats['launches']} shared vs {alone_launches} alone", flush=True)
    assert stats["launches"] < alone_launches


def test_tiny_budget_forces_eviction_and_stays_correct():
    probs = [synth.config_problem("hky1000", seed=20 + k, n_tips=200, n_patterns=3000) for k in range(6)]
    ws = B.phg_workspace_size(200, 3000, 4, 4, B.PHG_FP32_SCALED)
    print(f"[case] budget for 2 trees of {ws} bytes", flush=True)
    srv = B.phg_server_create(0, 2 * ws + (1 << 20), 8)
    try:
        tids = [B.phg_server_register_tree(srv, p, B.PHG_FP32_SCALED) for p in probs]
        rids = [B.phg_server_submit(srv, t, p.b) for _ in range(2) for t, p in zip(tids, probs)]
        out = [B.phg_server_wait(srv, r, 398) for r in rids]
        stats = B.phg_server_stats(srv)
    finally:
        B.phg_server_destroy(srv)
    print(f"[serving] eviction stats {stats}", flush=True)
    assert stats["evictions"] > 0 and stats["peak_bytes"] <= 2 * ws + (1 << 20)
    for k, p in enumerate(probs):
        l0, g0 = single_context(p, B.PHG_FP32_SCALED)
        for rep in range(2):
            l, g = out[rep * len(probs) + k]
            assert l == l0 and np.array_equal(g, g0)


def test_same_tree_requests_in_order_and_hmc_steps():
    prob = synth.config_problem("hky16", seed=3, n_patterns=500)
    rng = np.random.default_rng(2)
    bs = [prob.b * np.exp(rng.normal(0, 0.05, prob.b.shape)) for _ in range(5)]
    print("[case] five requests for one tree", flush=True)
    srv = B.phg_server_create(0, GiB, 4)
    try:
        tid = B.phg_server_register_tree(srv, prob, B.PHG_FP64)
        rids = [B.phg_server_submit(srv, tid, b) for b in bs]
        outs = [B.phg_server_wait(srv, r, 30) for r in rids]
    finally:
        B.phg_server_destroy(srv)
    for b, (l, g) in zip(bs, outs):
        ref = oracle.evaluate_problem(synth.Problem(**{**prob.__dict__, "b": b}))
        check("server-hmc", l, g, ref, 1e-12, 1e-9)


def test_numeric_error_and_release():
    pi = np.full(4, 0.25)
    Q = synth.hky_model(2.0, pi)
    V, Vinv, lam = synth.eigensystem(Q, pi)
    bad = synth.Problem(parent=np.array([2, 2, -1], np.int32), b=np.zeros(2), V=V, Vinv=Vinv, lam=lam,
                        pi=pi, rates=np.ones(1), weights=np.ones(1),
                        codes=np.array([[0, 1], [1, 1]], np.int32), pattern_weights=np.ones(2), Q=Q)
    good = synth.config_problem("hky16", seed=4, n_patterns=100)
    print("[case] numeric error + release", flush=True)
    srv = B.phg_server_create(0, GiB, 4)
    try:
        tb = B.phg_server_register_tree(srv, bad, B.PHG_FP32_SCALED)
        tg = B.phg_server_register_tree(srv, good, B.PHG_FP32_SCALED)
        r1 = B.phg_server_submit(srv, tb, bad.b)
        r2 = B.phg_server_submit(srv, tg, good.b)
        with pytest.raises(B.PhgError) as e:
            B.phg_server_wait(srv, r1, 2)
        assert e.value.status == B.PHG_ERR_NUMERIC
        l, g = B.phg_server_wait(srv, r2, 30)
        assert np.isfinite(l)
        B.phg_server_release_tree(srv, tb)
        with pytest.raises(B.PhgError) as e:
            B.phg_server_submit(srv, tb, bad.b)
        assert e.value.status == B.PHG_ERR_ARG
        with pytest.raises(B.PhgError):
            B.phg_server_submit(srv, tg, -good.b)
    finally:
        B.phg_server_destroy(srv)


def test_concurrent_submitters():
    probs = [synth.config_problem("hky1000", seed=40 + k, n_tips=100, n_patterns=800) for k in range(4)]
    refs = [single_context(p, B.PHG_FP32_SCALED) for p in probs]
    print("[case] 4 submitter threads", flush=True)
    srv = B.phg_server_create(0, 2 * GiB, 12)
    errors = []
    try:
        tids = [B.phg_server_register_tree(srv, p, B.PHG_FP32_SCALED) for p in probs]

        def worker(k):
            try:
                for _ in range(6):
                    rid = B.phg_server_submit(srv, tids[k], probs[k].b)
                    l, g = B.phg_server_wait(srv, rid, 198)
                    if not (l == refs[k][0] and np.array_equal(g, refs[k][1])):
                        errors.append(k)
            except Exception as ex:  # noqa: BLE001
                errors.append(repr(ex))

        th = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join(timeout=120)
        assert not any(t.is_alive() for t in th)
    finally:
        B.phg_server_destroy(srv)
    assert not errors, errors


def general_trees(seed=30):
    """Trees in the general form of the gradient-kernel section: one
    substitution model per rate category (4 and 20 states), and general tip
    partial vectors on some tips (4 and 61 states), beside plain trees."""
    rng = np.random.default_rng(seed)
    out = []
    p = synth.config_problem("hky1000", seed=seed, n_tips=150, n_patterns=700)
    p.Q, p.V, p.Vinv, p.lam = synth.category_models(4, 4, rng)
    out.append((p, B.PHG_FP32_SCALED))
    p = synth.config_problem("aa500", seed=seed + 1, n_tips=40, n_patterns=300)
    p.Q, p.V, p.Vinv, p.lam = synth.category_models(20, 4, rng)
    out.append((p, B.PHG_FP64))
    p = synth.config_problem("hky16", seed=seed + 2, n_patterns=400)
    p.tip_vectors = {t: rng.uniform(0.0, 1.0, (400, 4)) for t in (1, 5, 9)}
    out.append((p, B.PHG_FP32_SCALED))
    p = synth.config_problem("codon128", seed=seed + 3, n_tips=20, n_patterns=200)
    p.tip_vectors = {t: rng.uniform(0.0, 1.0, (200, 61)) for t in (0, 7)}
    out.append((p, B.PHG_FP32_SCALED))
    out.append((synth.config_problem("hky1000", seed=seed + 4, n_tips=300, n_patterns=2000), B.PHG_FP32_SCALED))
    return out


def test_general_trees_alone_vs_mix_and_oracle():
    """Per-category models and general tip vectors through the tree
    descriptor: each request's result is bitwise the same alone, in a mix and
    on a single context, and meets the oracle bar."""
    mix = general_trees()
    rng = np.random.default_rng(8)
    bs = [p.b * np.exp(rng.normal(0, 0.05, p.b.shape)) for p, _ in mix]
    alone = []
    print("[case] general trees alone", flush=True)
    srv = B.phg_server_create(0, 4 * GiB, 8)
    try:
        for (p, prec), b in zip(mix, bs):
            tid = B.phg_server_register_tree(srv, p, prec)
            alone.append(B.phg_server_wait(srv, B.phg_server_submit(srv, tid, b), 2 * p.n_tips - 2))
    finally:
        B.phg_server_destroy(srv)
    print("[case] general trees in a mix", flush=True)
    srv = B.phg_server_create(0, 4 * GiB, 8)
    try:
        tids = [B.phg_server_register_tree(srv, p, prec) for p, prec in mix]
        rids = [B.phg_server_submit(srv, tid, b) for tid, b in zip(tids, bs)]
        mixed = [B.phg_server_wait(srv, rid, 2 * p.n_tips - 2) for rid, (p, _) in zip(rids, mix)]
        busy, wall = B.phg_server_busy(srv)
    finally:
        B.phg_server_destroy(srv)
    assert 0 < busy < wall
    for k, ((p, prec), b) in enumerate(zip(mix, bs)):
        assert alone[k][0] == mixed[k][0] and np.array_equal(alone[k][1], mixed[k][1]), k
        l0, g0 = single_context(p, prec, b)
        assert alone[k][0] == l0 and np.array_equal(alone[k][1], g0), k
        q = synth.Problem(**{**p.__dict__, "b": b})
        tol = (1e-12, 1e-9) if prec == B.PHG_FP64 else (1e-6, 1e-4)
        check(f"server-general-{k}", mixed[k][0], mixed[k][1], oracle.evaluate_problem(q), *tol)
