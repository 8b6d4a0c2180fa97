"""Host-side checks of the C ABI: the library loads, exports every function
include/phg.h declares, validates inputs on the host, and reports states and
errors with the documented codes.  No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2303_04390_amd import binding as B
from paper_2303_04390_amd import synth
from tests.conftest import gpu_available

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "phg.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(phg_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B._SIGS), "binding and header disagree"


def test_create_validates_sizes():
    with pytest.raises(B.PhgError) as e:
        B.phg_create(1, 10, 4, 4, B.PHG_FP64)
    assert e.value.status == B.PHG_ERR_ARG
    for args in [(10, 0, 4, 4, 0), (10, 10, 1, 4, 0), (10, 10, 257, 4, 0), (10, 10, 4, 0, 0),
                 (10, 10, 4, 65, 0), (10, 10, 4, 4, 7)]:
        with pytest.raises(B.PhgError) as e:
            B.phg_create(*args)
        assert e.value.status == B.PHG_ERR_ARG
    with pytest.raises(B.PhgError):
        B.phg_create(10, 10, 4, 4, 0, -1)


def _ctx(N=6, C=10, S=4, R=4):
    return B.phg_create(N, C, S, R, B.PHG_FP32_SCALED, 0)


def test_topology_validation():
    ctx = _ctx()
    try:
        good = synth.yule_topology(6, np.random.default_rng(0))
        B.phg_set_topology(ctx, good)
        bad = good.copy(); bad[10] = 3
        with pytest.raises(B.PhgError) as e:
            B.phg_set_topology(ctx, bad)
        assert e.value.status == B.PHG_ERR_ARG and "root" in e.value.message
        bad = good.copy(); bad[0] = 2                      # parent is a tip
        with pytest.raises(B.PhgError):
            B.phg_set_topology(ctx, bad)
        bad = good.copy()                                   # three children under one node
        other = [v for v in range(10) if good[v] != good[0]][0]
        bad[other] = good[0]
        with pytest.raises(B.PhgError) as e:
            B.phg_set_topology(ctx, bad)
        assert "children" in e.value.message
        # nodes 6 and 7 are each other's parent; every degree is still 2
        cyc = np.array([6, 7, 8, 8, 9, 9, 7, 6, 10, 10, -1], np.int32)
        with pytest.raises(B.PhgError) as e:
            B.phg_set_topology(ctx, cyc)
        assert "cycle" in e.value.message
    finally:
        B.phg_destroy(ctx)


def test_value_validation():
    ctx = _ctx()
    try:
        b = np.full(10, 0.1)
        B.phg_set_branch_lengths(ctx, b)
        for bad in (-0.1, np.nan, np.inf):
            bb = b.copy(); bb[3] = bad
            with pytest.raises(B.PhgError) as e:
                B.phg_set_branch_lengths(ctx, bb)
            assert e.value.status == B.PHG_ERR_ARG
        codes = np.zeros((6, 10), np.int32)
        B.phg_set_tip_states(ctx, codes)
        codes[2, 3] = 5
        with pytest.raises(B.PhgError):
            B.phg_set_tip_states(ctx, codes)
        codes[2, 3] = -1
        with pytest.raises(B.PhgError):
            B.phg_set_tip_states(ctx, codes)
        codes[2, 3] = 4                                    # S = fully ambiguous is allowed
        B.phg_set_tip_states(ctx, codes)
        with pytest.raises(B.PhgError):
            B.phg_set_pattern_weights(ctx, np.r_[np.ones(9), -1.0])
        with pytest.raises(B.PhgError):
            B.phg_set_categories(ctx, np.ones(4), np.r_[np.ones(3), np.nan])
        with pytest.raises(B.PhgError):
            B.phg_set_root_frequencies(ctx, np.array([0.5, 0.5, -0.1, 0.1]))
        V = np.eye(4); V[1, 1] = np.inf
        with pytest.raises(B.PhgError):
            B.phg_set_eigen(ctx, V, np.eye(4), np.zeros(4))
    finally:
        B.phg_destroy(ctx)


def test_compute_before_inputs_is_state_error():
    ctx = _ctx()
    try:
        B.phg_set_topology(ctx, synth.yule_topology(6, np.random.default_rng(1)))
        with pytest.raises(B.PhgError) as e:
            B.phg_gradient(ctx, 10)
        assert e.value.status == B.PHG_ERR_STATE
        assert "branch_lengths" in e.value.message and "eigen" in e.value.message
    finally:
        B.phg_destroy(ctx)


def test_schedule_levels():
    N = 200
    ctx = B.phg_create(N, 10, 4, 4, B.PHG_FP32_SCALED, 0)
    try:
        parent = synth.caterpillar_topology(N)
        B.phg_set_topology(ctx, parent)
        post, pre, _ = B.phg_schedule_info(ctx)             # blocks: one per 3 depths
        assert post == pre == (N - 2) // 3 + 1
        B.phg_set_schedule(ctx, B.PHG_SCHEDULE_LEVELS)
        post, pre, launches = B.phg_schedule_info(ctx)
        assert post == N - 1 and pre == N - 1 and launches == 2 * N
        parent = synth.yule_topology(N, np.random.default_rng(3))
        B.phg_set_topology(ctx, parent)
        post, pre, _ = B.phg_schedule_info(ctx)
        assert post < 40 and pre < 40
    finally:
        B.phg_destroy(ctx)


def test_workspace_size_scales():
    a = B.phg_workspace_size(1000, 10000, 4, 4, B.PHG_FP32_SCALED)
    b = B.phg_workspace_size(1000, 10000, 4, 4, B.PHG_FP64)
    # internal partials dominate: (N-1) * Cpad * R * S * bytes
    part32 = 999 * 10048 * 16 * 4
    assert part32 < a < part32 * 1.2
    assert 1.8 * a < b < 2.2 * a


@pytest.mark.skipif(gpu_available(), reason="checks the no-GPU error path")
def test_compute_without_gpu_is_device_error():
    prob = synth.config_problem("hky16", seed=0, n_patterns=20)
    ctx = B.Context.for_problem(prob)
    try:
        with pytest.raises(B.PhgError) as e:
            ctx.gradient()
        assert e.value.status == B.PHG_ERR_DEVICE
    finally:
        ctx.close()


def test_one_hip_runtime_in_process():
    """libphg.so must share torch's HIP runtime (a second copy would make
    torch streams and memory foreign handles to the library)."""
    import subprocess
    import sys
    code = ("from paper_2303_04390_amd import binding as B; B.lib(); import torch; "
            "torch.cuda.device_count(); maps = open('/proc/self/maps').read().splitlines(); "
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         cwd=os.path.dirname(os.path.dirname(__file__)), timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_block_schedule_shape():
    N = 1000
    parent = synth.yule_topology(N, np.random.default_rng(0))
    ctx = B.phg_create(N, 10, 4, 4, B.PHG_FP32_SCALED, 0)
    try:
        B.phg_set_topology(ctx, parent)
        post_b, pre_b, _ = B.phg_schedule_info(ctx)        # AUTO -> blocks for 4 states
        assert B.phg_get_schedule(ctx) == B.PHG_SCHEDULE_BLOCKS
        B.phg_set_schedule(ctx, B.PHG_SCHEDULE_LEVELS)
        assert B.phg_get_schedule(ctx) == B.PHG_SCHEDULE_LEVELS
        post_l, pre_l, _ = B.phg_schedule_info(ctx)
        assert post_b == pre_b and post_b < post_l / 2 and pre_b < pre_l / 2
        B.phg_set_schedule(ctx, B.PHG_SCHEDULE_BLOCKS)
        assert B.phg_schedule_info(ctx)[0] == post_b
    finally:
        B.phg_destroy(ctx)
    ctx = B.phg_create(50, 10, 20, 4, B.PHG_FP32_SCALED, 0)
    try:
        with pytest.raises(B.PhgError) as e:
            B.phg_get_schedule(ctx)                        # no topology yet
        assert e.value.status == B.PHG_ERR_STATE
        B.phg_set_topology(ctx, synth.yule_topology(50, np.random.default_rng(1)))
        assert B.phg_get_schedule(ctx) == B.PHG_SCHEDULE_LEVELS   # 20 states: levels only
        with pytest.raises(B.PhgError) as e:
            B.phg_set_schedule(ctx, B.PHG_SCHEDULE_BLOCKS)
        assert e.value.status == B.PHG_ERR_ARG
    finally:
        B.phg_destroy(ctx)
    ctx = B.phg_create(50, 10, 4, 9, B.PHG_FP64, 0)
    try:
        with pytest.raises(B.PhgError):
            B.phg_set_schedule(ctx, B.PHG_SCHEDULE_BLOCKS)
    finally:
        B.phg_destroy(ctx)


def test_queue_schedule_is_opt_in_and_checked():
    N = 300
    parent = synth.yule_topology(N, np.random.default_rng(4))
    ctx = B.phg_create(N, 100, 4, 4, B.PHG_FP32_SCALED, 0)
    try:
        B.phg_set_topology(ctx, parent)
        assert B.phg_get_schedule(ctx) == B.PHG_SCHEDULE_BLOCKS       # AUTO: not the queue
        B.phg_set_schedule(ctx, B.PHG_SCHEDULE_QUEUE)
        assert B.phg_get_schedule(ctx) == B.PHG_SCHEDULE_QUEUE
        post_q, pre_q, _ = B.phg_schedule_info(ctx)
        B.phg_set_schedule(ctx, B.PHG_SCHEDULE_BLOCKS)
        assert B.phg_schedule_info(ctx)[:2] == (post_q, pre_q)         # the same block levels
        with pytest.raises(B.PhgError) as e:
            B.phg_set_schedule(ctx, 4)
        assert e.value.status == B.PHG_ERR_ARG
    finally:
        B.phg_destroy(ctx)
    # 4 states: FP32 and R in {1, 2, 4, 8}; else the vector-ALU and MFMA
    # kernels' shapes (17..256 states), not the small-state MFMA kernels
    for S, R, prec in ((4, 4, B.PHG_FP64), (4, 3, B.PHG_FP32_SCALED), (8, 4, B.PHG_FP32_SCALED),
                       (16, 2, B.PHG_FP64), (4, 16, B.PHG_FP32_SCALED)):
        ctx = B.phg_create(30, 10, S, R, prec, 0)
        try:
            with pytest.raises(B.PhgError) as e:
                B.phg_set_schedule(ctx, B.PHG_SCHEDULE_QUEUE)
            assert e.value.status == B.PHG_ERR_ARG
        finally:
            B.phg_destroy(ctx)
    for S, prec in ((20, B.PHG_FP32_SCALED), (32, B.PHG_FP32_SCALED), (20, B.PHG_FP64), (61, B.PHG_FP32_SCALED),
                    (200, B.PHG_FP64)):
        ctx = B.phg_create(30, 10, S, 4, prec, 0)
        try:
            B.phg_set_topology(ctx, synth.yule_topology(30, np.random.default_rng(5)))
            B.phg_set_schedule(ctx, B.PHG_SCHEDULE_QUEUE)
            assert B.phg_get_schedule(ctx) == B.PHG_SCHEDULE_QUEUE
            # per-chunk P(t) tables (a table budget below one table per branch): levels
            B.phg_set_table_budget(ctx, 1 << 16)
            assert B.phg_get_schedule(ctx) == B.PHG_SCHEDULE_LEVELS
        finally:
            B.phg_destroy(ctx)
    # launches per evaluation: 1 or 2, 4-state FP32 only
    B.phg_set_tuning(4, 0, B.PHG_FP32_SCALED, B.PHG_TUNE_QUEUE_LAUNCHES, 1)
    assert B.phg_get_tuning(4, 0, B.PHG_FP32_SCALED, B.PHG_TUNE_QUEUE_LAUNCHES) == 1
    B.phg_set_tuning(4, 0, B.PHG_FP32_SCALED, B.PHG_TUNE_QUEUE_LAUNCHES, 0)
    for S, prec, v in ((4, B.PHG_FP32_SCALED, 3), (4, B.PHG_FP64, 1), (20, B.PHG_FP32_SCALED, 1)):
        with pytest.raises(B.PhgError):
            B.phg_set_tuning(S, 0, prec, B.PHG_TUNE_QUEUE_LAUNCHES, v)
    # the wait bound: wherever the queue runs
    for S, prec in ((4, B.PHG_FP32_SCALED), (20, B.PHG_FP64), (61, B.PHG_FP32_SCALED)):
        B.phg_set_tuning(S, 0, prec, B.PHG_TUNE_QUEUE_WAIT_US, 5)
        assert B.phg_get_tuning(S, 0, prec, B.PHG_TUNE_QUEUE_WAIT_US) == 5
        B.phg_set_tuning(S, 0, prec, B.PHG_TUNE_QUEUE_WAIT_US, 0)
    with pytest.raises(B.PhgError):
        B.phg_set_tuning(4, 0, B.PHG_FP64, B.PHG_TUNE_QUEUE_WAIT_US, 5)


def test_time_tree_and_branch_set_validation():
    N = 6
    parent = synth.yule_topology(N, np.random.default_rng(2))
    heights, rates = synth.time_tree(parent, np.random.default_rng(3))
    ctx = B.phg_create(N, 10, 4, 4, B.PHG_FP64, 0)
    try:
        with pytest.raises(B.PhgError) as e:
            B.phg_set_time_tree(ctx, heights, rates)            # no topology yet
        assert e.value.status == B.PHG_ERR_STATE
        B.phg_set_topology(ctx, parent)
        bad = heights.copy()
        bad[0] = heights[parent[0]] + 1.0                       # tip above its parent
        with pytest.raises(B.PhgError) as e:
            B.phg_set_time_tree(ctx, bad, rates)
        assert e.value.status == B.PHG_ERR_ARG and "above its parent" in str(e.value)
        r = rates.copy()
        r[3] = -0.1
        with pytest.raises(B.PhgError):
            B.phg_set_time_tree(ctx, heights, r)
        r[3] = np.nan
        with pytest.raises(B.PhgError):
            B.phg_set_time_tree(ctx, heights, r)
        with pytest.raises(B.PhgError) as e:
            B.phg_time_tree_gradient(ctx, N)                     # no time tree
        assert e.value.status == B.PHG_ERR_STATE
        B.phg_set_time_tree(ctx, heights, rates)
        with pytest.raises(B.PhgError) as e:
            B.phg_time_tree_gradient(ctx, N, n_sets=2)           # sets wanted, none set
        assert e.value.status == B.PHG_ERR_STATE
        B.phg_set_branch_lengths(ctx, np.full(2 * N - 2, 0.1))  # leaves time-tree mode
        with pytest.raises(B.PhgError) as e:
            B.phg_time_tree_gradient(ctx, N)
        assert e.value.status == B.PHG_ERR_STATE
        E = 2 * N - 2
        with pytest.raises(B.PhgError) as e:
            B.phg_set_branch_sets(ctx, np.full(E, 2, np.int32), 2)   # entry out of range
        assert e.value.status == B.PHG_ERR_ARG
        with pytest.raises(B.PhgError):
            B.phg_set_branch_sets(ctx, np.zeros(E, np.int32), E + 1)
        with pytest.raises(B.PhgError) as e:
            B.phg_gradient_branch_sets(ctx, 2)                   # no sets
        assert e.value.status == B.PHG_ERR_STATE
        B.phg_set_branch_sets(ctx, np.arange(E, dtype=np.int32) % 2, 2)
        B.phg_set_branch_sets(ctx, None, 0)                      # clear
        with pytest.raises(B.PhgError) as e:
            B.phg_gradient_branch_sets(ctx, 2)
        assert e.value.status == B.PHG_ERR_STATE
    finally:
        B.phg_destroy(ctx)


def test_category_eigen_validation():
    ctx = B.phg_create(5, 10, 4, 3, B.PHG_FP64, 0)
    try:
        V = np.stack([np.eye(4)] * 3)
        lam = np.zeros((3, 4))
        B.phg_set_category_eigen(ctx, V, V, lam)
        lam[2, 1] = np.inf
        with pytest.raises(B.PhgError) as e:
            B.phg_set_category_eigen(ctx, V, V, lam)
        assert e.value.status == B.PHG_ERR_ARG
    finally:
        B.phg_destroy(ctx)


def test_tip_partials_validation_and_schedule():
    """phg_set_tip_partials: argument checks, and the schedule rule (a context
    with any general tip vector runs the level schedule)."""
    N, C, S = 40, 12, 4
    ctx = B.phg_create(N, C, S, 4, B.PHG_FP32_SCALED, 0)
    try:
        B.phg_set_topology(ctx, synth.yule_topology(N, np.random.default_rng(2)))
        assert B.phg_get_schedule(ctx) == B.PHG_SCHEDULE_BLOCKS
        good = np.full((C, S), 0.25)
        for tip in (-1, N):
            with pytest.raises(B.PhgError) as e:
                B.phg_set_tip_partials(ctx, tip, good)
            assert e.value.status == B.PHG_ERR_ARG
        for bad in (-1e-3, np.nan, np.inf):
            v = good.copy()
            v[3, 1] = bad
            with pytest.raises(B.PhgError) as e:
                B.phg_set_tip_partials(ctx, 5, v)
            assert e.value.status == B.PHG_ERR_ARG and "finite" in str(e.value)
        assert B.phg_get_schedule(ctx) == B.PHG_SCHEDULE_BLOCKS      # rejected calls change nothing
        B.phg_set_tip_partials(ctx, 5, good)
        assert B.phg_get_schedule(ctx) == B.PHG_SCHEDULE_LEVELS      # AUTO falls back to levels
        with pytest.raises(B.PhgError) as e:
            B.phg_set_schedule(ctx, B.PHG_SCHEDULE_BLOCKS)
        assert e.value.status == B.PHG_ERR_ARG
        B.phg_set_tip_partials(ctx, 5, None)                         # back to its code
        assert B.phg_get_schedule(ctx) == B.PHG_SCHEDULE_BLOCKS
        B.phg_set_schedule(ctx, B.PHG_SCHEDULE_BLOCKS)
        with pytest.raises(B.PhgError) as e:
            B.phg_set_tip_partials(ctx, 5, good)                     # forced blocks: rejected
        assert e.value.status == B.PHG_ERR_ARG
    finally:
        B.phg_destroy(ctx)


def test_noalloc_entry_refuses_oversized_workspace():
    """phg_gradient_async_noalloc checks the workspace against its static
    array before any device work (the output pointers are never touched)."""
    prob = synth.config_problem("hky1000", seed=0, n_patterns=64)
    big = B.Context(1000, 10000, 4, 4, B.PHG_FP32_SCALED)
    try:
        small = synth.config_problem("hky1000", seed=0)
        big.set_problem(small)
        with pytest.raises(B.PhgError) as e:
            B.phg_gradient_async_noalloc(big.handle, 256, 512)
        assert e.value.status == B.PHG_ERR_OOM and "static scratch" in e.value.message
    finally:
        big.close()
    assert B.phg_workspace_size(1000, 10000, 4, 4, B.PHG_FP32_SCALED) > (64 << 20)
    assert prob.n_tips == 1000


def test_tuning_table_validation():
    """phg_set_tuning accepts only values the kernels are built for; the
    table is read back through phg_get_tuning; value 0 restores the rule."""
    f32, f64 = B.PHG_FP32_SCALED, B.PHG_FP64
    RB, NU = B.PHG_TUNE_ROW_BLOCKS, B.PHG_TUNE_NARROW_UNITS
    try:
        for S, prec, ok, bad in [(20, f32, (1, 2, 4), (3, 8)), (20, f64, (1, 2), (4,)),
                                 (61, f32, (1, 2, 4), (3,)), (61, f64, (1,), (2, 4)),
                                 (122, f32, (2,), (1, 4)), (240, f64, (1,), (2,))]:
            for v in ok:
                B.phg_set_tuning(S, 0, prec, RB, v)
                assert B.phg_get_tuning(S, 4, prec, RB) == v
            for v in bad:
                with pytest.raises(B.PhgError) as e:
                    B.phg_set_tuning(S, 0, prec, RB, v)
                assert e.value.status == B.PHG_ERR_ARG
            B.phg_set_tuning(S, 0, prec, RB, 0)
            assert B.phg_get_tuning(S, 4, prec, RB) == 0
        with pytest.raises(B.PhgError):
            B.phg_set_tuning(4, 4, f32, RB, 2)          # 4 states do not take row blocks
        B.phg_set_tuning(4, 4, f32, NU, 1000)
        assert B.phg_get_tuning(4, 4, f32, NU) == 1000
        assert B.phg_get_tuning(4, 2, f32, NU) == 0     # another category count
        with pytest.raises(B.PhgError):
            B.phg_set_tuning(4, 4, f64, NU, 1000)
        # the context's tile follows the row blocks in effect at creation on
        # the MFMA kernels (20 states at 3 categories); the vector-ALU kernels
        # (20 states at 4 categories) have a fixed 64-pattern tile
        B.phg_set_tuning(20, 0, f32, RB, 4)
        big = B.phg_workspace_size(100, 1000, 20, 3, f32)
        vs_a = B.phg_workspace_size(100, 1000, 20, 4, f32)
        B.phg_set_tuning(20, 0, f32, RB, 1)
        small = B.phg_workspace_size(100, 1000, 20, 3, f32)
        vs_b = B.phg_workspace_size(100, 1000, 20, 4, f32)
        assert big != small                             # per-tile sums: Cpad / tile of them
        assert vs_a == vs_b
    finally:
        B.phg_set_tuning(4, 4, f32, NU, 0)
        B.phg_set_tuning(20, 0, f32, RB, 0)


def test_tuning_file_is_read_at_first_use(tmp_path):
    """libphg.so fills its tuning table from PHG_TUNE_FILE (format: 'gfx950 S R
    prec param value'); other devices, comments and values the kernels are not
    built for are skipped; PHG_TUNE=off ignores the file."""
    import subprocess
    import sys
    f = tmp_path / "tune.txt"
    f.write_text("# comment\ngfx950 20 0 1 0 4\ngfx942 61 0 1 0 4\ngfx950 61 0 0 0 4\ngfx950 4 4 1 1 777\n")
    code = ("from paper_2303_04390_amd import binding as B;"
            "print(B.phg_get_tuning(20, 4, 1, 0), B.phg_get_tuning(61, 4, 1, 0), B.phg_get_tuning(61, 4, 0, 0),"
            " B.phg_get_tuning(4, 4, 1, 1))")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, PHG_TUNE_FILE=str(f))
    env.pop("PHG_TUNE", None)
    out = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["4", "0", "0", "777"]
    env["PHG_TUNE"] = "off"
    out = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True)
    assert out.stdout.split() == ["0", "0", "0", "0"]


def test_graph_calls_on_cpu():
    ctx = _ctx()
    try:
        assert B.phg_graph_stats(ctx) == (0, 0)
        B.phg_set_graphs(ctx, False)
        B.phg_set_graphs(ctx, True)
    finally:
        B.phg_destroy(ctx)


def test_kernel_family_matches_the_routing_rule():
    """phg_kernel_family_of: 4 states at R <= 8 on the 4-state kernels; other
    shapes up to 16 states on the small MFMA kernels; 17..32 states (FP64
    17..24) at R in 1, 2, 4, 8 on the vector-ALU kernels while the pre-order
    workgroup's LDS fits 80 KiB; everything else above 16 states on the MFMA
    kernels; sizes phg_create refuses are PHG_ERR_ARG."""
    f32, f64 = B.PHG_FP32_SCALED, B.PHG_FP64
    fam = B.phg_kernel_family_of
    assert fam(4, 4, f32) == fam(4, 8, f64) == B.PHG_KERNELS_FOUR_STATE
    assert fam(4, 16, f32) == fam(8, 3, f64) == fam(16, 4, f32) == B.PHG_KERNELS_SMALL_MFMA
    for S in (17, 20, 24, 25, 32):
        for R in (1, 2, 4):
            assert fam(S, R, f32) == B.PHG_KERNELS_VECTOR_ALU, (S, R)
    assert fam(20, 8, f32) == B.PHG_KERNELS_VECTOR_ALU         # 72 KiB of LDS
    assert fam(24, 8, f32) == B.PHG_KERNELS_MFMA                # 94 KiB
    assert fam(20, 4, f64) == B.PHG_KERNELS_VECTOR_ALU
    assert fam(24, 4, f64) == B.PHG_KERNELS_MFMA                # 94 KiB
    assert fam(25, 1, f64) == B.PHG_KERNELS_MFMA                # FP64 stops at 24 states
    for S, R in ((20, 3), (20, 16), (33, 4), (61, 4), (256, 2)):
        assert fam(S, R, f32) == B.PHG_KERNELS_MFMA, (S, R)
    for S, R in ((1, 4), (257, 4), (20, 0), (20, 65)):
        with pytest.raises(B.PhgError) as e:
            fam(S, R, f32)
        assert e.value.status == B.PHG_ERR_ARG
