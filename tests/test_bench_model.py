"""The roofline numerator: bench.py's algorithmic bytes per evaluation,
checked on hand-countable trees and against the figures quoted for the
1000-taxon workload (no GPU)."""
import numpy as np

import bench
from paper_2303_04390_amd import synth


def balanced8():
    # tips 0..7; depth-2 nodes 8..11, depth-1 nodes 12, 13, root 14
    parent = np.full(15, -1, np.int32)
    for t in range(8):
        parent[t] = 8 + t // 2
    parent[8], parent[9], parent[10], parent[11] = 12, 12, 13, 13
    parent[12], parent[13] = 14, 14
    return parent


def caterpillar6():
    # internal nodes 6..10 chained: root 10 at depth 0, 9 at 1, ..., 6 at 4
    parent = np.full(11, -1, np.int32)
    parent[0], parent[1] = 6, 6
    for t in range(2, 6):
        parent[t] = 5 + t         # tip t hangs off node 5 + t (7..10)
    for v in range(6, 10):
        parent[v] = v + 1
    return parent


def test_level_model_closed_form():
    N, C, R, S, tsz = 8, 100, 4, 4, 4
    vec = R * S * tsz
    post, pre = bench.algorithmic_bytes(balanced8(), N, C, R, S, tsz)
    # every non-root internal partial written and read once (+ int32
    # exponents), every tip code read once, W_c and the site log-likelihood
    # at the root
    assert post == C * (N + 2 * (N - 2) * (vec + 4) + 16)
    # pre-order: each non-root internal node's p read and q written by its
    # parent and q read by itself; codes once; W_c once per level (3 levels);
    # one float64 gradient partial per branch and 64-pattern tile
    assert pre == C * (N + 3 * (N - 2) * vec + 8 * 3) + 8 * (2 * N - 2) * 2


def test_blocked_model_closed_form():
    C, R, S, tsz = 64, 2, 4, 4
    vec = R * S * tsz
    # balanced 8: only the root is a block root (depths 0..2)
    post, pre = bench.algorithmic_bytes_blocked(balanced8(), 8, C, R, S, tsz)
    assert post == C * (8 + 16)
    assert pre == C * (8 + 8) + 8 * 14 * 1
    # caterpillar of 6 tips: block roots at depths 0 and 3 -> one non-root
    post, pre = bench.algorithmic_bytes_blocked(caterpillar6(), 6, C, R, S, tsz)
    assert post == C * (6 + 2 * (vec + 4) + 16)
    assert pre == C * (6 + 3 * vec + 8 * 2) + 8 * 10 * 1


def test_headline_figures():
    """The 1000-taxon HKY+Gamma4 workload: 466 MB (post) and 683 MB
    (pre + gradient) per evaluation under the blocked schedule in FP32."""
    prob = synth.config_problem("hky1000", seed=0)
    post, pre = bench.algorithmic_bytes_blocked(prob.parent, 1000, 10000, 4, 4, 4)
    assert abs(post / 1e6 - 466) < 1 and abs(pre / 1e6 - 683) < 1
    assert abs(pre / 8 - 85323686) < 1e-6 * pre   # the per-launch figure bench reports


def test_bench_refuses_more_than_one_gpu():
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
