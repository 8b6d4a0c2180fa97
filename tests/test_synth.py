"""Properties of the seeded input generator (tree shapes, models, rates, sites)."""
import numpy as np
import pytest
import scipy.linalg

from paper_2303_04390_amd import synth


def _check_tree(parent):
    n = parent.shape[0]
    N = (n + 1) // 2
    root = n - 1
    assert parent[root] == -1
    kids = np.bincount(parent[parent >= 0], minlength=n)
    assert np.all(kids[:N] == 0)
    assert np.all(kids[N:] == 2)
    for v in range(n - 1):                # every node reaches the root
        x, steps = v, 0
        while x != root:
            x = parent[x]
            steps += 1
            assert steps < n


@pytest.mark.parametrize("N", [2, 3, 16, 257, 1000])
def test_yule_is_rooted_binary(N):
    _check_tree(synth.yule_topology(N, np.random.default_rng(N)))


def test_caterpillar_is_rooted_binary():
    for N in (2, 3, 10):
        _check_tree(synth.caterpillar_topology(N))


@pytest.mark.parametrize("which", ["hky", "gtr20", "gy94"])
def test_models_reversible_normalised(which):
    rng = np.random.default_rng(3)
    if which == "hky":
        pi = rng.dirichlet([10.0] * 4)
        Q = synth.hky_model(3.0, pi)
    elif which == "gtr20":
        pi = rng.dirichlet([1.0] * 20)
        Q = synth.gtr_model(rng.gamma(1.0, 1.0, 190), pi)
    else:
        pos = np.stack([rng.dirichlet([10.0] * 4) for _ in range(3)])
        Q, pi = synth.gy94_model(0.3, 2.0, pos)
        assert Q.shape == (61, 61)
    assert np.allclose(Q.sum(1), 0, atol=1e-12)
    assert np.allclose(pi @ Q, 0, atol=1e-12)
    F = pi[:, None] * Q
    assert np.allclose(F, F.T, atol=1e-13)             # detailed balance
    assert abs(-np.dot(pi, np.diag(Q)) - 1.0) < 1e-12   # mean rate 1
    V, Vinv, lam = synth.eigensystem(Q, pi)
    assert np.allclose(V @ np.diag(lam) @ Vinv, Q, atol=1e-12)
    assert np.allclose(V @ Vinv, np.eye(len(pi)), atol=1e-12)
    assert abs(np.max(lam)) < 1e-12                    # one zero eigenvalue


def test_gy94_structure():
    pos = np.full((3, 4), 0.25)
    Q, pi = synth.gy94_model(0.5, 2.0, pos)
    codons = synth.sense_codons()
    # multi-nucleotide changes are forbidden
    s = [c for c, _ in codons].index("TTT")
    t = [c for c, _ in codons].index("GGG")
    assert Q[s, t] == 0
    # TTT (F) -> TTC (F) is a synonymous transition: rate kappa*pi; TTT->TTA (L) nonsyn transversion: omega*pi
    a = [c for c, _ in codons].index("TTC")
    b = [c for c, _ in codons].index("TTA")
    assert abs(Q[s, a] / Q[s, b] - 2.0 / 0.5) < 1e-12


@pytest.mark.parametrize("alpha", [0.2, 0.5, 2.0])
def test_discrete_gamma_mean_one(alpha):
    r, w = synth.discrete_gamma(alpha, 4)
    assert abs(np.dot(r, w) - 1.0) < 1e-12
    assert np.all(np.diff(r) > 0)


def test_simulation_frequencies_match_pi():
    rng = np.random.default_rng(5)
    pi = np.array([0.1, 0.2, 0.3, 0.4])
    Q = synth.hky_model(2.0, pi)
    parent = synth.yule_topology(8, rng)
    b = np.full(14, 5.0)                  # long branches: tips ~ stationary
    codes = synth.simulate_codes(parent, b, Q, pi, np.ones(1), np.ones(1), 20000, rng)
    freq = np.bincount(codes.ravel(), minlength=4) / codes.size
    assert np.allclose(freq, pi, atol=0.01)


def test_config_shapes():
    p = synth.config_problem("hky16", seed=0)
    assert p.codes.shape == (16, 1000) and p.b.shape == (30,)
    p = synth.config_problem("hky1000", seed=1, n_patterns=200)
    assert p.codes.shape == (1000, 200)
    frac = np.mean(p.codes == 4)
    assert 0.03 < frac < 0.07
    assert np.all(p.pattern_weights >= 1)


def test_reroot_preserves_tree_length():
    rng = np.random.default_rng(9)
    parent = synth.yule_topology(12, rng)
    b = rng.exponential(0.1, 22)
    for u in range(22):
        if parent[u] == 22:
            continue
        p2, b2, _ = synth.reroot(parent, b, u, 0.4)
        _check_tree(p2)
        assert abs(b2.sum() - b.sum()) < 1e-12
