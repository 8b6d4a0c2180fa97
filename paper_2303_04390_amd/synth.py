"""Seeded synthetic inputs for the phylogenetic likelihood-gradient path.

This module only *prepares inputs*: tree shapes, branch lengths, substitution
models in eigen-decomposed form, discrete-Gamma rate categories, simulated
alignments, pattern weights and tip ambiguity.  It holds none of the
likelihood, pre-order or gradient arithmetic, so the FP64 oracle and the HIP
path can both be fed from it without sharing any of the method's code.

Conventions (the paper's Methods section, labelling paragraph): a rooted
bifurcating tree with N tips labelled 0..N-1, internal nodes N..2N-3 and the
root 2N-2 (0-based versions of the paper's 1..2N-1).  Every non-root node x
owns the branch to its parent, so branch lengths and gradients are indexed by
child node and have length 2N-2.

Substitution models are reversible: Q_st = X_st * pi_t for s != t with a
symmetric exchangeability matrix X, rows summing to zero and normalised to one
expected substitution per unit time (-sum_s pi_s Q_ss = 1).  The eigensystem is
taken from the symmetric form Pi^(1/2) Q Pi^(-1/2) = U diag(lam) U^T, giving
Q = V diag(lam) Vinv with V = Pi^(-1/2) U and Vinv = U^T Pi^(1/2).

Simulated sites use scipy.linalg.expm for the transition matrices, a library
routine that neither the oracle nor the GPU path uses.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.linalg
import scipy.special

__all__ = [
    "Problem", "yule_topology", "exponential_branch_lengths", "hky_model",
    "gtr_model", "gy94_model", "eigensystem", "discrete_gamma", "simulate_codes",
    "make_problem", "config_problem", "sense_codons", "reroot", "time_tree",
    "category_models",
]

NUC = "ACGT"


@dataclasses.dataclass
class Problem:
    """One likelihood-plus-gradient instance (all host-side numpy arrays).

    parent : int32 [2N-1]   parent[root] = -1, root = 2N-2
    b      : float64 [2N-2] branch length of the branch above each non-root node
    V, Vinv: float64 [S,S]  row-major eigenvectors, Q = V diag(lam) Vinv
             (or [R,S,S] with lam [R,S]: one model Q_r per rate category)
    lam    : float64 [S]    eigenvalues (real, one of them 0)
    pi     : float64 [S]    root distribution (stationary here)
    rates  : float64 [R]    category rate multipliers gamma_r
    weights: float64 [R]    category probabilities P(gamma_r)
    codes  : int32 [N, C]   tip states 0..S-1, or S for a fully ambiguous entry
    pattern_weights: float64 [C]
    Q      : float64 [S,S]  the generator itself (for tests and simulation; [R,S,S] per category)
    tip_vectors: optional {tip: float64 [C,S]} general tip partial vectors
             that replace those tips' codes
    """
    parent: np.ndarray
    b: np.ndarray
    V: np.ndarray
    Vinv: np.ndarray
    lam: np.ndarray
    pi: np.ndarray
    rates: np.ndarray
    weights: np.ndarray
    codes: np.ndarray
    pattern_weights: np.ndarray
    Q: np.ndarray
    name: str = ""
    tip_vectors: Optional[dict] = None

    @property
    def n_tips(self) -> int:
        return (self.parent.shape[0] + 1) // 2

    @property
    def n_patterns(self) -> int:
        return self.codes.shape[1]

    @property
    def n_states(self) -> int:
        return self.pi.shape[0]

    @property
    def n_categories(self) -> int:
        return self.rates.shape[0]

    def subset_patterns(self, idx) -> "Problem":
        """Same tree and model restricted to the given pattern columns."""
        return dataclasses.replace(
            self, codes=np.ascontiguousarray(self.codes[:, idx]),
            pattern_weights=np.ascontiguousarray(self.pattern_weights[idx]))


# ---------------------------------------------------------------- topology

def yule_topology(n_tips: int, rng: np.random.Generator,
                  shuffle_internal: bool = True) -> np.ndarray:
    """Pure-birth (Yule) rooted binary topology.

    Start from a root with two tips and repeatedly split a uniformly chosen
    current tip into a cherry until n_tips tips exist.  Tips are relabelled
    0..N-1, internal nodes N..2N-3 (in a random order when shuffle_internal,
    so nothing downstream can rely on a label order) and the root 2N-2.
    """
    if n_tips < 2:
        raise ValueError("a rooted binary tree needs at least 2 tips")
    # build with provisional ids; node 0 is the root
    par = [-1, 0, 0]
    tips = [1, 2]
    while len(tips) < n_tips:
        k = int(rng.integers(len(tips)))
        node = tips[k]
        a, b_ = len(par), len(par) + 1
        par.extend([node, node])
        tips[k] = a
        tips.append(b_)
    n_nodes = 2 * n_tips - 1
    assert len(par) == n_nodes
    is_tip = np.zeros(n_nodes, bool)
    is_tip[tips] = True
    internal = [v for v in range(1, n_nodes) if not is_tip[v]]
    if shuffle_internal:
        internal = [internal[i] for i in rng.permutation(len(internal))]
    tip_order = [tips[i] for i in rng.permutation(len(tips))]
    label = np.empty(n_nodes, np.int64)
    label[tip_order] = np.arange(n_tips)
    label[internal] = n_tips + np.arange(len(internal))
    label[0] = 2 * n_tips - 2
    parent = np.full(n_nodes, -1, np.int32)
    for v in range(1, n_nodes):
        parent[label[v]] = label[par[v]]
    return parent


def caterpillar_topology(n_tips: int) -> np.ndarray:
    """Fully unbalanced ("caterpillar") rooted tree: depth n_tips-1."""
    n_nodes = 2 * n_tips - 1
    parent = np.full(n_nodes, -1, np.int32)
    root = n_nodes - 1
    # internal chain: root -> N+? ... ; attach tip t to chain node
    chain = [root] + list(range(2 * n_tips - 3, n_tips - 1, -1))
    for d, node in enumerate(chain):
        if d + 1 < len(chain):
            parent[chain[d + 1]] = node
            parent[d] = node
        else:
            parent[d] = node
            parent[d + 1] = node
    return parent


def exponential_branch_lengths(n_tips: int, mean: float,
                               rng: np.random.Generator) -> np.ndarray:
    return rng.exponential(mean, size=2 * n_tips - 2)


def time_tree(parent: np.ndarray, rng: np.random.Generator, mean_interval: float = 0.02,
              tip_spread: float = 0.05, rate_median: float = 1.0, rate_sigma: float = 0.3):
    """Node heights and branch rate scalars for a topology (a dated tree with
    an uncorrelated log-normal relaxed clock).

    Tips are sampled at heights U[0, tip_spread] (heterochronous data); an
    internal node sits Exponential(mean_interval) above its higher child; each
    branch gets a rate scalar LogNormal(log rate_median, rate_sigma).
    Returns (heights [2N-1], rates [2N-2]), indexed by node / child node.
    """
    n = parent.shape[0]
    N = (n + 1) // 2
    heights = np.zeros(n)
    heights[:N] = rng.uniform(0.0, tip_spread, N)
    kids = [[] for _ in range(n)]
    for v in range(n - 1):
        kids[parent[v]].append(v)
    for v in reversed(_children_order(parent)):       # children before parents
        if v >= N:
            heights[v] = max(heights[c] for c in kids[v]) + rng.exponential(mean_interval)
    rates = rate_median * np.exp(rng.normal(0.0, rate_sigma, n - 1))
    return heights, rates


def reroot(parent: np.ndarray, b: np.ndarray, new_edge_child: int,
           fraction: float = 0.5):
    """Move the root onto the branch above ``new_edge_child``.

    The old root (degree 2) is suppressed: its two branches merge into one.
    The new root splits the chosen branch at ``fraction`` of its length.
    Returns (parent2, b2, mapping) where mapping[old_node] = new_node for every
    surviving node, and the root keeps label 2N-2.  Used by the re-rooting
    invariance (pulley) checks.
    """
    n_nodes = parent.shape[0]
    n_tips = (n_nodes + 1) // 2
    root = n_nodes - 1
    adj = {v: [] for v in range(n_nodes)}
    for v in range(n_nodes):
        if parent[v] >= 0:
            adj[v].append((int(parent[v]), float(b[v])))
            adj[int(parent[v])].append((v, float(b[v])))
    # suppress old root
    (a, la), (c, lc) = adj[root]
    adj[a] = [(x, l) for (x, l) in adj[a] if x != root] + [(c, la + lc)]
    adj[c] = [(x, l) for (x, l) in adj[c] if x != root] + [(a, la + lc)]
    del adj[root]
    u = int(new_edge_child)
    if u == root:
        raise ValueError("cannot reroot on the root")
    w = int(parent[u])
    if w == root:
        w = c if u == a else a
    luw = [l for (x, l) in adj[u] if x == w][0]
    new = root  # reuse the label for the new root
    adj[u] = [(x, l) for (x, l) in adj[u] if x != w] + [(new, fraction * luw)]
    adj[w] = [(x, l) for (x, l) in adj[w] if x != u] + [(new, (1 - fraction) * luw)]
    adj[new] = [(u, fraction * luw), (w, (1 - fraction) * luw)]
    parent2 = np.full(n_nodes, -1, np.int32)
    b2 = np.zeros(n_nodes - 1)
    stack = [new]
    seen = {new}
    while stack:
        v = stack.pop()
        for x, l in adj[v]:
            if x not in seen:
                seen.add(x)
                parent2[x] = v
                b2[x] = l
                stack.append(x)
    assert len(seen) == n_nodes
    mapping = np.arange(n_nodes)
    return parent2, b2, mapping


# ---------------------------------------------------------------- models

def _normalise(Q: np.ndarray, pi: np.ndarray) -> np.ndarray:
    np.fill_diagonal(Q, 0.0)
    np.fill_diagonal(Q, -Q.sum(axis=1))
    mu = -float(np.dot(pi, np.diag(Q)))
    return Q / mu


def reversible_q(exch: np.ndarray, pi: np.ndarray) -> np.ndarray:
    """Q_st = exch_st * pi_t (s != t), rows sum to 0, mean rate 1."""
    exch = np.asarray(exch, float)
    assert np.allclose(exch, exch.T)
    Q = exch * pi[None, :]
    return _normalise(Q, pi)


def hky_model(kappa: float, pi: np.ndarray) -> np.ndarray:
    """HKY85 in state order A, C, G, T: transitions (A<->G, C<->T) x kappa."""
    exch = np.ones((4, 4))
    exch[0, 2] = exch[2, 0] = kappa
    exch[1, 3] = exch[3, 1] = kappa
    return reversible_q(exch, np.asarray(pi, float))


def gtr_model(exch_upper: np.ndarray, pi: np.ndarray) -> np.ndarray:
    S = pi.shape[0]
    exch = np.zeros((S, S))
    iu = np.triu_indices(S, 1)
    exch[iu] = exch_upper
    exch = exch + exch.T
    return reversible_q(exch, np.asarray(pi, float))


# universal (standard) genetic code, bases in T, C, A, G order per position
_CODE_TCAG = "FFLLSSSSYY**CC*WLLLLPPPPHHQQRRRRIIIMTTTTNNKKSSRRVVVVAAAADDEEGGGG"


def sense_codons():
    """The 61 sense codons of the standard code as (codon string, amino acid)."""
    order = "TCAG"
    out = []
    for i, a in enumerate(order):
        for j, b_ in enumerate(order):
            for k, c in enumerate(order):
                aa = _CODE_TCAG[16 * i + 4 * j + k]
                if aa != "*":
                    out.append((a + b_ + c, aa))
    assert len(out) == 61
    return out


def _is_transition(x: str, y: str) -> bool:
    return {x, y} in ({"A", "G"}, {"C", "T"})


def gy94_model(omega: float, kappa: float, pos_freqs: np.ndarray):
    """Goldman-Yang 1994 codon model on the 61 sense codons, F3x4 frequencies.

    pos_freqs: [3, 4] nucleotide frequencies per codon position (A, C, G, T).
    Returns (Q, pi) with pi the normalised F3x4 codon frequencies.
    """
    codons = sense_codons()
    idx = {c: n for n, c in enumerate(NUC)}
    pi = np.array([np.prod([pos_freqs[p, idx[c[p]]] for p in range(3)])
                   for c, _ in codons])
    pi = pi / pi.sum()
    S = len(codons)
    exch = np.zeros((S, S))
    for s, (cs, as_) in enumerate(codons):
        for t, (ct, at) in enumerate(codons):
            if s == t:
                continue
            diff = [p for p in range(3) if cs[p] != ct[p]]
            if len(diff) != 1:
                continue
            p = diff[0]
            v = kappa if _is_transition(cs[p], ct[p]) else 1.0
            if as_ != at:
                v *= omega
            exch[s, t] = v
    return reversible_q(exch, pi), pi


def eigensystem(Q: np.ndarray, pi: np.ndarray):
    """Eigen-decomposition of a reversible generator via its symmetric form."""
    sq = np.sqrt(pi)
    A = sq[:, None] * Q / sq[None, :]
    A = 0.5 * (A + A.T)
    lam, U = np.linalg.eigh(A)
    V = U / sq[:, None]
    Vinv = U.T * sq[None, :]
    return np.ascontiguousarray(V), np.ascontiguousarray(Vinv), lam


def category_models(S: int, R: int, rng: np.random.Generator, spread: float = 1.0):
    """One reversible model per rate category (general Q^(r)): GTR with its own
    exchangeabilities ~Gamma(1/spread-ish) and frequencies ~Dir(4) for S = 4,
    ~Dir(2) otherwise.  Returns (Qs [R,S,S], V [R,S,S], Vinv [R,S,S],
    lam [R,S]), each category's eigensystem from its symmetric form."""
    Qs, Vs, Vis, ls = [], [], [], []
    for _ in range(R):
        pi = rng.dirichlet([4.0 if S == 4 else 2.0] * S)
        pi = np.maximum(pi, 1e-3)
        pi /= pi.sum()
        Q = gtr_model(rng.gamma(1.0 / spread, spread, S * (S - 1) // 2), pi)
        V, Vinv, lam = eigensystem(Q, pi)
        Qs.append(Q)
        Vs.append(V)
        Vis.append(Vinv)
        ls.append(lam)
    return np.stack(Qs), np.stack(Vs), np.stack(Vis), np.stack(ls)


def discrete_gamma(alpha: float, n_cat: int):
    """Yang (1994) discrete Gamma, mean-of-category rates, equal weights.

    Category boundaries are the k/R quantiles of Gamma(shape=alpha,
    rate=alpha); each rate is the conditional mean within its category,
    R * [I(alpha+1, alpha*x_hi) - I(alpha+1, alpha*x_lo)], so the mean rate
    is exactly 1.
    """
    if n_cat == 1:
        return np.ones(1), np.ones(1)
    q = np.arange(1, n_cat) / n_cat
    x = scipy.special.gammaincinv(alpha, q) / alpha
    cdf1 = np.concatenate([[0.0], scipy.special.gammainc(alpha + 1, alpha * x), [1.0]])
    rates = n_cat * np.diff(cdf1)
    rates = rates / rates.mean()
    return rates, np.full(n_cat, 1.0 / n_cat)


# ---------------------------------------------------------------- simulation

def _children_order(parent: np.ndarray):
    """Nodes in an order where each parent precedes its children."""
    n = parent.shape[0]
    root = n - 1
    kids = [[] for _ in range(n)]
    for v in range(n):
        if parent[v] >= 0:
            kids[parent[v]].append(v)
    order, stack = [], [root]
    while stack:
        v = stack.pop()
        order.append(v)
        stack.extend(kids[v])
    return order


def simulate_codes(parent, b, Q, pi, rates, weights, n_sites,
                   rng: np.random.Generator) -> np.ndarray:
    """Simulate n_sites i.i.d. sites down the tree; returns tip states [N, C].

    Each site draws a category r ~ weights and a root state ~ pi, then each
    child state is drawn from row (parent state) of expm(gamma_r * b * Q).
    """
    n_nodes = parent.shape[0]
    n_tips = (n_nodes + 1) // 2
    S = Q.shape[0]
    R = rates.shape[0]
    cat = rng.choice(R, size=n_sites, p=weights)
    states = np.empty((n_nodes, n_sites), np.int32)
    root = n_nodes - 1
    states[root] = rng.choice(S, size=n_sites, p=pi)
    # all transition matrices at once (scipy's expm accepts stacked matrices)
    t = (np.asarray(b, float)[:, None] * np.asarray(rates, float)[None, :]).reshape(-1)
    P = scipy.linalg.expm(t[:, None, None] * Q[None, :, :]).reshape(n_nodes - 1, R, S, S)
    P = np.clip(P, 0.0, None)
    P /= P.sum(axis=-1, keepdims=True)
    cum = np.cumsum(P, axis=-1)
    for v in _children_order(parent):
        if v == root:
            continue
        u = rng.random(n_sites)
        rows = cum[v][cat, states[parent[v]]]          # [C, S]
        states[v] = np.minimum((u[:, None] >= rows).sum(axis=1), S - 1)
    return np.ascontiguousarray(states[:n_tips])


# ---------------------------------------------------------------- configs

def make_problem(parent, b, Q, pi, rates, weights, n_patterns, rng,
                 pattern_weights=None, ambiguous_fraction=0.0, name="") -> Problem:
    codes = simulate_codes(parent, b, Q, pi, rates, weights, n_patterns, rng)
    S = Q.shape[0]
    if ambiguous_fraction > 0:
        mask = rng.random(codes.shape) < ambiguous_fraction
        codes[mask] = S
    if pattern_weights is None:
        pattern_weights = np.ones(n_patterns)
    V, Vinv, lam = eigensystem(Q, pi)
    return Problem(parent=np.ascontiguousarray(parent, np.int32),
                   b=np.ascontiguousarray(b, float), V=V, Vinv=Vinv, lam=lam,
                   pi=np.ascontiguousarray(pi, float),
                   rates=np.ascontiguousarray(rates, float),
                   weights=np.ascontiguousarray(weights, float),
                   codes=np.ascontiguousarray(codes, np.int32),
                   pattern_weights=np.ascontiguousarray(pattern_weights, float),
                   Q=Q, name=name)


def config_problem(which: str, seed: int = 0, n_patterns: Optional[int] = None,
                   n_tips: Optional[int] = None) -> Problem:
    """The workload shapes the benchmarks and parity tests use.

    "hky16":    16 taxa, b~Exp(0.1), HKY kappa=2, pi~Dir(10^4), Gamma4 a=0.5,
                1000 simulated patterns, unit weights, no ambiguity.
    "hky1000":  1000 taxa, b~Exp(0.01), HKY kappa~U[1,5], Gamma4 a~U[0.2,2],
                pi~Dir(10^4), 10,000 patterns, weights 1+Poisson(3), 5% of the
                (tip, pattern) entries fully ambiguous.
    "aa500":    500 taxa, 20-state reversible model, exchangeabilities
                ~Gamma(1,1), pi~Dir(1^20), Gamma4 a=0.5, b~Exp(0.05), 5000 patterns.
    "codon128": 128 taxa, b~Exp(0.05), GY94 omega=0.3 kappa=2, F3x4 with
                per-position Dir(10^4), Gamma4 a=0.5, 4000 patterns.
    "s122":     128 taxa, b~Exp(0.05), 122-state GTR (exchangeabilities
                ~Gamma(1,1), pi~Dir(2^122)), Gamma4 a=0.5, 2000 patterns (the
                size of a Markov-modulated codon model).
    "s240":     as "s122" with 240 states and 1000 patterns (near the
                256-state models the paper's Discussion names).
    "s256big":  10,000 taxa, b~Exp(0.05), 256-state GTR as "s122", Gamma4
                a=0.5, 256 patterns of uniformly drawn tip states (not
                simulated: a throughput shape for 20,000 branches at 256
                states, where simulating down the tree would take minutes).
    ``n_patterns``/``n_tips`` override the sizes (smaller parity cases).
    """
    rng = np.random.default_rng(seed)
    if which == "hky16":
        N, C = n_tips or 16, n_patterns or 1000
        parent = yule_topology(N, rng)
        b = exponential_branch_lengths(N, 0.1, rng)
        pi = rng.dirichlet([10.0] * 4)
        Q = hky_model(2.0, pi)
        rates, w = discrete_gamma(0.5, 4)
        return make_problem(parent, b, Q, pi, rates, w, C, rng, name=which)
    if which == "hky1000":
        N, C = n_tips or 1000, n_patterns or 10000
        parent = yule_topology(N, rng)
        b = exponential_branch_lengths(N, 0.01, rng)
        kappa = rng.uniform(1.0, 5.0)
        alpha = rng.uniform(0.2, 2.0)
        pi = rng.dirichlet([10.0] * 4)
        Q = hky_model(kappa, pi)
        rates, w = discrete_gamma(alpha, 4)
        pw = 1.0 + rng.poisson(3.0, size=C)
        return make_problem(parent, b, Q, pi, rates, w, C, rng,
                            pattern_weights=pw, ambiguous_fraction=0.05, name=which)
    if which == "aa500":
        N, C = n_tips or 500, n_patterns or 5000
        parent = yule_topology(N, rng)
        b = exponential_branch_lengths(N, 0.05, rng)
        pi = rng.dirichlet([1.0] * 20)
        pi = np.maximum(pi, 1e-4)
        pi = pi / pi.sum()
        exch = rng.gamma(1.0, 1.0, size=190)
        Q = gtr_model(exch, pi)
        rates, w = discrete_gamma(0.5, 4)
        return make_problem(parent, b, Q, pi, rates, w, C, rng, name=which)
    if which == "codon128":
        N, C = n_tips or 128, n_patterns or 4000
        parent = yule_topology(N, rng)
        b = exponential_branch_lengths(N, 0.05, rng)
        pos = np.stack([rng.dirichlet([10.0] * 4) for _ in range(3)])
        Q, pi = gy94_model(0.3, 2.0, pos)
        rates, w = discrete_gamma(0.5, 4)
        return make_problem(parent, b, Q, pi, rates, w, C, rng, name=which)
    if which in ("s122", "s240"):
        S = 122 if which == "s122" else 240
        N, C = n_tips or 128, n_patterns or (2000 if S == 122 else 1000)
        parent = yule_topology(N, rng)
        b = exponential_branch_lengths(N, 0.05, rng)
        pi = rng.dirichlet([2.0] * S)
        Q = gtr_model(rng.gamma(1.0, 1.0, S * (S - 1) // 2), pi)
        rates, w = discrete_gamma(0.5, 4)
        return make_problem(parent, b, Q, pi, rates, w, C, rng, name=which)
    if which == "s256big":
        S = 256
        N, C = n_tips or 10000, n_patterns or 256
        parent = yule_topology(N, rng)
        b = exponential_branch_lengths(N, 0.05, rng)
        pi = rng.dirichlet([2.0] * S)
        Q = gtr_model(rng.gamma(1.0, 1.0, S * (S - 1) // 2), pi)
        rates, w = discrete_gamma(0.5, 4)
        V, Vinv, lam = eigensystem(Q, pi)
        return Problem(parent=parent, b=b, V=V, Vinv=Vinv, lam=lam, pi=pi, rates=rates, weights=w,
                       codes=rng.integers(0, S, (N, C)).astype(np.int32), pattern_weights=np.ones(C),
                       Q=Q, name=which)
    raise ValueError(f"unknown config {which!r}")


def serving_stream(seed: int, n_requests: int, rate_per_s: float = 500.0,
                   taxa=(64, 4096), patterns=(500, 20000), reuse=0.5,
                   sigma=0.05, max_tips=None, max_patterns=None):
    """Request stream for the serving loop (HMC-like arrivals).

    Poisson arrivals; each request is either a new Yule tree (HKY+Gamma4 drawn
    as in "hky1000", taxa and patterns log-uniform in the given ranges) or,
    with probability ``reuse``, a branch-length perturbation b*exp(N(0,sigma))
    of an earlier tree.  Yields dicts with arrival time, tree key, problem and
    (for perturbations) the new branch lengths.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    trees: List[Problem] = []
    out = []
    for n in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        if trees and rng.random() < reuse:
            k = int(rng.integers(len(trees)))
            base = trees[k]
            b = base.b * np.exp(rng.normal(0.0, sigma, size=base.b.shape))
            out.append(dict(arrival=t, tree=k, b=b))
            continue
        lo, hi = taxa
        N = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        lo, hi = patterns
        C = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        if max_tips:
            N = min(N, max_tips)
        if max_patterns:
            C = min(C, max_patterns)
        p = config_problem("hky1000", seed=int(rng.integers(1 << 31)),
                           n_tips=N, n_patterns=C)
        trees.append(p)
        out.append(dict(arrival=t, tree=len(trees) - 1, b=p.b))
    return trees, out
