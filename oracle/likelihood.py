"""Plain FP64 CPU oracle for the tree log-likelihood and its branch gradient.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library: it takes plain numpy arrays and follows the paper's
equations step by step, in float64, with no blocking or fusion.

Paper references (Gangavarapu et al., "Many-core algorithms for
high-dimensional gradients on phylogenetic trees", arXiv:2303.04390), all in
the Methods section:
  * transition matrices  P^(r)(b_i) = exp(gamma_r b_i Q)       (Eq. for P)
  * post-order pruning   p_k = [P(b_i)] p_i o [P(b_j)] p_j      (pruning Eq.)
  * sequence likelihood  P(Y) = prod_c sum_r P(gamma_r) p_root^T pi
  * pre-order recursion  q_i = P(b_i)^T { q_k o P(b_j) p_j }, q_root = pi
                                                               (eq:preorder)
  * pre.post identity    sum_r P(gamma_r) p_i^T q_i = P(Y_c) at any node i
  * gradient             d/db_i log P(Y_c) =
         sum_r P(gamma_r) gamma_r p_i^T Q^T q_i / sum_r P(gamma_r) p_i^T q_i
                                                               (eq:gradient)
    summed over columns with their pattern weights     (eq:gradientSumAcrossColumns)

Readings where the paper is silent (each also listed in the design notes):
  * Q is rebuilt from its eigensystem, Q = V diag(lam) Vinv, the same
    eigensystem the caller passes; P(t) = V diag(exp(lam t)) Vinv.
  * Tip code S means a fully ambiguous observation (all-ones partial).
  * Underflow: the paper does not discuss it.  The oracle rescales a node's
    partials for one pattern by an exact power of two, shared across
    categories, only when their maximum drops below 2^-256, and tracks the
    integer exponent; results are bitwise those of the unscaled recursion
    whenever no rescale fires.
  * Pattern weight W_c multiplies column c's log-likelihood and derivative
    (pattern compression, Methods).
"""
from __future__ import annotations

import numpy as np

SCALE_THRESHOLD_EXP = -256          # rescale when max < 2^-256

__all__ = [
    "rate_matrix", "transition_matrices", "tree_structure", "tip_partials",
    "postorder", "site_log_likelihoods", "log_likelihood", "preorder",
    "branch_gradients", "evaluate",
]


def rate_matrix(V, Vinv, lam):
    """Q = V diag(lam) Vinv (infinitesimal generator, Methods).

    With per-category eigensystems (V [R,S,S], lam [R,S]) returns the stack
    of Q_r; the generator of category r is then gamma_r Q_r, the general
    Q^(r) the gradient-kernel section allows.
    """
    V = np.asarray(V, np.float64)
    lam = np.asarray(lam, np.float64)
    return (V * lam[..., None, :]) @ np.asarray(Vinv, np.float64)


def transition_matrices(V, Vinv, lam, rates, b):
    """P^(r)(b_x) = exp(gamma_r b_x Q) = V diag(exp(gamma_r b_x lam)) Vinv.

    Per-category eigensystems (V, Vinv [R,S,S], lam [R,S]) give
    P^(r)(b_x) = exp(gamma_r b_x Q_r).

    Returns an array [E, R, S, S] indexed by child node x and category r;
    entry [x, r, s, t] is the probability of state t at the child given s at
    the parent (Methods, equation for P).
    """
    V = np.asarray(V, np.float64)
    Vinv = np.asarray(Vinv, np.float64)
    lam = np.asarray(lam, np.float64)
    b = np.asarray(b, np.float64)
    rates = np.asarray(rates, np.float64)
    E, R, S = b.shape[0], rates.shape[0], lam.shape[-1]
    per_cat = V.ndim == 3                     # one eigensystem per category
    P = np.empty((E, R, S, S))
    for x in range(E):
        for r in range(R):
            Vr, Vir, lr = (V[r], Vinv[r], lam[r]) if per_cat else (V, Vinv, lam)
            diag = np.exp(rates[r] * b[x] * lr)
            P[x, r] = (Vr * diag[None, :]) @ Vir
    return P


def tree_structure(parent):
    """Children lists and a post-order node list (children before parents).

    The tree is the paper's rooted bifurcating graph: N tips 0..N-1, internal
    nodes N..2N-3, root 2N-2, branches indexed by their child node.
    """
    parent = np.asarray(parent)
    n = parent.shape[0]
    root = n - 1
    kids = [[] for _ in range(n)]
    for v in range(n):
        if parent[v] >= 0:
            kids[int(parent[v])].append(v)
    pre = []
    stack = [root]
    while stack:
        v = stack.pop()
        pre.append(v)
        stack.extend(sorted(kids[v], reverse=True))
    post = pre[::-1]
    return kids, post, pre


def tip_partials(codes_row, S):
    """Tip partial [C, S]: one-hot of the observed state, all-ones for code S."""
    codes_row = np.asarray(codes_row)
    C = codes_row.shape[0]
    out = np.zeros((C, S))
    obs = codes_row < S
    out[np.nonzero(obs)[0], codes_row[obs]] = 1.0
    out[~obs, :] = 1.0
    return out


def _rescale(x, exps):
    """Power-of-two rescale per column when max_{r,s} < 2^-256 (exact)."""
    mx = x.max(axis=(0, 2))                               # [C]
    need = (mx > 0) & (mx < np.ldexp(1.0, SCALE_THRESHOLD_EXP))
    if np.any(need):
        _, e = np.frexp(mx[need])
        x[:, need, :] = np.ldexp(x[:, need, :], -e[None, :, None])
        exps = exps.copy()
        exps[need] += e
    return x, exps


def postorder(parent, P, codes, S, R, tip_vectors=None):
    """Post-order (Felsenstein pruning) partials for every node.

    p_k,r,c = [P^(r)(b_i)] p_i,r,c  o  [P^(r)(b_j)] p_j,r,c   (pruning Eq.)
    A tip's partial is built from its code, or taken from tip_vectors[tip]
    ([C, S], the general tip vector of the pruning recursion) when given.
    Returns (p, E) where p[v] is [R, C, S] and the true partial equals
    p[v] * 2^E[v] (E[v] is an int64 [C] exponent vector).
    """
    kids, post, _ = tree_structure(parent)
    n = len(kids)
    n_tips = (n + 1) // 2
    C = codes.shape[1]
    p = [None] * n
    E = [None] * n
    for v in range(n_tips):
        if tip_vectors is not None and v in tip_vectors:
            tv = np.asarray(tip_vectors[v], dtype=np.float64).reshape(C, S)
        else:
            tv = tip_partials(codes[v], S)
        p[v] = np.broadcast_to(tv, (R, C, S))
        E[v] = np.zeros(C, np.int64)
    for k in post:
        if k < n_tips:
            continue
        i, j = kids[k]
        mi = np.matmul(p[i], np.swapaxes(P[i], -1, -2))   # (P_i p_i)_s = sum_t P_st p_t
        mj = np.matmul(p[j], np.swapaxes(P[j], -1, -2))
        x = mi * mj
        p[k], E[k] = _rescale(x, E[i] + E[j])
    return p, E


def site_log_likelihoods(p_root, E_root, pi, weights):
    """ln P(Y_c) = ln sum_r P(gamma_r) p_root,r,c^T pi  (+ E ln 2)."""
    s = np.einsum("r,rcs,s->c", np.asarray(weights), p_root, np.asarray(pi))
    # a site likelihood that is zero (or a round-off negative) is ln 0 = -inf
    with np.errstate(divide="ignore"):
        return np.where(s > 0, np.log(np.where(s > 0, s, 1.0)), -np.inf) + E_root * np.log(2.0)


def log_likelihood(site_ll, pattern_weights):
    """log P(Y) = sum_c W_c ln P(Y_c) over weighted unique patterns."""
    W = np.asarray(pattern_weights, np.float64)
    terms = np.where(W != 0, W * site_ll, 0.0)
    return float(np.sum(terms))


def preorder(parent, P, p, E, pi, R):
    """Pre-order partials for every node (eq:preorder).

    q_root = pi;  q_i = [P^(r)(b_i)]^T { q_k o [P^(r)(b_j)] p_j }  with k the
    parent and j the sibling of i.  Returns (q, F): true q[v] = q[v] * 2^F[v].
    """
    kids, _, pre = tree_structure(parent)
    n = len(kids)
    root = n - 1
    C = p[0].shape[1]
    S = np.asarray(pi).shape[0]
    q = [None] * n
    F = [None] * n
    q[root] = np.broadcast_to(np.asarray(pi, np.float64), (R, C, S)).copy()
    F[root] = np.zeros(C, np.int64)
    for k in pre:
        if not kids[k]:
            continue
        for i in kids[k]:
            j = [c for c in kids[k] if c != i][0]
            mj = np.matmul(p[j], np.swapaxes(P[j], -1, -2))    # P_j p_j
            u = q[k] * mj
            qi = np.matmul(u, P[i])                             # (P_i^T u)_t = sum_s P_st u_s
            q[i], F[i] = _rescale(qi, F[k] + E[j])
    return q, F


def branch_gradients(parent, Q, p, q, rates, weights, pattern_weights):
    """Per-branch gradient of log P(Y) (eq:gradient, eq:gradientSumAcrossColumns).

    d_ic = sum_r w_r gamma_r p_ir^T Q^T q_ir / sum_r w_r p_ir^T q_ir (Q_r in
    place of Q when Q is a per-category stack [R,S,S]) and
    g_i = sum_c W_c d_ic.  Also returns A_i = sum_c W_c |d_ic| (the scale of
    the cancelling sum, used to state gradient tolerances) and d itself.
    The per-node scale exponents of p and q cancel in the ratio.
    """
    n = len(p)
    Q = np.asarray(Q, np.float64)
    w = np.asarray(weights, np.float64)
    g = np.asarray(rates, np.float64)
    W = np.asarray(pattern_weights, np.float64)
    grad = np.zeros(n - 1)
    absg = np.zeros(n - 1)
    d_all = np.zeros((n - 1, W.shape[0]))
    for i in range(n - 1):
        Qtq = np.matmul(q[i], Q)                  # (Q^T q)_s = sum_t Q_ts q_t (per r for a stack)
        num = np.einsum("r,r,rcs,rcs->c", w, g, p[i], Qtq)
        den = np.einsum("r,rcs,rcs->c", w, p[i], q[i])
        with np.errstate(divide="ignore", invalid="ignore"):
            d = num / den
        d = np.where(W != 0, d, 0.0)
        d_all[i] = d
        grad[i] = float(np.sum(W * d))
        absg[i] = float(np.sum(W * np.abs(d)))
    return grad, absg, d_all


def evaluate(parent, b, V, Vinv, lam, pi, rates, weights, codes, pattern_weights,
             want_partials=False, tip_vectors=None):
    """logL and all 2N-2 branch derivatives for one instance.

    Returns a dict with keys logl, grad [2N-2], absgrad [2N-2] and site_ll [C];
    with want_partials also p, E, q, F, P.
    """
    codes = np.asarray(codes)
    S = np.asarray(lam).shape[-1]
    R = np.asarray(rates).shape[0]
    P = transition_matrices(V, Vinv, lam, rates, b)
    p, E = postorder(parent, P, codes, S, R, tip_vectors)
    root = len(p) - 1
    sll = site_log_likelihoods(p[root], E[root], pi, weights)
    logl = log_likelihood(sll, pattern_weights)
    q, F = preorder(parent, P, p, E, pi, R)
    Q = rate_matrix(V, Vinv, lam)
    grad, absg, _ = branch_gradients(parent, Q, p, q, rates, weights, pattern_weights)
    out = dict(logl=logl, grad=grad, absgrad=absg, site_ll=sll)
    if want_partials:
        out.update(p=p, E=E, q=q, F=F, P=P, Q=Q)
    return out


def evaluate_problem(prob, want_partials=False):
    """evaluate() on an object with the fields of a synthetic Problem."""
    return evaluate(prob.parent, prob.b, prob.V, prob.Vinv, prob.lam, prob.pi,
                    prob.rates, prob.weights, prob.codes, prob.pattern_weights,
                    want_partials=want_partials, tip_vectors=getattr(prob, "tip_vectors", None))
