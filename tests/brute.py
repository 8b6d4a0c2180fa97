"""Independent checks used to pin the oracle (tests only).

Nothing here calls the oracle.  Transition matrices come from
scipy.linalg.expm of gamma_r * b * Q on the generator Q itself, and the
likelihood is the plain definition: a sum over every assignment of states to
the internal nodes of the product of the root prior and one transition
probability per branch (Methods, sequence-likelihood equation before pruning
is applied).
"""
import itertools

import numpy as np
import scipy.linalg


def expm_P(Q, rates, b):
    """P, dP/db for every (branch, category); Q may be one generator [S,S] or
    one per category [R,S,S] (category r then evolves under rates[r] * Q[r])."""
    Q = np.asarray(Q)
    E, R, S = len(b), len(rates), Q.shape[-1]
    P = np.empty((E, R, S, S))
    dP = np.empty((E, R, S, S))
    for x in range(E):
        for r in range(R):
            Qr = Q[r] if Q.ndim == 3 else Q
            M = scipy.linalg.expm(rates[r] * b[x] * Qr)
            P[x, r] = M
            dP[x, r] = rates[r] * (Qr @ M)
    return P, dP


def brute_site_likelihood(parent, P, codes, pi, weights, deriv_branch=None, dP=None, tip_vectors=None):
    """L_c = sum_r w_r sum_{internal states} pi_root prod_branches P[x][s_par, s_x].

    Tip x with code y contributes P[x][s_par, y]; code S (ambiguous) sums over
    the unobserved tip state.  A tip with a general vector v (tip_vectors[x],
    [C, S]) contributes sum_t P[x][s_par, t] v[c, t]: its state summed out,
    weighted by v.  With deriv_branch, that branch's factor uses dP instead of
    P, giving d L_c / d b_x.
    Returns [C] site values.
    """
    n = len(parent)
    n_tips = (n + 1) // 2
    root = n - 1
    S = len(pi)
    R = len(weights)
    C = codes.shape[1]
    internal = list(range(n_tips, n))
    total = np.zeros(C)
    for r in range(R):
        acc = np.zeros(C)
        for assign in itertools.product(range(S), repeat=len(internal)):
            st = dict(zip(internal, assign))
            val = np.full(C, pi[st[root]])
            for x in range(n - 1):
                M = (dP if x == deriv_branch else P)[x, r]
                sp = st[int(parent[x])]
                if x < n_tips and tip_vectors is not None and x in tip_vectors:
                    fac = np.asarray(tip_vectors[x]) @ M[sp]
                elif x < n_tips:
                    y = codes[x]
                    row = M[sp]
                    fac = np.where(y < S, row[np.minimum(y, S - 1)], row.sum())
                else:
                    fac = M[sp, st[x]]
                val = val * fac
            acc += val
        total += weights[r] * acc
    return total


def pruning_site_likelihood(parent, P, codes, pi, weights, deriv_branch=None, dP=None):
    """Felsenstein pruning written independently of the oracle (recursive),
    with branch ``deriv_branch`` using dP: the O(N^2) per-branch derivative
    scheme the paper contrasts with the linear-time method."""
    n = len(parent)
    n_tips = (n + 1) // 2
    S = len(pi)
    kids = {v: [] for v in range(n)}
    for v in range(n - 1):
        kids[int(parent[v])].append(v)
    C = codes.shape[1]
    R = len(weights)
    out = np.zeros(C)
    for r in range(R):
        def part(v):
            if v < n_tips:
                y = codes[v]
                m = np.zeros((C, S))
                ok = y < S
                m[np.nonzero(ok)[0], y[ok]] = 1.0
                m[~ok] = 1.0
                return m
            acc = np.ones((C, S))
            for x in kids[v]:
                M = (dP if x == deriv_branch else P)[x, r]
                acc = acc * (part(x) @ M.T)
            return acc
        out += weights[r] * (part(n - 1) @ pi)
    return out
