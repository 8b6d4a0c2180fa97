"""FP64 CPU oracle for the parameter chain rules built on the branch gradient.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library.

Paper references (Gangavarapu et al., arXiv:2303.04390):
  * Methods, problem statement: a branch length is indexed by its child node
    and may be the difference between the parent's and the child's node
    heights (time units) multiplied by a possibly branch-specific rate
    scalar:  b_i = (h_parent(i) - h_i) * rho_i.
  * Gradient-kernel section, final paragraphs: for models such as a strict
    molecular clock the per-branch derivatives are further summed over a
    chosen set of branches to a single value.
  * Results (West Nile virus analysis): HMC samples branch-specific rate
    scalars and node heights, i.e. it needs d logL / d rho_i and
    d logL / d h_k.

Chain rule from g_i = d logL / d b_i (the branch-length gradient):
  d logL / d rho_i = (h_parent(i) - h_i) * g_i
  d logL / d h_k   = sum_{children c of k} rho_c g_c  -  [k not root] rho_k g_k
A set-shared rate mu_j (rho_i = mu_j for every branch i of set j) has
  d logL / d mu_j = sum_{i in set j} (h_parent(i) - h_i) * g_i.
"""
from __future__ import annotations

import numpy as np

__all__ = ["branch_lengths_from_time_tree", "time_tree_gradients", "branch_set_sums"]


def branch_lengths_from_time_tree(parent, heights, rates):
    """b_i = (h_parent(i) - h_i) * rho_i for every non-root node i."""
    parent = np.asarray(parent)
    n = parent.shape[0]
    b = np.empty(n - 1)
    for i in range(n - 1):
        b[i] = (heights[parent[i]] - heights[i]) * rates[i]
    return b


def time_tree_gradients(parent, heights, rates, grad_b):
    """(d logL / d heights (2N-1), d logL / d rates (2N-2)) by the chain rule."""
    parent = np.asarray(parent)
    n = parent.shape[0]
    d_rates = np.empty(n - 1)
    d_heights = np.zeros(n)
    for i in range(n - 1):
        k = parent[i]
        d_rates[i] = (heights[k] - heights[i]) * grad_b[i]
        # b_i grows with the parent's height and shrinks with the child's
        d_heights[k] += rates[i] * grad_b[i]
        d_heights[i] -= rates[i] * grad_b[i]
    return d_heights, d_rates


def branch_set_sums(values, set_of, n_sets):
    """out[j] = sum of values[i] over branches i with set_of[i] == j
    (set_of[i] < 0 leaves branch i out)."""
    out = np.zeros(n_sets)
    for i, j in enumerate(set_of):
        if j >= 0:
            out[j] += values[i]
    return out
