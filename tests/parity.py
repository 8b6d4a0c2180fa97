"""Tolerance rules for comparing the HIP path with the FP64 oracle.

log-likelihood: relative error |l - l*| / |l*|.
gradient component x: |g_x - g*_x| <= tol * max(|g*_x|, 1e-2 * A_x), where
A_x = sum_c W_c |d_xc| is the scale of the cancelling per-pattern sum the
component is made of (a component that is nearly zero by cancellation is
judged against 1% of that scale).  A component with A_x = 0 must be zero to
1e-12 absolute.
"""
import sys

import numpy as np


def grad_errors(grad, ref):
    g, gs, A = np.asarray(grad), ref["grad"], ref["absgrad"]
    denom = np.maximum(np.abs(gs), 1e-2 * A)
    err = np.abs(g - gs)
    rel = np.where(denom > 0, err / np.where(denom > 0, denom, 1.0), np.where(err <= 1e-12, 0.0, np.inf))
    floor_used = int(np.sum(1e-2 * A > np.abs(gs)))
    pure = np.abs(g - gs) / np.maximum(np.abs(gs), 1e-300)
    return rel, floor_used, pure


def check(name, logl, grad, ref, tol_ll, tol_g):
    rel_ll = abs(logl - ref["logl"]) / abs(ref["logl"])
    rel, floor_used, pure = grad_errors(grad, ref)
    worst = int(np.argmax(rel))
    print(f"[parity] {name}: logL rel err {rel_ll:.3e} (tol {tol_ll:.0e}); grad max scaled err "
          f"{rel.max():.3e} (tol {tol_g:.0e}) at branch {worst}; floor used by {floor_used}/"
          f"{len(rel)}; max pure rel err {pure.max():.3e}, {int(np.sum(pure > tol_g))} components "
          f"above {tol_g:.0e} pure relative", flush=True)
    sys.stdout.flush()
    assert np.isfinite(logl)
    assert rel_ll <= tol_ll, (name, rel_ll)
    assert rel.max() <= tol_g, (name, worst, grad[worst], ref["grad"][worst], ref["absgrad"][worst])
    return rel_ll, rel.max()
