"""Helpers for the GPU parity tests: tolerances and state set-up."""
import numpy as np

U64 = 2.0 ** -53      # unit roundoff, binary64
U32 = 2.0 ** -24      # unit roundoff, binary32

# Tolerances of the two paths against the FP64 oracle (relative, per
# particle, |gpu - oracle| / |oracle|).
TOL_FP64 = 1e-13
TOL_MIXED = 1e-6


def rel_err_vec(got, ref):
    """Per-particle |got - ref| / |ref| for (3, n) arrays."""
    return np.linalg.norm(got - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)


def check_fp64(name, got, ref, cond, n_sum, tol=TOL_FP64):
    """FP64 parity: |d| <= tol |ref|, or, for particles whose sum cancels
    strongly, |d| <= 4 sqrt(N) u sum_j |term_j| (rounding-order bound).
    Returns the number of particles that needed the second clause."""
    got, ref = np.atleast_2d(got), np.atleast_2d(ref)
    err = np.linalg.norm(got - ref, axis=0)
    mag = np.linalg.norm(ref, axis=0)
    order_bound = 4.0 * np.sqrt(max(n_sum, 1)) * U64 * cond
    ok = (err <= tol * mag) | (err <= order_bound)
    assert np.all(ok), "%s: %d bad, worst rel %.3e (cond ratio %.1f)" % (
        name, np.sum(~ok), np.max(err / np.maximum(mag, 1e-300)),
        float(np.max(cond / np.maximum(mag, 1e-300))))
    return int(np.sum(err > tol * mag))


def check_mixed(name, got, ref, cond, tol=TOL_MIXED, cond_factor=16.0):
    """Mixed parity: |d| <= tol |ref|, or, where the pair sum cancels, the
    FP32 pair-arithmetic bound |d| <= cond_factor u32 sum_j |term_j|.

    cond_factor = 16: each pair term passes through about eight FP32
    roundings (<= u32/2 each, so <= 4 u32 relative per term) and a 16-term
    FP32 run sum adds <= 8 u32 of the run's absolute sum; 4 + 8 <= 16.
    Returns (n_second_clause, worst relative error)."""
    got, ref = np.atleast_2d(got), np.atleast_2d(ref)
    err = np.linalg.norm(got - ref, axis=0)
    mag = np.linalg.norm(ref, axis=0)
    bound = cond_factor * U32 * cond
    ok = (err <= tol * mag) | (err <= bound)
    rel = err / np.maximum(mag, 1e-300)
    assert np.all(ok), "%s: %d bad, worst rel %.3e" % (name, np.sum(~ok), rel.max())
    return int(np.sum(err > tol * mag)), float(rel.max())


def plummer_state(n, seed):
    from paper_1104_2700_amd import inputs
    x, v, m = inputs.plummer(n, seed)
    return x, v, m
