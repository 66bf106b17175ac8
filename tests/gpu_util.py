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


def check_mixed(name, got, ref, cond, tol=TOL_MIXED, cond_factor=4.0, max_second=0):
    """Mixed parity: |d| <= tol |ref| for every particle, except that at most
    max_second of them may instead meet |d| <= cond_factor u32 sum_j |term_j|.

    cond_factor = 4: rounding the FP64 differences to FP32 alone, with all
    later arithmetic exact, stays within 4 u32 sum_j |term_j| on the N = 65536
    Plummer sample (tests/test_mixed_tolerance.py).  The default policy
    (near field in FP64, refinement of particles whose FP32 error estimate is
    large) brings every particle under tol, so callers allow the second
    clause only where a test's mode has no refinement (the paper-faithful
    mode).  Returns (n_second_clause, worst relative error)."""
    got, ref = np.atleast_2d(got), np.atleast_2d(ref)
    err = np.linalg.norm(got - ref, axis=0)
    mag = np.linalg.norm(ref, axis=0)
    bound = cond_factor * U32 * cond
    ok = (err <= tol * mag) | (err <= bound)
    rel = err / np.maximum(mag, 1e-300)
    assert np.all(ok), "%s: %d bad, worst rel %.3e" % (name, np.sum(~ok), rel.max())
    n_second = int(np.sum(err > tol * mag))
    assert n_second <= max_second, "%s: %d particles above %.0e (allowed %d), worst %.3e" % (
        name, n_second, tol, max_second, rel.max())
    return n_second, float(rel.max())


def fp32_policy(H, ctx, near_factor=3.0):
    """Makes the mixed precisions sweep every system and every block in
    FP32 (with their near field and refinement), as they do by default for
    N >= 32768 and blocks of at least 5e7 interactions; returns the previous
    policies for restore_policy."""
    saved = {p: (ctx.get_mixed_policy(p), ctx.get_mixed_small_blocks(p))
             for p in (H.MIXED, H.MIXED_2F)}
    for p in (H.MIXED, H.MIXED_2F):
        ctx.set_mixed_policy(p, near_factor, 0)
        ctx.set_mixed_small_blocks(p, 0)
    return saved


def restore_policy(ctx, saved):
    for p, ((f, b), sb) in saved.items():
        ctx.set_mixed_policy(p, f, b)
        ctx.set_mixed_small_blocks(p, sb)


def plummer_state(n, seed):
    from paper_1104_2700_amd import inputs
    x, v, m = inputs.plummer(n, seed)
    return x, v, m
