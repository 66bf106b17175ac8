"""The rule a run selects blocks by (CPU; no GPU code involved).

With power-of-two steps, every t_i a multiple of its dt_i and every
particle due after the last block time, the block scheme's selection
(procedure step 1: T = min_i (t_i + dt_i), active = {i : t_i + dt_i = T})
reduces to: T is the first multiple of the smallest step after the last
block time, and the active particles are those whose step divides T.  The
corrector's quantiser (a step at most doubles and must divide the block
time) keeps those conditions, so ordering the particles by step size makes
every block a prefix of the order.  These tests evolve random step
hierarchies under the quantiser's rules and check each selection of the
oracle against the rule."""
import numpy as np
import pytest

from oracle import oracle as O

TB = 20


def _quantised_steps(rng, T, k_old, k_min, k_max, tb=TB):
    """New step levels for the particles of a block at time T: a random
    wish (biased towards the old level, so that deep levels stay occupied),
    then the quantiser's limits (at most doubling; T a multiple of the step,
    raising k as far as k_max)."""
    k = np.where(rng.random(k_old.shape[0]) < 0.5,
                 k_old + rng.integers(-1, 2, size=k_old.shape[0]),
                 rng.integers(k_min, k_max + 1, size=k_old.shape[0]))
    k = np.maximum(k, k_old - 1)
    k = np.clip(k, k_min, k_max)
    for q in range(k.shape[0]):
        while k[q] < k_max and T % (1 << (tb - int(k[q]))) != 0:
            k[q] += 1
    return k


@pytest.mark.parametrize("seed,n,k_min,k_max,tb", [(1, 50, 3, 12, 20), (2, 400, 0, 20, 20),
                                                   (3, 1000, 5, 9, 20), (4, 7, 10, 10, 20),
                                                   (8, 400, 3, 32, 40), (9, 60, 20, 32, 40)])
def test_selection_is_a_prefix_of_the_step_order(seed, n, k_min, k_max, tb):
    """Also at a deep hierarchy (tick_bits 40, k_max 32: steps down to 2^-32
    of the coarsest time unit)."""
    rng = np.random.default_rng(seed)
    k = rng.integers(k_min, k_max + 1, size=n)
    dt = (np.int64(1) << (tb - k)).astype(np.int64)
    t = np.zeros(n, dtype=np.int64)
    T_last = 0
    for _ in range(300):
        T, idx = O.select(t, dt)
        # the rule: first multiple of the smallest step after T_last
        dmin = int(dt.min())
        assert T == (T_last // dmin + 1) * dmin
        active = np.nonzero(T % dt == 0)[0]
        assert np.array_equal(idx, active)
        # a prefix of the order by step size, of the size the counts give
        b = np.log2(dt).astype(int)
        z = (T & -T).bit_length() - 1
        assert idx.shape[0] == np.count_nonzero(b <= z)
        if idx.shape[0] < n:
            inactive = np.setdiff1d(np.arange(n), idx)
            assert dt[idx].max() < dt[inactive].min()
        # correct the block: t = T, quantised new steps, each dividing T
        k_old = tb - b[idx]
        k_new = _quantised_steps(rng, T, k_old, k_min, k_max, tb)
        t[idx] = T
        dt[idx] = np.int64(1) << (tb - k_new)
        assert np.all(T % dt[idx] == 0)
        T_last = T


def test_rule_needs_the_grid_condition():
    """A time off its step's grid breaks the rule (the run then falls back
    to the selection from t and dt): particle 0 at t = 1 with dt = 4 is due
    at 5, not at the rule's 4."""
    t = np.array([1, 0, 0], dtype=np.int64)
    dt = np.array([4, 8, 16], dtype=np.int64)
    T, idx = O.select(t, dt)
    assert T == 5 and list(idx) == [0]
    T_last = int(t.max())
    assert (T_last // 4 + 1) * 4 == 4 != T


@pytest.mark.parametrize("seed,n,k_min,k_max,tb", [(5, 300, 2, 14, 20), (6, 2000, 0, 20, 20),
                                                   (10, 500, 4, 32, 40)])
def test_order_kept_by_resorting_the_block_only(seed, n, k_min, k_max, tb):
    """The structure a run keeps: a permutation by step size and a count per
    step size.  Each step only the previous block (a prefix) is re-sorted by
    its new steps, and the counts of the step sizes that were active are
    replaced by the block's new counts; the order stays sorted, the counts
    stay exact, and every block the oracle selects is the prefix of the
    size the counts give."""
    rng = np.random.default_rng(seed)
    k = rng.integers(k_min, k_max + 1, size=n)
    dt = (np.int64(1) << (tb - k)).astype(np.int64)
    t = np.zeros(n, dtype=np.int64)
    b = np.log2(dt).astype(int)
    perm = np.argsort(b, kind="stable")
    cnt = np.bincount(b, minlength=64)
    T_last, na_prev, T_prev = 0, 0, 0
    for _ in range(300):
        if na_prev > 0:
            z = (T_prev & -T_prev).bit_length() - 1
            blk = perm[:na_prev]
            nb = np.log2(dt[blk]).astype(int)
            perm[:na_prev] = blk[np.argsort(nb, kind="stable")]
            cnt[:z + 1] = 0
            cnt += np.bincount(nb, minlength=64)
            T_last = T_prev
        bl = np.log2(dt).astype(int)
        assert np.all(np.diff(bl[perm]) >= 0)
        assert np.array_equal(cnt, np.bincount(bl, minlength=64))
        bmin = int(np.nonzero(cnt)[0][0])
        T = ((T_last >> bmin) + 1) << bmin
        z = (T & -T).bit_length() - 1
        na = int(cnt[:z + 1].sum())
        T_o, idx = O.select(t, dt)
        assert T == T_o and np.array_equal(np.sort(perm[:na]), idx)
        k_new = _quantised_steps(rng, T, tb - bl[idx], k_min, k_max, tb)
        t[idx] = T
        dt[idx] = np.int64(1) << (tb - k_new)
        na_prev, T_prev = na, T


def _levels(dt):
    return (np.frexp(dt.astype(np.float64))[1] - 1).astype(int)


@pytest.mark.parametrize("seed,sizes,k_min,k_max,tb",
                         [(11, [40, 1, 300, 0, 77, 5], 2, 14, 20),
                          (12, [200] * 12, 0, 20, 20),
                          (13, [90, 400, 3, 250], 6, 32, 40)])
def test_ensemble_orders_per_cluster(seed, sizes, k_min, k_max, tb):
    """The ensemble form: each cluster keeps its own order in its range of
    the permutation, its step counts and their running sums; the ensemble's
    counts are kept by adding each re-sorted cluster's changes.  Each step
    every cluster re-sorts only its part of the last block; the selection
    takes the block time from the smallest occupied step of the ensemble's
    counts and cluster c's part as the prefix of its range given by its
    running sum at the block time's level, listed at the exclusive scan of
    those counts.  Checked against the oracle's
    selection over the whole ensemble, with every list position in range
    and every cluster's order sorted, through steps of a deep hierarchy
    (tick_bits 40, k_max 32) too."""
    rng = np.random.default_rng(seed)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n, C = int(off[-1]), len(sizes)
    k = rng.integers(k_min, k_max + 1, size=n)
    dt = (np.int64(1) << (tb - k)).astype(np.int64)
    t = np.zeros(n, dtype=np.int64)
    b = _levels(dt)
    perm = np.zeros(n, dtype=np.int64)
    ccnt = np.zeros((C, 64), dtype=np.int64)
    for c in range(C):
        r = np.arange(off[c], off[c + 1])
        perm[off[c]:off[c + 1]] = r[np.argsort(b[r], kind="stable")]
        ccnt[c] = np.bincount(b[r], minlength=64)
    ccum = np.cumsum(ccnt, axis=1)
    gcnt = np.bincount(b, minlength=64)      # the ensemble's counts
    cna = np.zeros(C, dtype=np.int64)
    T_last, na_prev, T_prev = int(t.max()), 0, 0
    for _ in range(300):
        # re-sort: every cluster's part of the last block, on its own range
        if na_prev > 0:
            T_last = T_prev
            z = (T_prev & -T_prev).bit_length() - 1
            for c in range(C):
                m = int(cna[c])
                if m == 0:
                    continue
                assert m <= off[c + 1] - off[c]
                blk = perm[off[c]:off[c] + m]
                nb = _levels(dt[blk])
                assert nb.max() <= z
                perm[off[c]:off[c] + m] = blk[np.argsort(nb, kind="stable")]
                old = ccnt[c].copy()
                ccnt[c, :z + 1] = 0
                ccnt[c] += np.bincount(nb, minlength=64)
                ccum[c] = np.cumsum(ccnt[c])
                gcnt += ccnt[c] - old
        bl = _levels(dt)
        for c in range(C):
            seg = bl[perm[off[c]:off[c + 1]]]
            assert np.all(np.diff(seg) >= 0)
            assert np.array_equal(ccnt[c], np.bincount(bl[off[c]:off[c + 1]], minlength=64))
            assert np.array_equal(np.sort(perm[off[c]:off[c + 1]]), np.arange(off[c], off[c + 1]))
        assert np.array_equal(gcnt, np.bincount(bl, minlength=64))
        # selection: block time, per-cluster counts and first positions
        bm = int(np.nonzero(gcnt)[0][0])
        T = ((T_last >> bm) + 1) << bm
        zn = (T & -T).bit_length() - 1
        counts = ccum[:, zn]
        start = np.concatenate([[0], np.cumsum(counts)])
        na = int(start[-1])
        idx = np.full(na, -1, dtype=np.int64)
        for c in range(C):
            cnt = int(counts[c])
            pos = start[c] + np.arange(cnt)
            assert cnt == 0 or (pos.min() >= 0 and pos.max() < na)
            idx[pos] = perm[off[c]:off[c] + cnt]
            cna[c] = cnt
        T_o, idx_o = O.select(t, dt)
        assert T == T_o
        assert np.array_equal(np.sort(idx), idx_o)
        # the list is grouped by cluster in cluster order
        cl_of = np.searchsorted(off, idx, side="right") - 1
        assert np.all(np.diff(cl_of) >= 0)
        k_new = _quantised_steps(rng, T, tb - bl[idx], k_min, k_max, tb)
        t[idx] = T
        dt[idx] = np.int64(1) << (tb - k_new)
        na_prev, T_prev = na, T
