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


def _quantised_steps(rng, T, k_old, k_min, k_max):
    """New step levels for the particles of a block at time T: a random
    wish, then the quantiser's limits (at most doubling; T a multiple of
    the step, raising k as far as k_max)."""
    k = rng.integers(k_min, k_max + 1, size=k_old.shape[0])
    k = np.maximum(k, k_old - 1)
    k = np.clip(k, k_min, k_max)
    for q in range(k.shape[0]):
        while k[q] < k_max and T % (1 << (TB - k[q])) != 0:
            k[q] += 1
    return k


@pytest.mark.parametrize("seed,n,k_min,k_max", [(1, 50, 3, 12), (2, 400, 0, 20),
                                                (3, 1000, 5, 9), (4, 7, 10, 10)])
def test_selection_is_a_prefix_of_the_step_order(seed, n, k_min, k_max):
    rng = np.random.default_rng(seed)
    k = rng.integers(k_min, k_max + 1, size=n)
    dt = (np.int64(1) << (TB - k)).astype(np.int64)
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
        k_old = TB - b[idx]
        k_new = _quantised_steps(rng, T, k_old, k_min, k_max)
        t[idx] = T
        dt[idx] = np.int64(1) << (TB - k_new)
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


@pytest.mark.parametrize("seed,n,k_min,k_max", [(5, 300, 2, 14), (6, 2000, 0, 20)])
def test_order_kept_by_resorting_the_block_only(seed, n, k_min, k_max):
    """The structure a run keeps: a permutation by step size and a count per
    step size.  Each step only the previous block (a prefix) is re-sorted by
    its new steps, and the counts of the step sizes that were active are
    replaced by the block's new counts; the order stays sorted, the counts
    stay exact, and every block the oracle selects is the prefix of the
    size the counts give."""
    rng = np.random.default_rng(seed)
    k = rng.integers(k_min, k_max + 1, size=n)
    dt = (np.int64(1) << (TB - k)).astype(np.int64)
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
        k_new = _quantised_steps(rng, T, TB - bl[idx], k_min, k_max)
        t[idx] = T
        dt[idx] = np.int64(1) << (TB - k_new)
        na_prev, T_prev = na, T
