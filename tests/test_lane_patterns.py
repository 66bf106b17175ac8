"""The cross-lane patterns of the sweep's butterflies and the wave scans,
modelled on the CPU lane by lane (64 lanes, 16-lane rows, DPP as the GCN
ISA defines its quad permutes, row mirrors, row shifts and row broadcasts):

* the butterfly that takes its in-row partners from quad permutes and the
  half-row and row mirrors gives every lane bit for bit what the xor
  butterfly gives, for any group size L (the lanes of an aligned group of
  2 O hold equal values after each step, so any partner in the other half
  of the group adds the same value);
* the DPP inclusive scan (row shifts 1, 2, 4, 8 with zero past the row
  start, then the row-15 broadcast into rows 1 and 3 and the row-31
  broadcast into rows 2 and 3) equals the prefix sum.

This checks the reasoning behind the kernels' lane moves; the GPU tests
check the kernels themselves."""
import numpy as np

W = 64


def quad_perm(v, perm):
    out = v.copy()
    for i in range(W):
        out[i] = v[(i & ~3) + perm[i & 3]]
    return out


def half_row_mirror(v):
    return np.array([v[(i & ~7) + 7 - (i & 7)] for i in range(W)], dtype=v.dtype)


def row_mirror(v):
    return np.array([v[(i & ~15) + 15 - (i & 15)] for i in range(W)], dtype=v.dtype)


def xor_lane(v, o):
    return np.array([v[i ^ o] for i in range(W)], dtype=v.dtype)


def row_shr(v, k):
    # bound_ctrl: a lane whose source lies before its row's start reads 0
    return np.array([v[i - k] if (i & 15) >= k else 0 for i in range(W)], dtype=v.dtype)


def row_bcast(v, src_lane_in_row, row_mask):
    # lanes of the rows enabled by row_mask read the given lane of the row
    # below (row_bcast:15: lane 15 of row r-1; row_bcast:31: lane 31)
    out = np.zeros_like(v)
    for i in range(W):
        r = i >> 4
        if row_mask >> r & 1:
            out[i] = v[15 + 16 * (r - 1)] if src_lane_in_row == 15 else v[31]
    return out


DPP_PARTNER = {
    1: lambda v: quad_perm(v, [1, 0, 3, 2]),
    2: lambda v: quad_perm(v, [2, 3, 0, 1]),
    4: half_row_mirror,
    8: row_mirror,
}


def butterfly(v, L, partner):
    v = v.copy()
    o = 1
    while o < L:
        v = v + partner(v, o)
        o <<= 1
    return v


def test_dpp_butterfly_equals_xor_butterfly_bitwise():
    rng = np.random.default_rng(7)
    for L in (1, 2, 4, 8, 16, 32, 64):
        for _ in range(50):
            v = rng.standard_normal(W) * 10.0 ** rng.integers(-8, 8, W)
            ref = butterfly(v, L, xor_lane)
            got = butterfly(v, L, lambda x, o: DPP_PARTNER[o](x) if o < 16 else xor_lane(x, o))
            assert np.array_equal(ref.view(np.int64), got.view(np.int64)), L
            # every lane of an aligned group of L holds the group's sum
            for g in range(0, W, L):
                assert np.all(got[g:g + L] == got[g])


def test_dpp_min_and_max_reductions():
    rng = np.random.default_rng(8)
    for _ in range(50):
        v = rng.integers(-2**62, 2**62, W)
        mn, mx = v.copy(), v.copy()
        o = 1
        while o < W:
            p = DPP_PARTNER[o] if o < 16 else (lambda x, o=o: xor_lane(x, o))
            mn = np.minimum(mn, p(mn))
            mx = np.maximum(mx, p(mx))
            o <<= 1
        assert np.all(mn == v.min()) and np.all(mx == v.max())


def test_dpp_inclusive_scan():
    rng = np.random.default_rng(9)
    for _ in range(100):
        x = rng.integers(0, 1 << 20, W).astype(np.int64)
        y = x.copy()
        for k in (1, 2, 4, 8):
            y = y + row_shr(y, k)
        y = y + row_bcast(y, 15, 0xA)
        y = y + row_bcast(y, 31, 0xC)
        assert np.array_equal(y, np.cumsum(x))
