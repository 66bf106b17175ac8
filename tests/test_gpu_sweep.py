"""GPU force/jerk/potential sweep vs the FP64 CPU oracle, through the C ABI.

Equations (acc), (jrk), (pot) of Section 2.  Sizes span several LDS tiles,
ragged tails, tiny and empty active lists, random non-contiguous index
lists, and the full N = 65536 Plummer sweep on a 1024-particle sample and
on every particle.  The mixed precisions are held to 1e-6 relative on
every particle (acc, jerk and pot): they sweep in FP32 with the near pairs
in FP64 and refine in FP64 the particles whose FP32 error estimate is
large.  Their small-system FP64 dispatch is checked separately.
"""
import numpy as np
import pytest

from tests.gpu_util import (check_fp64, check_mixed, fp32_policy, plummer_state,
                            restore_policy)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def H():
    from paper_1104_2700_amd import hermite
    return hermite


@pytest.fixture(scope="module")
def ctx(H):
    c = H.Context(0)
    yield c
    c.close()


def _state(H, n, seed):
    x, v, m = plummer_state(n, seed)
    s = H.State(x, v, m)
    s.xp.copy_(s.x)
    s.vp.copy_(s.v)
    return s, x, v, m


def _idx(n, n_act, seed):
    if n_act == n:
        return np.arange(n, dtype=np.int32)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=n_act, replace=False)).astype(np.int32)


CASES = [(1, 1), (2, 2), (3, 3), (63, 63), (64, 7), (65, 65), (255, 1), (256, 256),
         (257, 64), (1023, 1000), (1024, 65), (4097, 4097), (5000, 1)]


@pytest.mark.parametrize("n,n_act", CASES)
def test_fp64_sweep_parity(H, ctx, n, n_act):
    from oracle import oracle as O
    s, x, v, m = _state(H, n, 100 + n)
    eps2 = (4.0 / max(n, 64)) ** 2
    idx = _idx(n, n_act, n + n_act)
    acc, jrk, pot = ctx.force_jerk(s, torch.from_numpy(idx).cuda(), eps2, H.FP64)
    torch.cuda.synchronize()
    ra, rj, rp, cond = O.force(x, v, m, idx, eps2, with_cond=True)
    check_fp64("acc", acc.cpu().numpy(), ra, cond[0], n)
    check_fp64("jerk", jrk.cpu().numpy(), rj, cond[1], n)
    check_fp64("pot", pot.cpu().numpy()[None], rp[None], cond[2], n)


@pytest.fixture
def variant(H, ctx, request):
    """Installs launch-shape variant `request.param` for every precision
    (bit 0: two particles per lane, bit 1: split FP32 differences, bit 2:
    FP32 runs of 32 terms)."""
    saved = [ctx.get_tuning(p) for p in range(4)]
    for p in range(4):
        t = ctx.get_tuning(p)
        t.variant = request.param
        ctx.set_tuning(p, t)
    yield request.param
    for p in range(4):
        ctx.set_tuning(p, saved[p])


@pytest.mark.parametrize("variant", [0, 1, 2, 3], indirect=True)
@pytest.mark.parametrize("n,n_act", [(3, 3), (300, 300), (1023, 1000), (2049, 9)])
def test_fp64_sweep_parity_variants(H, ctx, variant, n, n_act):
    from oracle import oracle as O
    s, x, v, m = _state(H, n, 300 + n)
    eps2 = (4.0 / max(n, 64)) ** 2
    idx = _idx(n, n_act, n + 11)
    acc, jrk, pot = ctx.force_jerk(s, torch.from_numpy(idx).cuda(), eps2, H.FP64)
    torch.cuda.synchronize()
    ra, rj, rp, cond = O.force(x, v, m, idx, eps2, with_cond=True)
    check_fp64("acc", acc.cpu().numpy(), ra, cond[0], n)
    check_fp64("jerk", jrk.cpu().numpy(), rj, cond[1], n)
    check_fp64("pot", pot.cpu().numpy()[None], rp[None], cond[2], n)


@pytest.fixture
def fp32(H, ctx):
    """The mixed precisions sweep every system in FP32 (the default policy
    does so from N = 32768 on)."""
    saved = fp32_policy(H, ctx)
    yield
    restore_policy(ctx, saved)


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7], indirect=True)
@pytest.mark.parametrize("prec", ["mixed", "mixed2f"])
@pytest.mark.parametrize("n,n_act", [(1, 1), (64, 7), (257, 257), (1024, 1024),
                                     (4097, 65), (5000, 1), (6000, 6000)])
def test_mixed_sweep_parity(H, ctx, fp32, variant, prec, n, n_act):
    from oracle import oracle as O
    s, x, v, m = _state(H, n, 200 + n)
    eps2 = (4.0 / max(n, 64)) ** 2
    idx = _idx(n, n_act, n + 7)
    acc, jrk, pot = ctx.force_jerk(s, torch.from_numpy(idx).cuda(), eps2, prec)
    torch.cuda.synchronize()
    ra, rj, rp, cond = O.force(x, v, m, idx, eps2, with_cond=True)
    check_mixed("acc", acc.cpu().numpy(), ra, cond[0])
    check_mixed("jerk", jrk.cpu().numpy(), rj, cond[1])
    check_mixed("pot", pot.cpu().numpy()[None], rp[None], cond[2])


@pytest.mark.parametrize("near", [0.0, 1.0, 6.0])
def test_mixed_near_factor_range(H, ctx, near):
    """Any near-field radius gives the 1e-6 bar: a small one leaves more
    particles to the FP64 refinement (0: only the self pair is near), a
    large one sums more pairs in FP64 directly."""
    from oracle import oracle as O
    saved = fp32_policy(H, ctx, near_factor=near)
    try:
        n = 3000
        s, x, v, m = _state(H, n, 271)
        eps2 = (4.0 / n) ** 2
        c0 = ctx.counters()["refined"]
        acc, jrk, pot = ctx.force_jerk(s, None, eps2, H.MIXED)
        torch.cuda.synchronize()
        refined = ctx.counters()["refined"] - c0
        ra, rj, rp, cond = O.force(x, v, m, np.arange(n, dtype=np.int32), eps2, with_cond=True)
        check_mixed("acc", acc.cpu().numpy(), ra, cond[0])
        check_mixed("jerk", jrk.cpu().numpy(), rj, cond[1])
        check_mixed("pot", pot.cpu().numpy()[None], rp[None], cond[2])
        assert 0 <= refined < n
        if near == 0.0:
            assert refined > 0
    finally:
        restore_policy(ctx, saved)


def test_mixed_small_systems_take_fp64(H, ctx):
    """Default policy: a system below fp64_below = 32768 particles is swept
    with the FP64 kernel (same launch shape), so the mixed results equal the
    FP64 ones bit for bit; policy arguments are validated."""
    assert ctx.get_mixed_policy(H.MIXED) == (3.0, 32768)
    assert ctx.get_mixed_policy(H.MIXED_SP) == (0.0, 0)
    n = 4096
    s, *_ = _state(H, n, 12)
    eps2 = (4.0 / n) ** 2
    outs = [ctx.force_jerk(s, None, eps2, p) for p in (H.FP64, H.MIXED, H.MIXED_2F)]
    torch.cuda.synchronize()
    for q in range(3):
        assert torch.equal(outs[0][q], outs[1][q]) and torch.equal(outs[0][q], outs[2][q])
    for args in ((H.FP64, 1.0, 0), (H.MIXED, -1.0, 0), (H.MIXED, float("nan"), 0),
                 (H.MIXED, 1.0, -1), (H.MIXED_SP, 0.0, 100)):
        with pytest.raises(H.HermiteError) as err:
            ctx.set_mixed_policy(*args)
        assert err.value.code == H.EINVAL
    assert ctx.get_mixed_policy(H.MIXED) == (3.0, 32768)


def test_mixed_small_blocks_take_fp64(H, ctx):
    """Default block policy: a mixed sweep of fewer than 5e7 interactions is
    done by the FP64 kernel (decided on the device from the active count),
    so it equals the FP64 sweep bit for bit at the same launch shape; a
    larger one uses FP32 pair arithmetic and meets the mixed bar; the
    setting is validated.  (Systems from 8192 particles on are swept in
    FP32 here, so that the block rule decides.)"""
    assert ctx.get_mixed_small_blocks(H.MIXED) == 50000000
    assert ctx.get_mixed_small_blocks(H.MIXED_2F) == 50000000
    assert ctx.get_mixed_small_blocks(H.MIXED_SP) == 0
    n = 20000
    s, x, v, m = _state(H, n, 13)
    eps2 = (4.0 / n) ** 2
    saved = {p: ctx.get_mixed_policy(p) for p in (H.MIXED, H.MIXED_2F)}
    for p, (near, _) in saved.items():
        ctx.set_mixed_policy(p, near, 8192)
    try:
        _small_blocks_cases(H, ctx, s, x, v, m, eps2, n)
    finally:
        for p, args in saved.items():
            ctx.set_mixed_policy(p, *args)
    for args in ((H.FP64, 0), (H.MIXED_SP, 10), (H.MIXED, -1)):
        with pytest.raises(H.HermiteError) as err:
            ctx.set_mixed_small_blocks(*args)
        assert err.value.code == H.EINVAL
    assert ctx.get_mixed_small_blocks(H.MIXED) == 50000000


def _small_blocks_cases(H, ctx, s, x, v, m, eps2, n):
    from oracle import oracle as O
    for n_act, small in ((64, True), (2400, True), (4000, False)):
        idx = _idx(n, n_act, 77)
        ti = torch.from_numpy(idx).cuda()
        ref = ctx.force_jerk(s, ti, eps2, H.FP64)
        for prec in (H.MIXED, H.MIXED_2F):
            got = ctx.force_jerk(s, ti, eps2, prec)
            torch.cuda.synchronize()
            same = all(torch.equal(got[q], ref[q]) for q in range(3))
            assert same == small, (n_act, prec)
            if not small:
                ra, rj, rp, cond = O.force(x, v, m, idx[:300], eps2, with_cond=True)
                check_mixed("acc", got[0].cpu().numpy()[:, :300], ra, cond[0])
                check_mixed("jerk", got[1].cpu().numpy()[:, :300], rj, cond[1])
                check_mixed("pot", got[2].cpu().numpy()[None, :300], rp[None], cond[2])


def test_force_jerk_timed_matches_and_times(H, ctx):
    """hermite_force_jerk_timed gives hermite_force_jerk's results bit for
    bit and positive phase times that add up to the whole call; bad
    arguments are rejected."""
    n = 9000
    s, *_ = _state(H, n, 14)
    eps2 = (4.0 / n) ** 2
    idx = torch.from_numpy(_idx(n, 3000, 5)).cuda()
    for prec in (H.FP64, H.MIXED):
        ref = ctx.force_jerk(s, idx, eps2, prec)
        a, j, p, ms = ctx.force_jerk_timed(s, idx, eps2, prec, reps=3)
        torch.cuda.synchronize()
        assert torch.equal(a, ref[0]) and torch.equal(j, ref[1]) and torch.equal(p, ref[2])
        assert all(ms[k] > 0 for k in ("plan", "sweep", "finish", "total"))
        assert abs(ms["plan"] + ms["sweep"] + ms["finish"] - ms["total"]) <= 1e-9 * ms["total"] + 1e-12
    for kw in ({"reps": 0},):
        with pytest.raises(H.HermiteError) as err:
            ctx.force_jerk_timed(s, idx, eps2, H.FP64, **kw)
        assert err.value.code == H.EINVAL


def test_mixed_ensemble_straddling_threshold(H, ctx):
    """An ensemble whose clusters straddle fp64_below (set to 8192 here)
    runs two kernels: the small clusters' sums equal the FP64 sweep's bit
    for bit, the large ones meet the mixed bar against the oracle.  A small
    block of the same ensemble (below 5e7 interactions) is swept in FP64
    altogether, through the refine sweep's launch: every active particle's
    sums equal the FP64 sweep's bit for bit."""
    from oracle import oracle as O
    from paper_1104_2700_amd import inputs
    sizes = [300, 9000, 1000, 12000, 64]
    xs, vs, ms = [], [], []
    for c, nc in enumerate(sizes):
        x, v, m = inputs.plummer(nc, 600 + c)
        xs.append(x); vs.append(v); ms.append(m)
    x = np.concatenate(xs, 1); v = np.concatenate(vs, 1); m = np.concatenate(ms)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    eps2 = (4.0 / np.maximum(np.array(sizes, float), 64)) ** 2
    cl = H.Clusters(off, eps2)
    s = H.State(x, v, m)
    s.xp.copy_(s.x); s.vp.copy_(s.v)
    A64, J64, P64 = ctx.force_jerk(s, None, 0.0, H.FP64, clusters=cl)
    small = torch.arange(7, int(off[-1]), 200, dtype=torch.int32, device="cuda")
    S64 = ctx.force_jerk(s, small, 0.0, H.FP64, clusters=cl)
    saved = ctx.get_mixed_policy(H.MIXED)
    ctx.set_mixed_policy(H.MIXED, saved[0], 8192)
    try:
        A, J, P = ctx.force_jerk(s, None, 0.0, H.MIXED, clusters=cl)
        Sm = ctx.force_jerk(s, small, 0.0, H.MIXED, clusters=cl)
        torch.cuda.synchronize()
    finally:
        ctx.set_mixed_policy(H.MIXED, *saved)
    assert all(torch.equal(Sm[q], S64[q]) for q in range(3))
    for c, nc in enumerate(sizes):
        lo, hi = off[c], off[c + 1]
        if nc < 8192:
            assert torch.equal(A[:, lo:hi], A64[:, lo:hi]) and torch.equal(J[:, lo:hi], J64[:, lo:hi])
            continue
        sample = np.sort(np.random.default_rng(c).choice(np.arange(lo, hi), 300, replace=False))
        sample = sample.astype(np.int32)
        ra, rj, rp, cond = O.force(x, v, m, sample, eps2[c], j_range=(lo, hi), with_cond=True)
        check_mixed("acc%d" % c, A.cpu().numpy()[:, sample], ra, cond[0])
        check_mixed("jerk%d" % c, J.cpu().numpy()[:, sample], rj, cond[1])
        check_mixed("pot%d" % c, P.cpu().numpy()[sample][None], rp[None], cond[2])


@pytest.mark.parametrize("variant", [0, 1, 4, 5], indirect=True)
@pytest.mark.parametrize("n,n_act", [(1, 1), (64, 7), (257, 257), (1024, 1024),
                                     (4097, 65), (5000, 1)])
def test_mixed_sp_sweep_parity(H, ctx, variant, n, n_act):
    """FP32-velocity / FP32-jerk mode (Section 3.2 as printed; no near field
    beyond the self pair, no refinement).  Acc and pot meet the mixed bar,
    at most one particle in a thousand through the 4 u32 sum_j |term_j|
    clause.  The jerk is an FP32 running sum per lane over up to n terms,
    so its rounding-order bound is the recursive-summation one,
    (16 + n) u32 sum_j |term_j|; the FP32 rounding of the velocities adds
    <= u32 (|v_i| + |v_j|) per term, inside the 16."""
    from oracle import oracle as O
    s, x, v, m = _state(H, n, 400 + n)
    eps2 = (4.0 / max(n, 64)) ** 2
    idx = _idx(n, n_act, n + 13)
    acc, jrk, pot = ctx.force_jerk(s, torch.from_numpy(idx).cuda(), eps2, H.MIXED_SP)
    torch.cuda.synchronize()
    ra, rj, rp, cond = O.force(x, v, m, idx, eps2, with_cond=True)
    cap = n_act // 1000
    check_mixed("acc", acc.cpu().numpy(), ra, cond[0], max_second=cap)
    check_mixed("pot", pot.cpu().numpy()[None], rp[None], cond[2], max_second=cap)
    check_mixed("jerk", jrk.cpu().numpy(), rj, cond[1], tol=0.0, cond_factor=16.0 + n,
                max_second=n_act)


def test_identity_index_and_device_count(H, ctx):
    """idx = NULL (identity) and a device-resident n_act smaller than the
    output stride give the same columns as an explicit list."""
    n = 700
    s, x, v, m = _state(H, n, 5)
    eps2 = 1e-4
    a0, j0, p0 = ctx.force_jerk(s, None, eps2, H.FP64)
    idx = torch.arange(n, dtype=torch.int32, device="cuda")
    na = torch.tensor([300], dtype=torch.int32, device="cuda")
    a1, j1, p1 = ctx.force_jerk(s, idx, eps2, H.FP64, n_act_dev=na, n_act_max=n)
    torch.cuda.synchronize()
    assert torch.equal(a0[:, :300], a1[:, :300])
    assert torch.equal(j0[:, :300], j1[:, :300])
    assert torch.equal(p0[:300], p1[:300])


def test_empty_active_list(H, ctx):
    n = 100
    s, *_ = _state(H, n, 6)
    idx = torch.arange(n, dtype=torch.int32, device="cuda")
    na = torch.zeros(1, dtype=torch.int32, device="cuda")
    acc = torch.full((3, n), 7.0, dtype=torch.float64, device="cuda")
    ctx.force_jerk(s, idx, 1e-4, H.FP64, n_act_dev=na, n_act_max=n, acc=acc)
    torch.cuda.synchronize()
    assert torch.all(acc == 7.0)
    # n_act_max = 0 is a no-op as well
    ctx.force_jerk(s, idx[:0], 1e-4, H.FP64, n_act_max=0)


def test_run_to_run_bitwise(H, ctx):
    n = 3000
    s, *_ = _state(H, n, 8)
    idx = torch.arange(0, n, 3, dtype=torch.int32, device="cuda")
    outs = [ctx.force_jerk(s, idx, 1e-4, p) for p in (0, 0, 1, 1)]
    torch.cuda.synchronize()
    for q in range(3):
        assert torch.equal(outs[0][q], outs[1][q])
        assert torch.equal(outs[2][q], outs[3][q])


def test_zero_softening_two_body(H, ctx):
    """eps = 0 (Kepler pair): Newton's law, exercised through the GPU path."""
    from paper_1104_2700_amd import inputs
    from oracle import oracle as O
    x, v, m = inputs.kepler_pair(0.3, 0.5, 0.4, 0.6, 1.0)
    s = H.State(x, v, m)
    s.xp.copy_(s.x); s.vp.copy_(s.v)
    for prec in (0, 1, 2, 3):
        acc, jrk, pot = ctx.force_jerk(s, None, 0.0, prec)
        torch.cuda.synchronize()
        ra, rj, rp, cond = O.force(x, v, m, np.arange(2, dtype=np.int32), 0.0, with_cond=True)
        tol = 1e-13 if prec == 0 else 1e-6
        assert np.allclose(acc.cpu().numpy(), ra, rtol=tol, atol=0)
        assert np.allclose(pot.cpu().numpy(), rp, rtol=tol, atol=0)


@pytest.mark.parametrize("variant", [1, 3, 5, 7], indirect=True)
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_full_sweep_65536_sampled(H, ctx, variant, prec):
    """The full N = 65536 Plummer sweep (both forms of the FP32 differences:
    FP64 subtraction then cast, variants 1 and 5, and FP32 hi/lo words,
    variants 3 and 7; FP32 runs of 16 or 32 terms),
    checked on the 1024 sampled particles against the oracle and, for the
    mixed precisions, on all 65536 particles against the FP64 sweep (itself
    checked on the sample); plus the momentum invariants over all
    particles."""
    from oracle import oracle as O
    n = 65536
    s, x, v, m = _state(H, n, 3)
    eps2 = (4.0 / n) ** 2
    acc, jrk, pot = ctx.force_jerk(s, None, eps2, prec)
    torch.cuda.synchronize()
    A, J, P = acc.cpu().numpy(), jrk.cpu().numpy(), pot.cpu().numpy()
    sample = np.sort(np.random.default_rng(1003).choice(n, 1024, replace=False)).astype(np.int32)
    ra, rj, rp, cond = O.force(x, v, m, sample, eps2, with_cond=True)
    if prec == 0:
        check_fp64("acc", A[:, sample], ra, cond[0], n)
        check_fp64("jerk", J[:, sample], rj, cond[1], n)
        check_fp64("pot", P[sample][None], rp[None], cond[2], n)
    else:
        # every sampled particle within 1e-6 of the oracle in acc, jerk, pot
        check_mixed("acc", A[:, sample], ra, cond[0])
        check_mixed("jerk", J[:, sample], rj, cond[1])
        check_mixed("pot", P[sample][None], rp[None], cond[2])
        # and every particle within 1e-6 of the FP64 sweep
        a64, j64, p64 = ctx.force_jerk(s, None, eps2, H.FP64)
        torch.cuda.synchronize()
        a64, j64, p64 = a64.cpu().numpy(), j64.cpu().numpy(), p64.cpu().numpy()
        ea = np.linalg.norm(A - a64, axis=0) / np.linalg.norm(a64, axis=0)
        ej = np.linalg.norm(J - j64, axis=0) / np.linalg.norm(j64, axis=0)
        ep = np.abs(P - p64) / np.abs(p64)
        assert ea.max() < 1e-6 and ej.max() < 1e-6 and ep.max() < 1e-6, (
            ea.max(), ej.max(), ep.max())
    # Newton's third law over the whole system
    scale = np.sum(m * np.linalg.norm(A, axis=0))
    assert np.abs(A @ m).max() < (1e-12 if prec == 0 else 1e-5) * scale


@pytest.mark.parametrize("prec", [0, 1])
def test_autotune_shape_within_tolerance(H, ctx, prec, tmp_path):
    """The autotuner's chosen launch shape gives results within the
    precision's tolerance of the oracle, and its JSON cache round-trips."""
    from oracle import oracle as O
    n = 4096
    s, x, v, m = _state(H, n, 77)
    eps2 = (4.0 / n) ** 2
    cache = tmp_path / "tune.json"
    default = ctx.get_tuning(prec)
    tuned = ctx.autotune(s, eps2, prec, n_act=n, cache_path=cache)
    try:
        acc, jrk, pot = ctx.force_jerk(s, None, eps2, prec)
        torch.cuda.synchronize()
        ra, rj, rp, cond = O.force(x, v, m, np.arange(n, dtype=np.int32), eps2, with_cond=True)
        if prec == 0:
            check_fp64("acc", acc.cpu().numpy(), ra, cond[0], n)
            check_fp64("jerk", jrk.cpu().numpy(), rj, cond[1], n)
        else:
            check_mixed("acc", acc.cpu().numpy(), ra, cond[0])
            check_mixed("jerk", jrk.cpu().numpy(), rj, cond[1])
        assert cache.exists() and "target_lanes" in cache.read_text()
        ctx.set_tuning(prec, default)
        assert ctx.load_tuning(cache, prec, n, n)
        assert ctx.get_tuning(prec).as_dict() == tuned.as_dict()
        assert not ctx.load_tuning(cache, prec, 1 << 20, 1 << 20)
    finally:
        ctx.set_tuning(prec, default)
