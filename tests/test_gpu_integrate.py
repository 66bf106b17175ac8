"""GPU block-step stages vs the oracle, through the C ABI: selection
(bit-exact), predictor, corrector + next step, first step, energy, one-step
lockstep integration, graph replay vs eager, ensembles vs per-cluster."""
import numpy as np
import pytest

from tests.gpu_util import check_fp64, check_mixed, fp32_policy, restore_policy

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TB = 20


@pytest.fixture(scope="module")
def H():
    from paper_1104_2700_amd import hermite
    return hermite


@pytest.fixture(scope="module")
def ctx(H):
    c = H.Context(0)
    yield c
    c.close()


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda", dtype=dtype) if dtype else t.cuda()


def _near_boundary(crit, rel=1e-7):
    """True where a criterion lies within rel of a power of two."""
    crit = np.asarray(crit, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        l2 = np.log2(crit)
    return np.abs(l2 - np.rint(l2)) < rel / np.log(2)


@pytest.mark.parametrize("n", [1, 5, 1023, 1024, 1025, 70000])
def test_select_bit_exact(H, ctx, n):
    from oracle import oracle as O
    from paper_1104_2700_amd import inputs
    T = 3 << 14
    t, dt = inputs.synced_block_times(n, n, TB, 3, 14, T)
    s = H.State(np.zeros((3, n)), np.zeros((3, n)), np.ones(n), TB)
    s.t.copy_(_dev(t)); s.dt.copy_(_dev(dt))
    idx = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    na = torch.zeros(1, dtype=torch.int32, device="cuda")
    Td = torch.zeros(1, dtype=torch.int64, device="cuda")
    ctx.select_block(s, idx, na, Td)
    torch.cuda.synchronize()
    T_ref, idx_ref = O.select(t, dt)
    assert int(Td.item()) == T_ref
    k = int(na.item())
    assert k == idx_ref.shape[0]
    assert np.array_equal(idx[:k].cpu().numpy(), idx_ref)
    # a block time past T_end selects nothing
    ctx.select_block(s, idx, na, Td, T_end=T_ref - 1)
    torch.cuda.synchronize()
    assert int(na.item()) == 0 and int(Td.item()) == T_ref


def test_predict_parity(H, ctx):
    from oracle import oracle as O
    from paper_1104_2700_amd import inputs
    n = 3001
    rng = np.random.default_rng(4)
    x, v, a, j = rng.normal(size=(4, 3, n))
    T = 5 << 12
    t, dt = inputs.synced_block_times(n, 9, TB, 3, 20, T)
    s = H.State(x, v, np.ones(n), TB)
    s.a.copy_(_dev(a)); s.j.copy_(_dev(j)); s.t.copy_(_dev(t))
    ctx.predict(s, T_host=T)
    torch.cuda.synchronize()
    xp, vp = O.predict(x, v, a, j, t, T, TB)
    scale_x = np.abs(x) + np.abs(v) + np.abs(a) + np.abs(j)
    assert np.all(np.abs(s.xp.cpu().numpy() - xp) <= 4e-16 * scale_x)
    assert np.all(np.abs(s.vp.cpu().numpy() - vp) <= 4e-16 * scale_x)
    # device block time and a zero active count (no-op)
    Td = torch.tensor([T], dtype=torch.int64, device="cuda")
    s.xp.zero_()
    ctx.predict(s, T_dev=Td)
    torch.cuda.synchronize()
    assert np.all(np.abs(s.xp.cpu().numpy() - xp) <= 4e-16 * scale_x)
    s.xp.zero_()
    ctx.predict(s, T_dev=Td, n_act_dev=torch.zeros(1, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    assert torch.all(s.xp == 0)


def test_correct_parity(H, ctx):
    """Corrector, a0/j0 update, t and the next step for a random active list
    (inputs are random but consistent: t_i + dt_i = T)."""
    from oracle import oracle as O
    n = 2000
    rng = np.random.default_rng(5)
    T = 1 << 15
    k = rng.integers(5, 15, size=n)
    dt = (np.int64(1) << (TB - k)).astype(np.int64)
    t = (T - dt).astype(np.int64)
    x, v, a0, j0 = rng.normal(size=(4, 3, n))
    ostate = O.new_state(x, v, np.ones(n), TB)
    ostate["a"][...] = a0; ostate["j"][...] = j0
    ostate["t"][...] = t; ostate["dt"][...] = dt
    xp, vp = O.predict(x, v, a0, j0, t, T, TB)
    idx = np.sort(rng.choice(n, 700, replace=False)).astype(np.int32)
    h = (dt[idx] * 2.0**-TB)[None]
    a1 = a0[:, idx] + j0[:, idx] * h + rng.normal(size=(3, 700)) * h * h
    j1 = j0[:, idx] + rng.normal(size=(3, 700)) * h
    p1 = rng.normal(size=700)
    s = H.State(x, v, np.ones(n), TB)
    s.a.copy_(_dev(a0)); s.j.copy_(_dev(j0)); s.t.copy_(_dev(t)); s.dt.copy_(_dev(dt))
    s.xp.copy_(_dev(xp)); s.vp.copy_(_dev(vp))
    params = H.dt_params(0.02, H.DT_PAPER, 3, 20)
    crit = torch.zeros(700, dtype=torch.float64, device="cuda")
    ctx.correct(s, _dev(idx), _dev(a1), _dev(j1), _dev(p1), params, T_host=T, crit_out=crit)
    torch.cuda.synchronize()
    crit_ref = np.zeros(700)
    O.correct(ostate, idx, T, xp, vp, a1, j1, p1, 0.02, 0, 3, 20, crit_out=crit_ref)
    g = s.to_numpy()
    sc = np.abs(xp) + 1.0
    assert np.all(np.abs(g["x"] - ostate["x"]) <= 1e-14 * sc)
    assert np.all(np.abs(g["v"] - ostate["v"]) <= 1e-14 * (np.abs(vp) + 1.0))
    assert np.array_equal(g["a"], ostate["a"]) and np.array_equal(g["j"], ostate["j"])
    assert np.array_equal(g["t"], ostate["t"]) and np.array_equal(g["pot"], ostate["pot"])
    c = crit.cpu().numpy()
    assert np.allclose(c, crit_ref, rtol=1e-9)
    mism = g["dt"] != ostate["dt"]
    assert np.all(_near_boundary(crit_ref[np.searchsorted(idx, np.nonzero(mism)[0])], 1e-9)) \
        if mism.any() else True


def _c1_setup(H, n=1024, seed=1, eps=1.0 / 64):
    from paper_1104_2700_amd import inputs
    x, v, m = inputs.plummer(n, seed)
    return x, v, m, eps * eps


@pytest.mark.parametrize("form,eta_init", [(0, 0.0), (1, 0.0), (0, 0.05)])
def test_initialize_and_energy(H, ctx, form, eta_init):
    from oracle import oracle as O
    x, v, m, eps2 = _c1_setup(H)
    n = m.shape[0]
    eta = 0.02
    params = H.dt_params(eta, form, 3, 20, eta_init=eta_init)
    s = H.State(x, v, m, TB)
    ctx.initialize(s, eps2, params, H.FP64)
    e = ctx.energy(s, eps2)
    torch.cuda.synchronize()
    ost = O.new_state(x, v, m, TB)
    O.initialize(ost, eps2, eta, form, 3, 20, eta_init=eta_init)
    g = s.to_numpy()
    _, _, _, cond = O.force(x, v, m, np.arange(n, dtype=np.int32), eps2, with_cond=True)
    check_fp64("a0", g["a"], ost["a"], cond[0], n)
    check_fp64("j0", g["j"], ost["j"], cond[1], n)
    assert np.all(g["t"] == 0)
    # start-up factor (written out here only to locate quantisation ties)
    eta_s = eta_init if eta_init > 0 else (eta if form == 0 else np.sqrt(eta))
    crit = eta_s * np.linalg.norm(ost["a"], axis=0) / np.linalg.norm(ost["j"], axis=0)
    mism = g["dt"] != ost["dt"]
    assert np.all(_near_boundary(crit[mism], 1e-9))
    K, W = O.energy(x, v, m, eps2)
    Kg, Wg = e[0].tolist()
    assert Kg == pytest.approx(K, rel=1e-14)
    assert Wg == pytest.approx(W, rel=1e-13)


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_lockstep_block_steps(H, ctx, prec):
    """One block step at a time (N = 1024): the oracle takes the GPU's
    pre-step state; block times and active lists must be identical, and the
    new forces agree with the oracle's to the precision's bar on every
    active particle: FP64 1e-13 (rounding-order clause), the mixed
    precisions (swept in FP32 here, with their near field and refinement)
    1e-6 for acc, jerk and pot, the paper-faithful mode 1e-6 for acc and
    pot and its recursive-summation bound for the FP32 jerk.  FP64: the
    oracle's whole step agrees (positions ~1e-15, step sizes except at
    criterion ties).  Mixed: the oracle's corrector given the GPU's forces
    reproduces the GPU's corrected state (the criterion differences the
    forces over a step, so force errors of a few 1e-8 can move it by more
    than a tie where the step is short)."""
    from oracle import oracle as O
    x, v, m, eps2 = _c1_setup(H)
    n = m.shape[0]
    params = H.dt_params(0.02, H.DT_PAPER, 3, 20)
    saved = fp32_policy(H, ctx)
    try:
        s = H.State(x, v, m, TB)
        ctx.initialize(s, eps2, params, H.FP64)
        torch.cuda.synchronize()
        ties = 0
        for step in range(40):
            pre = s.to_numpy()
            ost = {k: (pre[k].copy() if isinstance(pre[k], np.ndarray) else pre[k]) for k in pre}
            T, idx = O.select(ost["t"], ost["dt"])
            xp, vp = O.predict(ost["x"], ost["v"], ost["a"], ost["j"], ost["t"], T, TB)
            a1, j1, p1, cond = O.force(xp, vp, m, idx, eps2, with_cond=True)
            ctx.step(s, eps2, params, prec)
            cnt = ctx.counters()
            g = s.to_numpy()
            assert cnt["T"] == T and cnt["n_act"] == idx.shape[0]
            ga, gj, gp = g["a"][:, idx], g["j"][:, idx], g["pot"][idx]
            if prec == 0:
                check_fp64("a", ga, a1, cond[0], n)
                check_fp64("j", gj, j1, cond[1], n)
                fa, fj, fp = a1, j1, p1
            else:
                check_mixed("a", ga, a1, cond[0])
                check_mixed("pot", gp[None], p1[None], cond[2])
                if prec == 3:
                    check_mixed("j", gj, j1, cond[1], tol=0.0, cond_factor=16.0 + n,
                                max_second=idx.shape[0])
                else:
                    check_mixed("j", gj, j1, cond[1])
                fa, fj, fp = ga.copy(), gj.copy(), gp.copy()
            crit_ref = np.zeros(idx.shape[0])
            O.correct(ost, idx, T, xp, vp, fa, fj, fp, 0.02, 0, 3, 20, crit_out=crit_ref)
            assert np.array_equal(g["t"], ost["t"])
            rel_x = np.abs(g["x"] - ost["x"]).max() / np.abs(ost["x"]).max()
            assert rel_x < (1e-14 if prec == 0 else 1e-13), rel_x
            mism = g["dt"] != ost["dt"]
            if mism.any():
                pos = np.searchsorted(idx, np.nonzero(mism)[0])
                assert np.all(_near_boundary(crit_ref[pos], 1e-6 if prec == 0 else 1e-9))
                ratio = g["dt"][mism] / ost["dt"][mism]
                assert np.all((ratio == 2) | (ratio == 0.5))
                ties += int(mism.sum())
                # continue from the oracle's decision so the runs stay in step
                s.dt.copy_(_dev(ost["dt"]))
        assert ties <= 2
    finally:
        restore_policy(ctx, saved)


def test_mixed_small_block_steps_take_fp64(H, ctx):
    """Block steps with the default block policy: while a block's sweep is
    below 5e7 interactions it is done in FP64 (with the mixed path's
    flagging reduce and corrector), so the state follows FP64 steps bit for
    bit; hermite_run and hermite_step agree too.  (Systems from 8192
    particles on are swept in FP32 here, so that the block rule decides.)"""
    n = 20000
    x, v, m, _ = _c1_setup(H, n=n, seed=51)
    eps2 = (4.0 / n) ** 2
    params = H.dt_params(0.02, H.DT_PAPER, 3, 20)
    s0 = H.State(x, v, m, TB)
    ctx.initialize(s0, eps2, params, H.FP64)
    saved = ctx.get_mixed_policy(H.MIXED)
    ctx.set_mixed_policy(H.MIXED, saved[0], 8192)
    try:
        _small_block_steps(H, ctx, s0, eps2, params, n)
    finally:
        ctx.set_mixed_policy(H.MIXED, *saved)


def test_mixed_small_block_steps_take_fp64_ensemble(H, ctx):
    """The same for an ensemble whose clusters straddle fp64_below (8192
    here): small blocks are swept in FP64 through the refine sweep's launch
    and reduced by the corrector, so the state follows FP64 steps bit for
    bit, in hermite_step and hermite_run."""
    from paper_1104_2700_amd import inputs
    sizes = [300, 9000, 1000, 12000, 64]
    xs, vs, ms = [], [], []
    for c, nc in enumerate(sizes):
        x, v, m = inputs.plummer(nc, 700 + c)
        xs.append(x); vs.append(v); ms.append(m)
    x = np.concatenate(xs, 1); v = np.concatenate(vs, 1); m = np.concatenate(ms)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cl = H.Clusters(off, (4.0 / np.maximum(np.array(sizes, float), 64)) ** 2)
    params = H.dt_params(0.02, H.DT_PAPER, 3, 20)
    s0 = H.State(x, v, m, TB)
    ctx.initialize(s0, 0.0, params, H.FP64, clusters=cl)
    saved = ctx.get_mixed_policy(H.MIXED)
    ctx.set_mixed_policy(H.MIXED, saved[0], 8192)
    try:
        _small_block_steps(H, ctx, s0, 0.0, params, max(sizes), clusters=cl)
    finally:
        ctx.set_mixed_policy(H.MIXED, *saved)


def _small_block_steps(H, ctx, s0, eps2, params, n, clusters=None):
    """n: the largest system, so that n_act * n bounds a block's interactions."""
    sa, sb = s0.clone(), s0.clone()
    checked = 0
    for k in range(16):
        ctx.step(sa, eps2, params, H.FP64, clusters=clusters)
        na = ctx.counters()["n_act"]
        ctx.step(sb, eps2, params, H.MIXED, clusters=clusters)
        torch.cuda.synchronize()
        if na * n >= 50000000:
            break
        for key in ("x", "v", "a", "j", "pot", "t", "dt"):
            assert torch.equal(getattr(sa, key), getattr(sb, key)), (k, key)
        checked += 1
    assert checked >= 8
    sc = s0.clone()
    ctx.run(sc, eps2, params, 1 << (TB - 3), H.MIXED, max_steps=checked, clusters=clusters)
    sd = s0.clone()
    for k in range(checked):
        ctx.step(sd, eps2, params, H.FP64, clusters=clusters)
    torch.cuda.synchronize()
    for key in ("x", "v", "a", "j", "pot", "t", "dt"):
        assert torch.equal(getattr(sc, key), getattr(sd, key)), key


@pytest.mark.parametrize("n", [3, 3000, 6000, 20000, 200000])
def test_lockstep_larger_systems(H, ctx, n):
    """Block steps of systems on each selection path: selection fused into
    the sweep (n = 3), one selection workgroup (n = 3000), several selection
    blocks with the last-block ticket (n = 6000, 20000), many blocks with
    separate passes and plan (n = 200000, 49 blocks): active list, block time
    and corrected state equal the oracle's step from the same pre-step
    state."""
    from oracle import oracle as O
    x, v, m, _ = _c1_setup(H, n=n, seed=31)
    eps2 = (4.0 / n) ** 2
    params = H.dt_params(0.02, H.DT_PAPER, 3, 20)
    s = H.State(x, v, m, TB)
    ctx.initialize(s, eps2, params, H.FP64)
    torch.cuda.synchronize()
    for k in range(4):
        pre = s.to_numpy()
        T, idx = O.select(pre["t"], pre["dt"])
        ctx.step(s, eps2, params, H.FP64, use_graph=(k % 2 == 1))
        cnt = ctx.counters()
        g = s.to_numpy()
        assert cnt["T"] == T and cnt["n_act"] == idx.shape[0]
        sub = {kk: (vv.copy() if isinstance(vv, np.ndarray) else vv) for kk, vv in pre.items()}
        xp, vp = O.predict(sub["x"], sub["v"], sub["a"], sub["j"], sub["t"], T, TB)
        a1, j1, p1 = O.force(xp, vp, sub["m"], idx, eps2)
        crit_ref = np.zeros(idx.shape[0])
        O.correct(sub, idx, T, xp, vp, a1, j1, p1, 0.02, 0, 3, 20, crit_out=crit_ref)
        assert np.abs(g["x"] - sub["x"]).max() <= 1e-14 * (np.abs(sub["x"]).max() + 1)
        assert np.array_equal(g["t"], sub["t"])
        mism = g["dt"] != sub["dt"]
        if mism.any():
            # a power-of-two decision may differ only at a boundary tie
            pos = np.searchsorted(idx, np.nonzero(mism)[0])
            assert np.all(_near_boundary(crit_ref[pos], 1e-6))
            s.dt.copy_(_dev(sub["dt"]))


@pytest.mark.parametrize("fp32", [False, True], ids=["default", "fp32"])
def test_graph_replay_matches_eager(H, ctx, fp32):
    """Graph-replayed mixed block steps equal eager ones bit for bit, with
    the default policy (this system is swept in FP64) and with every system
    in FP32 (the flagging reduce, refine list, FP64 refine sweep and
    corrector inside each captured step)."""
    x, v, m, eps2 = _c1_setup(H, n=2048, seed=11)
    params = H.dt_params(0.02, H.DT_PAPER, 3, 20)
    saved = fp32_policy(H, ctx, near_factor=1.0) if fp32 else None
    try:
        s0 = H.State(x, v, m, TB)
        ctx.initialize(s0, eps2, params, H.FP64)
        sa, sb = s0.clone(), s0.clone()
        c0 = ctx.counters()["refined"]
        for _ in range(30):
            ctx.step(sa, eps2, params, H.MIXED, use_graph=False)
        c1 = ctx.counters()["refined"]
        for k in range(30):
            ctx.step(sb, eps2, params, H.MIXED, use_graph=True)
            if k % 7 == 3:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        c2 = ctx.counters()["refined"]
        assert c2 - c1 == c1 - c0
        if fp32:
            assert c1 > c0
        for key in ("x", "v", "a", "j", "pot", "t", "dt"):
            assert torch.equal(getattr(sa, key), getattr(sb, key)), key
    finally:
        if saved:
            restore_policy(ctx, saved)


def test_run_c1_energy_and_oracle(H, ctx):
    """Plummer N = 1024, eps = 1/64, eta = 0.02, t = 0 -> 0.125 (FP64):
    graph-replayed run, energy conserved like the oracle's run."""
    from oracle import oracle as O
    x, v, m, eps2 = _c1_setup(H)
    params = H.dt_params(0.02, H.DT_PAPER, 3, 20)
    T_end = 1 << (TB - 3)
    s = H.State(x, v, m, TB)
    ctx.initialize(s, eps2, params, H.FP64)
    e0 = ctx.energy(s, eps2)[0].sum().item()
    steps, inter = ctx.run(s, eps2, params, T_end, H.FP64, use_graph=True, sync_every=32)
    e1 = ctx.energy(s, eps2)[0].sum().item()
    g = s.to_numpy()
    assert np.all(g["t"] == T_end)
    ost = O.new_state(x, v, m, TB)
    stats = O.run(ost, T_end, eps2, 0.02, 0, 3, 20)
    K0, W0 = O.energy(x, v, m, eps2)
    K1, W1 = O.energy(ost["x"], ost["v"], m, eps2)
    d_gpu = abs(e1 - e0) / abs(e0)
    d_ora = abs((K1 + W1) - (K0 + W0)) / abs(K0 + W0)
    assert d_gpu < 1e-6 and d_ora < 1e-6
    assert abs(steps - stats["steps"]) <= 0.02 * stats["steps"]
    assert np.abs(g["x"] - ost["x"]).max() < 1e-6


def test_ensemble_force_and_lockstep(H, ctx):
    """Clusters of uneven size (including a lone particle) in one state:
    per-cluster sums and softening, and a few lockstep block steps."""
    from oracle import oracle as O
    from paper_1104_2700_amd import inputs
    sizes = [300, 1000, 64, 1, 2000, 513]
    xs, vs, ms = [], [], []
    for c, nc in enumerate(sizes):
        x, v, m = inputs.plummer(nc, 500 + c)
        xs.append(x); vs.append(v); ms.append(m)
    x = np.concatenate(xs, 1); v = np.concatenate(vs, 1); m = np.concatenate(ms)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    eps2 = (4.0 / np.maximum(np.array(sizes, float), 64)) ** 2
    cl = H.Clusters(off, eps2)
    s = H.State(x, v, m, TB)
    s.xp.copy_(s.x); s.vp.copy_(s.v)
    n = m.shape[0]
    acc, jrk, pot = ctx.force_jerk(s, None, 0.0, H.FP64, clusters=cl)
    torch.cuda.synchronize()
    A, J, P = acc.cpu().numpy(), jrk.cpu().numpy(), pot.cpu().numpy()
    for c in range(len(sizes)):
        lo, hi = off[c], off[c + 1]
        ids = np.arange(lo, hi, dtype=np.int32)
        ra, rj, rp, cond = O.force(x, v, m, ids, eps2[c], j_range=(lo, hi), with_cond=True)
        check_fp64("acc%d" % c, A[:, lo:hi], ra, cond[0], hi - lo)
        check_fp64("jerk%d" % c, J[:, lo:hi], rj, cond[1], hi - lo)
    # energies per cluster
    e = ctx.energy(s, 0.0, clusters=cl).cpu().numpy()
    for c in range(len(sizes)):
        lo, hi = off[c], off[c + 1]
        K, W = O.energy(x[:, lo:hi], v[:, lo:hi], m[lo:hi], eps2[c])
        assert e[c, 0] == pytest.approx(K, rel=1e-13)
        assert e[c, 1] == pytest.approx(W, rel=1e-12, abs=1e-300)
    # lockstep: the union of clusters on one timeline equals each cluster
    params = H.dt_params(0.02, H.DT_PAPER, 3, 20)
    ctx.initialize(s, 0.0, params, H.FP64, clusters=cl)
    torch.cuda.synchronize()
    for _ in range(10):
        pre = s.to_numpy()
        T, idx = O.select(pre["t"], pre["dt"])
        ctx.step(s, 0.0, params, H.FP64, clusters=cl)
        g = s.to_numpy()
        for c in range(len(sizes)):
            lo, hi = off[c], off[c + 1]
            act = idx[(idx >= lo) & (idx < hi)]
            if act.size == 0:
                assert np.array_equal(g["x"][:, lo:hi], pre["x"][:, lo:hi])
                continue
            sub = {k: (pre[k][..., lo:hi].copy() if isinstance(pre[k], np.ndarray) else pre[k])
                   for k in pre}
            xp, vp = O.predict(sub["x"], sub["v"], sub["a"], sub["j"], sub["t"], T, TB)
            la = (act - lo).astype(np.int32)
            a1, j1, p1 = O.force(xp, vp, sub["m"], la, eps2[c])
            O.correct(sub, la, T, xp, vp, a1, j1, p1, 0.02, 0, 3, 20)
            assert np.abs(g["x"][:, lo:hi] - sub["x"]).max() <= 1e-14 * (np.abs(sub["x"]).max() + 1)
            assert np.array_equal(g["t"][lo:hi], sub["t"])


@pytest.mark.parametrize("n,prec", [(1024, 0), (6000, 1), (10000, 2)])
def test_run_graph_batches_match_eager(H, ctx, n, prec):
    """hermite_run replays graphs of several steps (8 per graph, then single
    steps for the rest of a batch): the state, the step count and the
    counters match eager steps bit for bit, for one-block (n <= 4096) and
    multi-block selection; n = 10000 sweeps in FP32 with refinement."""
    x, v, m, eps2 = _c1_setup(H, n=n, seed=21)
    params = H.dt_params(0.02, H.DT_PAPER, 3, 20)
    s0 = H.State(x, v, m, TB)
    ctx.initialize(s0, eps2, params, prec)
    sa, sb = s0.clone(), s0.clone()
    T_end = 1 << (TB - 3)
    c0 = ctx.counters()
    st_a, it_a = ctx.run(sa, eps2, params, T_end, prec, use_graph=False, sync_every=13,
                         max_steps=45)
    c1 = ctx.counters()
    st_b, it_b = ctx.run(sb, eps2, params, T_end, prec, use_graph=True, sync_every=13,
                         max_steps=45)
    c2 = ctx.counters()
    torch.cuda.synchronize()
    assert st_a == st_b == 45 and it_a == it_b
    assert c1["steps"] - c0["steps"] == c2["steps"] - c1["steps"] == 45
    for key in ("x", "v", "a", "j", "pot", "t", "dt"):
        assert torch.equal(getattr(sa, key), getattr(sb, key)), key


def test_steps_past_the_end_change_nothing(H, ctx):
    """Once every particle is at T_end, further steps (single or in a graph
    of several) change neither the state nor the counters."""
    x, v, m, eps2 = _c1_setup(H, n=512, seed=23)
    params = H.dt_params(0.04, H.DT_PAPER, 3, 20)
    s = H.State(x, v, m, TB)
    ctx.initialize(s, eps2, params, H.FP64)
    T_end = 1 << (TB - 3)
    ctx.run(s, eps2, params, T_end, H.FP64, use_graph=True, sync_every=64)
    torch.cuda.synchronize()
    g0 = s.to_numpy()
    assert np.all(g0["t"] == T_end)
    c0, h0 = ctx.counters(), ctx.block_histogram()
    for k in range(3):
        ctx.step(s, eps2, params, H.FP64, T_end=T_end, use_graph=(k % 2 == 0))
    st, it = ctx.run(s, eps2, params, T_end, H.FP64, use_graph=True, sync_every=16)
    torch.cuda.synchronize()
    g1 = s.to_numpy()
    assert st == 0 and it == 0
    assert ctx.counters() == c0 and ctx.block_histogram() == h0
    assert h0[0] == 0
    for key in ("x", "v", "a", "j", "t", "dt"):
        assert np.array_equal(g0[key], g1[key]), key


@pytest.mark.parametrize("sizes", [[3000, 1, 2500, 700, 64], [9000, 1, 8000, 2500, 700]],
                         ids=["n6265", "n20201"])
def test_ensemble_multiblock_lockstep(H, ctx, sizes):
    """Ensembles larger than one selection block (n = 6265 and 20201): the
    selection's cluster bookkeeping across blocks gives, per cluster, the
    oracle's block step."""
    from oracle import oracle as O
    from paper_1104_2700_amd import inputs
    xs, vs, ms = [], [], []
    for c, nc in enumerate(sizes):
        x, v, m = inputs.plummer(nc, 700 + c)
        xs.append(x); vs.append(v); ms.append(m)
    x = np.concatenate(xs, 1); v = np.concatenate(vs, 1); m = np.concatenate(ms)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    eps2 = (4.0 / np.maximum(np.array(sizes, float), 64)) ** 2
    cl = H.Clusters(off, eps2)
    s = H.State(x, v, m, TB)
    params = H.dt_params(0.02, H.DT_PAPER, 3, 20)
    ctx.initialize(s, 0.0, params, H.FP64, clusters=cl)
    torch.cuda.synchronize()
    for step in range(8):
        pre = s.to_numpy()
        T, idx = O.select(pre["t"], pre["dt"])
        ctx.step(s, 0.0, params, H.FP64, clusters=cl, use_graph=(step % 2 == 1))
        g = s.to_numpy()
        for c in range(len(sizes)):
            lo, hi = off[c], off[c + 1]
            act = idx[(idx >= lo) & (idx < hi)]
            if act.size == 0:
                assert np.array_equal(g["x"][:, lo:hi], pre["x"][:, lo:hi])
                continue
            sub = {k: (pre[k][..., lo:hi].copy() if isinstance(pre[k], np.ndarray) else pre[k])
                   for k in pre}
            xp, vp = O.predict(sub["x"], sub["v"], sub["a"], sub["j"], sub["t"], T, TB)
            la = (act - lo).astype(np.int32)
            a1, j1, p1 = O.force(xp, vp, sub["m"], la, eps2[c])
            O.correct(sub, la, T, xp, vp, a1, j1, p1, 0.02, 0, 3, 20)
            assert np.abs(g["x"][:, lo:hi] - sub["x"]).max() <= 1e-14 * (np.abs(sub["x"]).max() + 1)
            assert np.array_equal(g["t"][lo:hi], sub["t"])


def _ensemble(H, sizes, seed0=700):
    from paper_1104_2700_amd import inputs
    xs, vs, ms = [], [], []
    for c, nc in enumerate(sizes):
        x, v, m = inputs.plummer(nc, seed0 + c)
        xs.append(x); vs.append(v); ms.append(m)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    eps2 = (4.0 / np.maximum(np.array(sizes, float), 64)) ** 2
    return (np.concatenate(xs, 1), np.concatenate(vs, 1), np.concatenate(ms),
            H.Clusters(off, eps2))


def _run_vs_steps(H, ctx, s0, eps2, params, prec, K, clusters=None, T_end=1 << (TB - 3),
                  sync_every=16):
    """K steps by hermite_run (selection from the step-size order) and by K
    hermite_step calls (selection from t and dt): same state bit for bit,
    same counters and block-size histogram."""
    sa, sb = s0.clone(), s0.clone()
    c0, h0 = ctx.counters(), ctx.block_histogram()
    st, it = ctx.run(sa, eps2, params, T_end, prec, use_graph=True, sync_every=sync_every,
                     max_steps=K, clusters=clusters)
    c1, h1 = ctx.counters(), ctx.block_histogram()
    for k in range(K):
        ctx.step(sb, eps2, params, prec, T_end=T_end, use_graph=(k % 3 == 0), clusters=clusters)
    c2, h2 = ctx.counters(), ctx.block_histogram()
    torch.cuda.synchronize()
    assert st == c1["steps"] - c0["steps"] == c2["steps"] - c1["steps"]
    assert it == c1["interactions"] - c0["interactions"] == c2["interactions"] - c1["interactions"]
    assert c1["clamped"] - c0["clamped"] == c2["clamped"] - c1["clamped"]
    assert [b - a for a, b in zip(h0, h1)] == [b - a for a, b in zip(h1, h2)]
    for key in ("x", "v", "a", "j", "pot", "t", "dt"):
        assert torch.equal(getattr(sa, key), getattr(sb, key)), key
    return st, sa


@pytest.mark.parametrize("n,prec", [(3000, 0), (6000, 1), (20000, 0)])
def test_run_order_selection_matches_steps(H, ctx, n, prec):
    """Block steps selected from the step-size order (hermite_run) give the
    state of steps selected from t and dt (hermite_step), for one selection
    workgroup (n = 3000) and several (n = 6000, 20000), over several run
    batches (each batch's graph replays and syncs in between)."""
    x, v, m, _ = _c1_setup(H, n=n, seed=41)
    eps2 = (4.0 / n) ** 2
    params = H.dt_params(0.02, H.DT_PAPER, 3, 20)
    s0 = H.State(x, v, m, TB)
    ctx.initialize(s0, eps2, params, prec)
    st, _ = _run_vs_steps(H, ctx, s0, eps2, params, prec, 45, sync_every=13)
    assert st == 45


@pytest.mark.parametrize("clustered", [False, True], ids=["one", "clusters"])
def test_run_order_selection_whole_blocks(H, ctx, clustered):
    """Every particle on one shared step at t = 0: the first block is the
    whole system (6000 / 6265 particles), larger than the selection's LDS
    staging, so the next step re-sorts (and groups by cluster) through
    global memory; the state still follows hermite_step bit for bit."""
    if clustered:
        x, v, m, cl = _ensemble(H, [3000, 1, 2500, 700, 64])
        eps2 = 0.0
    else:
        x, v, m, _ = _c1_setup(H, n=6000, seed=43)
        cl, eps2 = None, (4.0 / 6000) ** 2
    params = H.dt_params(0.02, H.DT_PAPER, 3, 20)
    s0 = H.State(x, v, m, TB)
    ctx.initialize(s0, eps2, params, H.FP64, clusters=cl)
    s0.dt.fill_(1 << (TB - 12))
    s0.t.zero_()
    s1 = s0.clone()
    ctx.run(s1, eps2, params, 1 << (TB - 3), H.FP64, max_steps=1, clusters=cl)
    assert ctx.counters()["n_act"] == s0.n
    _run_vs_steps(H, ctx, s0, eps2, params, H.FP64, 24, clusters=cl)


@pytest.mark.parametrize("sizes", [[9000, 1, 8000, 2500, 700], [300] * 40],
                         ids=["n20201", "c40"])
def test_run_order_selection_ensemble(H, ctx, sizes):
    """Ensembles: the block grouped by cluster from the step-size order
    gives the state of the selection from t and dt."""
    x, v, m, cl = _ensemble(H, sizes, seed0=900)
    params = H.dt_params(0.02, H.DT_PAPER, 3, 20)
    s0 = H.State(x, v, m, TB)
    ctx.initialize(s0, 0.0, params, H.MIXED, clusters=cl)
    _run_vs_steps(H, ctx, s0, 0.0, params, H.MIXED, 40, clusters=cl)


@pytest.mark.parametrize("case", ["t_off_grid", "dt_not_pow2", "dt_below_floor", "overdue"])
def test_run_inconsistent_state_falls_back(H, ctx, case):
    """A state the block scheme cannot have produced (a time off its step's
    grid, a step that is not a power of two or is finer than 2^-k_max, a
    particle due before the last block time) is run with the selection from
    t and dt: the result equals hermite_step's."""
    n = 5000
    x, v, m, _ = _c1_setup(H, n=n, seed=47)
    eps2 = (4.0 / n) ** 2
    params = H.dt_params(0.02, H.DT_PAPER, 3, 18)
    s0 = H.State(x, v, m, TB)
    ctx.initialize(s0, eps2, params, H.FP64)
    torch.cuda.synchronize()
    g = s0.to_numpy()
    t, dt = g["t"].copy(), g["dt"].copy()
    if case == "t_off_grid":
        t[17] = 1
    elif case == "dt_not_pow2":
        dt[17] = 3 * (1 << 6)
    elif case == "dt_below_floor":
        dt[17] = 1
    else:
        # particle 17 at t = 2 dt with its next time before another's t
        t[:] = 0
        dt[:] = 1 << (TB - 8)
        t[18] = 4 * dt[18]
        t[17] = 0
    s0.t.copy_(_dev(t))
    s0.dt.copy_(_dev(dt))
    torch.cuda.synchronize()
    _run_vs_steps(H, ctx, s0, eps2, params, H.FP64, 20)


def test_run_order_selection_to_the_end(H, ctx):
    """A run to T_end through the step-size order (n = 3000, several calls)
    ends with every particle at T_end, then steps change nothing; the same
    run of hermite_step calls gives the same state."""
    n = 3000
    x, v, m, _ = _c1_setup(H, n=n, seed=49)
    eps2 = (4.0 / n) ** 2
    params = H.dt_params(0.05, H.DT_AARSETH, 6, 14)
    s0 = H.State(x, v, m, TB)
    ctx.initialize(s0, eps2, params, H.FP64)
    T_end = 1 << (TB - 6)       # one coarsest step
    sa = s0.clone()
    total = calls = 0
    while True:
        st, it, done = ctx.run(sa, eps2, params, T_end, H.FP64, sync_every=3, max_steps=7,
                               with_done=True)
        total += st
        calls += 1
        if done:
            break
    torch.cuda.synchronize()
    g = sa.to_numpy()
    assert np.all(g["t"] == T_end) and total > 20 and calls > 3
    sb = s0.clone()
    for k in range(total + 5):
        ctx.step(sb, eps2, params, H.FP64, T_end=T_end, use_graph=(k % 2 == 0))
    torch.cuda.synchronize()
    for key in ("x", "v", "a", "j", "pot", "t", "dt"):
        assert torch.equal(getattr(sa, key), getattr(sb, key)), key
    st, it = ctx.run(sa, eps2, params, T_end, H.FP64, sync_every=16)
    assert st == 0 and it == 0


def test_check_finite_and_run_stops_on_nonfinite(H, ctx):
    """hermite_check_finite flags a NaN anywhere in x, v, a, j; a run of a
    system with two coincident particles and zero softening (infinite
    force) stops with HERMITE_ENONFINITE instead of integrating on."""
    x, v, m, eps2 = _c1_setup(H, n=256, seed=41)
    s = H.State(x, v, m, TB)
    params = H.dt_params(0.02, H.DT_PAPER, 3, 20)
    ctx.initialize(s, eps2, params, H.FP64)
    assert ctx.check_finite(s)
    for key, d, i in (("x", 1, 7), ("v", 2, 200), ("a", 0, 255), ("j", 2, 0)):
        bad = s.clone()
        getattr(bad, key)[d, i] = float("nan")
        assert not ctx.check_finite(bad), key
    x2 = x.copy()
    x2[:, 5] = x2[:, 9]                     # particles 5 and 9 coincide
    s2 = H.State(x2, v, m, TB)
    ctx.initialize(s2, 0.0, params, H.FP64)
    with pytest.raises(H.HermiteError) as err:
        ctx.run(s2, 0.0, params, 1 << (TB - 3), H.FP64, use_graph=True, sync_every=16)
    assert err.value.code == H.ENONFINITE


def test_counters_and_clamped(H, ctx):
    """A hard binary forces steps below 2^-k_max: the clamped count rises."""
    from paper_1104_2700_amd import inputs
    x, v, m = inputs.kepler_pair(1e-2, 0.5, 0.5, 0.5, 0.0)
    s = H.State(x, v, m, TB)
    params = H.dt_params(0.02, H.DT_PAPER, 3, 8)
    c0 = ctx.counters()
    ctx.initialize(s, 0.0, params, H.FP64)
    ctx.run(s, 0.0, params, 1 << (TB - 3), H.FP64, use_graph=False, sync_every=8)
    c1 = ctx.counters()
    assert c1["clamped"] > c0["clamped"]
    assert c1["steps"] > c0["steps"]


def test_context_destroy_frees_run_scratch(H):
    """Contexts that ran (step-size order, sweep, graphs) give back their
    device scratch when destroyed: free device memory is unchanged over
    repeated create / run / destroy cycles (n = 400000: the order alone is
    3.2 MB per context)."""
    from paper_1104_2700_amd import inputs
    n = 400000
    x, v, m = inputs.plummer(n, 51)
    eps2 = (4.0 / n) ** 2
    params = H.dt_params(0.02, H.DT_PAPER, 3, 20)
    s0 = H.State(x, v, m, TB)
    c = H.Context(0)
    c.initialize(s0, eps2, params, H.MIXED)
    c.close()
    s = s0.clone()
    torch.cuda.synchronize()

    def cycle():
        c = H.Context(0)
        s.t.copy_(s0.t)
        s.dt.copy_(s0.dt)
        c.run(s, eps2, params, 1 << (TB - 3), H.MIXED, sync_every=8, max_steps=8)
        c.close()
        torch.cuda.synchronize()

    cycle()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(6):
        cycle()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 < 4 << 20, (free0, free1)
