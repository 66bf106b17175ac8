"""Seeded synthetic initial conditions.

This module is shared by the GPU path's tests/benchmark and by the oracle's
tests.  It contains sampling only -- none of the method's arithmetic (no
force, potential, predictor, corrector or timestep code) -- so that sharing
it couples nothing between the two sides.

Units are the standard N-body (Henon) units the paper uses (Section 4):
G = M = 1, virial radius 1, total energy -1/4.

Plummer model (Section 4 workload): radii by inverse CDF of the cumulative
mass M(<r) = r^3 / (1 + r^2)^{3/2}, isotropic directions, speeds by
rejection from g(q) = q^2 (1 - q^2)^{7/2} with v = q sqrt(2) (1 + r^2)^{-1/4}
(the escape speed at r), centre-of-mass frame, then the analytic scaling of
a Plummer sphere of scale radius b to Henon units (b = 3 pi / 16), which
makes E = -1/4 in the large-N limit.  The mass fraction X is drawn from
(0, cap] to avoid the unbounded tail.
"""
from __future__ import annotations

import numpy as np

HENON_B = 3.0 * np.pi / 16.0


def _isotropic(rng, r):
    """Vectors of length ``r`` with uniformly random directions."""
    n = r.shape[0]
    z = 1.0 - 2.0 * rng.random(n)
    phi = 2.0 * np.pi * rng.random(n)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * s * np.cos(phi), r * s * np.sin(phi), r * z])


def plummer(n: int, seed: int, cap: float = 0.999, total_mass: float = 1.0,
            masses: np.ndarray | None = None):
    """Plummer sphere of ``n`` particles in Henon units (equal masses).

    Returns ``(x, v, m)`` with ``x, v`` of shape (3, n) float64 and ``m``
    (n,) float64 summing to ``total_mass``.  ``masses`` replaces the equal
    masses (it is normalised to ``total_mass``).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.default_rng(seed)
    X = cap * (1.0 - rng.random(n))                 # (0, cap]
    r = 1.0 / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    x = _isotropic(rng, r)
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        qq = rng.random(todo.size)
        yy = 0.1 * rng.random(todo.size)
        ok = yy < qq * qq * (1.0 - qq * qq) ** 3.5
        q[todo[ok]] = qq[ok]
        todo = todo[~ok]
    speed = q * np.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    v = _isotropic(rng, speed)
    if masses is None:
        m = np.full(n, total_mass / n)
    else:
        m = np.asarray(masses, dtype=np.float64) * (total_mass / np.sum(masses))
    x -= (x @ m)[:, None] / total_mass
    v -= (v @ m)[:, None] / total_mass
    x *= HENON_B
    v /= np.sqrt(HENON_B)
    return np.ascontiguousarray(x), np.ascontiguousarray(v), m


def kepler_pair(a: float, e: float, m1: float = 0.5, m2: float = 0.5,
                mean_anomaly: float = 0.0):
    """Two bodies on a Kepler orbit (G = 1), centre of mass at rest at 0.

    The relative orbit lies in the x-y plane with periapsis on +x.  Returns
    ``(x, v, m)`` with shapes (3, 2), (3, 2), (2,).  Used for the
    closed-form orbit checks; ``kepler_relative`` gives the same orbit at
    any time.
    """
    rel_x, rel_v = kepler_relative(a, e, m1 + m2, mean_anomaly)
    mt = m1 + m2
    x = np.stack([-m2 / mt * rel_x, m1 / mt * rel_x], axis=1)
    v = np.stack([-m2 / mt * rel_v, m1 / mt * rel_v], axis=1)
    return x, v, np.array([m1, m2])


def solve_kepler(M: float, e: float) -> float:
    """Eccentric anomaly E with E - e sin E = M (Newton iteration)."""
    M = np.fmod(M, 2.0 * np.pi)
    E = M if e < 0.8 else np.pi
    for _ in range(100):
        f = E - e * np.sin(E) - M
        dE = f / (1.0 - e * np.cos(E))
        E -= dE
        if abs(dE) < 1e-16:
            break
    return float(E)


def kepler_relative(a: float, e: float, mt: float, mean_anomaly: float):
    """Relative position and velocity (r2 - r1, v2 - v1) on a Kepler orbit."""
    nmot = np.sqrt(mt / a ** 3)
    E = solve_kepler(mean_anomaly, e)
    cE, sE = np.cos(E), np.sin(E)
    fac = np.sqrt(1.0 - e * e)
    rel_x = np.array([a * (cE - e), a * fac * sE, 0.0])
    den = 1.0 - e * cE
    rel_v = np.array([-a * nmot * sE / den, a * nmot * fac * cE / den, 0.0])
    return rel_x, rel_v


def _random_rotation(rng):
    """A uniformly random rotation matrix (QR of a Gaussian matrix)."""
    A = rng.standard_normal((3, 3))
    Q, R = np.linalg.qr(A)
    Q = Q @ np.diag(np.sign(np.diag(R)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def salpeter_masses(n: int, rng, alpha: float = 2.35, ratio: float = 100.0):
    """Masses from dN/dm ~ m^-alpha on [1, ratio] (inverse CDF), unnormalised."""
    u = rng.random(n)
    p = 1.0 - alpha
    lo, hi = 1.0, ratio
    return (lo ** p + u * (hi ** p - lo ** p)) ** (1.0 / p)


def plummer_imf_binaries(n: int, seed: int, binary_fraction: float = 0.1,
                         a_range=(1e-4, 1e-2), alpha: float = 2.35,
                         ratio: float = 100.0, cap: float = 0.999):
    """Plummer sphere with a Salpeter mass spectrum and primordial binaries.

    ``binary_fraction`` of the ``n`` particles are binary members
    (n * fraction / 2 pairs).  Each member's mass is drawn from the mass
    function; semi-major axes are log-uniform in ``a_range``; eccentricities
    are thermal (e = sqrt(U)); orientation and mean anomaly are random.  A
    binary's centre of mass takes the position and velocity of one Plummer
    particle.  Total mass is 1; returns ``(x, v, m)`` in Henon units.
    """
    rng = np.random.default_rng(seed)
    n_pairs = int(round(n * binary_fraction / 2.0))
    n_single = n - 2 * n_pairs
    n_com = n_single + n_pairs
    mass = salpeter_masses(n, rng, alpha, ratio)
    mass /= mass.sum()
    m_single = mass[:n_single]
    m1 = mass[n_single:n_single + n_pairs]
    m2 = mass[n_single + n_pairs:]
    m_com = np.concatenate([m_single, m1 + m2])
    xc, vc, _ = plummer(n_com, seed * 7919 + 1, cap=cap, masses=m_com)
    x = np.empty((3, n)); v = np.empty((3, n)); m = np.empty(n)
    x[:, :n_single] = xc[:, :n_single]
    v[:, :n_single] = vc[:, :n_single]
    m[:n_single] = m_single
    la, lb = np.log(a_range[0]), np.log(a_range[1])
    for k in range(n_pairs):
        a = float(np.exp(rng.uniform(la, lb)))
        e = float(np.sqrt(rng.random()))
        M = float(2.0 * np.pi * rng.random())
        R = _random_rotation(rng)
        ma, mb = float(m1[k]), float(m2[k])
        rx, rv = kepler_relative(a, e, ma + mb, M)
        rx, rv = R @ rx, R @ rv
        c = n_single + 2 * k
        cx, cv = xc[:, n_single + k], vc[:, n_single + k]
        mt = ma + mb
        x[:, c] = cx - mb / mt * rx
        x[:, c + 1] = cx + ma / mt * rx
        v[:, c] = cv - mb / mt * rv
        v[:, c + 1] = cv + ma / mt * rv
        m[c], m[c + 1] = ma, mb
    return np.ascontiguousarray(x), np.ascontiguousarray(v), m


def ensemble(n_clusters: int = 256, seed: int = 4, n_min: int = 256,
             n_max: int = 8192):
    """Independent Plummer clusters, N_c log-uniform in [n_min, n_max].

    Cluster c uses seed ``1000 * seed + c`` and its own Henon units
    (M_c = 1).  Returns ``(x, v, m, offsets)`` with the clusters
    concatenated and ``offsets`` int64 (C+1,), plus the per-cluster
    softening eps_c = 4 / N_c as a float64 array.
    """
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(np.log(n_min), np.log(n_max),
                                       n_clusters))).astype(np.int64)
    offsets = np.zeros(n_clusters + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    xs, vs, ms = [], [], []
    for c in range(n_clusters):
        x, v, m = plummer(int(sizes[c]), 1000 * seed + c)
        xs.append(x); vs.append(v); ms.append(m)
    eps = 4.0 / sizes.astype(np.float64)
    return (np.ascontiguousarray(np.concatenate(xs, axis=1)),
            np.ascontiguousarray(np.concatenate(vs, axis=1)),
            np.concatenate(ms), offsets, eps)


def random_active(n: int, n_act: int, seed: int) -> np.ndarray:
    """A sorted random subset of ``n_act`` distinct indices in [0, n)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=n_act, replace=False)).astype(np.int32)


def synced_block_times(n: int, seed: int, tick_bits: int, k_min: int,
                       k_max: int, T: int):
    """Random (t, dt) tick pairs that are valid block-step states at time T.

    Every dt is 2^-k ticks with k in [k_min, k_max], every t is a multiple of
    its dt, and t <= T < t + dt... used by the selection and predictor
    tests.  Returns ``(t, dt)`` int64 arrays.
    """
    rng = np.random.default_rng(seed)
    k = rng.integers(k_min, k_max + 1, size=n)
    dt = (np.int64(1) << (tick_bits - k)).astype(np.int64)
    t = (T // dt) * dt
    return t.astype(np.int64), dt
