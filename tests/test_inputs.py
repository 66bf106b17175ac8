"""The synthetic workloads' recipes, against closed forms (CPU).

Plummer spheres in Henon units (G = M = 1, E = -1/4; Section 4's test
systems), the Salpeter-like mass spectrum, primordial binaries, and the
ensemble's log-uniform cluster sizes.  Statistical checks use tolerances of
several standard deviations at the sample sizes used."""
import numpy as np

from oracle import oracle as O
from paper_1104_2700_amd import inputs


def _energies(x, v, m):
    _, _, pot = O.force(x, v, m, np.arange(m.shape[0], dtype=np.int32), 0.0)
    K = 0.5 * float(np.sum(m * np.sum(v * v, axis=0)))
    W = 0.5 * float(np.sum(m * pot))
    return K, W


def test_plummer_is_in_henon_units():
    n = 4096
    x, v, m = inputs.plummer(n, 17)
    assert x.shape == (3, n) and v.shape == (3, n) and m.shape == (n,)
    assert abs(m.sum() - 1.0) < 1e-14
    assert np.abs(x @ m).max() < 1e-14 and np.abs(v @ m).max() < 1e-14
    K, W = _energies(x, v, m)
    # Henon units: K = 1/4, W = -1/2, E = -1/4 (finite-N and the mass cap
    # at 0.999 shift these by a few per cent)
    assert abs(K - 0.25) < 0.02
    assert abs(W + 0.5) < 0.03
    assert abs(2.0 * K / -W - 1.0) < 0.08
    # half-mass radius of a Plummer sphere: b / sqrt(2^(2/3) - 1), b = 3 pi / 16
    rh = 3.0 * np.pi / 16.0 / np.sqrt(2.0 ** (2.0 / 3.0) - 1.0)
    r = np.sqrt(np.sum(x * x, axis=0))
    assert abs(np.median(r) / rh - 1.0) < 0.05


def test_mass_spectrum_mean_and_range():
    rng = np.random.default_rng(5)
    alpha, ratio, n = 2.35, 100.0, 200000
    mass = inputs.salpeter_masses(n, rng, alpha, ratio)
    assert mass.min() >= 1.0 and mass.max() <= ratio
    # mean of dN/dm ~ m^-alpha on [1, ratio]
    mean = ((ratio ** (2 - alpha) - 1) / (2 - alpha)) / ((ratio ** (1 - alpha) - 1) / (1 - alpha))
    assert abs(mass.mean() / mean - 1.0) < 0.02


def test_binaries_are_bound_with_the_stated_axes():
    n = 2048
    x, v, m = inputs.plummer_imf_binaries(n, 9)
    assert abs(m.sum() - 1.0) < 1e-12
    assert m.max() / m.min() <= 100.0 * (1 + 1e-12)
    n_pairs = int(round(n * 0.1 / 2.0))
    n_single = n - 2 * n_pairs
    a_fit = np.empty(n_pairs)
    for k in range(n_pairs):
        c = n_single + 2 * k
        dr = x[:, c + 1] - x[:, c]
        dv = v[:, c + 1] - v[:, c]
        mt = m[c] + m[c + 1]
        r = np.linalg.norm(dr)
        # vis-viva: 1/a = 2/r - v^2 / (G M)
        a_fit[k] = 1.0 / (2.0 / r - np.dot(dv, dv) / mt)
    assert np.all(a_fit > 0)                         # every pair is bound
    assert a_fit.min() >= 1e-4 * (1 - 1e-9) and a_fit.max() <= 1e-2 * (1 + 1e-9)


def test_ensemble_sizes_and_units():
    x, v, m, off, eps = inputs.ensemble(256, 4)
    sizes = np.diff(off)
    assert off[0] == 0 and off[-1] == m.shape[0] == x.shape[1]
    assert sizes.min() >= 256 and sizes.max() <= 8192
    # log-uniform on [256, 8192]: mean of ln N_c is the midpoint
    mid = 0.5 * (np.log(256.0) + np.log(8192.0))
    assert abs(np.log(sizes).mean() - mid) < 0.25
    assert np.allclose(eps, 4.0 / sizes)
    for c in range(0, 256, 37):
        assert abs(m[off[c]:off[c + 1]].sum() - 1.0) < 1e-12
