"""Why the mixed path's jerk bar has a second clause (CPU; no GPU code).

The mixed scheme (Section 3.2) rounds the FP64 relative coordinates and
velocities to FP32 before the pair arithmetic.  Emulated here with only that
rounding (every later operation in FP64) on the 1024-particle evaluation
sample of the N = 65536 Plummer state: the accelerations meet the 1e-6
relative bar outright, but a jerk with strong cancellation does not, even
though this emulation is more accurate than any FP32 pair arithmetic.  Its
error is still a small multiple of u32 * sum_j |jerk_ij|, which is the
second clause of the bar the GPU parity tests apply (16 u32 sum_j |term|)."""
import numpy as np

from oracle import oracle as O
from paper_1104_2700_amd import inputs

U32 = 2.0 ** -24


def test_rounded_differences_alone_reach_the_jerk_bar():
    n = 65536
    x, v, m = inputs.plummer(n, 3)
    eps2 = (4.0 / n) ** 2
    sample = np.sort(np.random.default_rng(1003).choice(n, 1024, replace=False)).astype(np.int32)
    ra, rj, _, cond = O.force(x, v, m, sample, eps2, with_cond=True)
    f32 = np.float32
    ej = np.empty(sample.shape[0])
    ea = np.empty(sample.shape[0])
    scaled = np.empty(sample.shape[0])
    for k, i in enumerate(sample):
        dx = (x - x[:, i:i + 1]).astype(f32).astype(np.float64)
        dv = (v - v[:, i:i + 1]).astype(f32).astype(np.float64)
        r2 = (dx * dx).sum(0) + eps2
        ri = 1.0 / np.sqrt(r2)
        ri[i] = 0.0                                   # no self term
        mr3 = m * ri ** 3
        rv = (dx * dv).sum(0)
        a = (mr3 * dx).sum(1)                         # eq. (acc)
        j = (mr3 * (dv - 3.0 * rv * ri * ri * dx)).sum(1)   # eq. (jrk)
        dj = np.linalg.norm(j - rj[:, k])
        ej[k] = dj / np.linalg.norm(rj[:, k])
        ea[k] = np.linalg.norm(a - ra[:, k]) / np.linalg.norm(ra[:, k])
        scaled[k] = dj / (U32 * cond[1, k])
    assert ea.max() < 1e-7                 # accelerations: far inside 1e-6
    assert ej.max() > 1e-6                 # a jerk misses 1e-6 from the rounding alone
    assert np.count_nonzero(ej > 1e-6) <= 4
    assert scaled.max() < 4.0              # within a few u32 of sum_j |jerk_ij|
