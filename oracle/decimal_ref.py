"""50-digit decimal brute force of the pair sums (test infrastructure only).

Equations (acc), (jrk), (pot) of Section 2 evaluated in Python ``decimal``
arithmetic at 50 significant digits for tiny N.  It pins the rounding of the
binary64 oracle (its compensated sums must agree to ~1e-15), not its
formula; the formula is pinned by closed forms, derivatives and invariants
in the tests.
"""
from __future__ import annotations

from decimal import Decimal, getcontext

getcontext().prec = 50


def pair_sums(x, v, m, eps2, i):
    """(acc[3], jerk[3], pot) of particle i as Decimals, j != i."""
    n = len(m)
    D = Decimal
    e2 = D(float(eps2))
    ax = [D(0)] * 3
    jx = [D(0)] * 3
    ph = D(0)
    xi = [D(float(x[d][i])) for d in range(3)]
    vi = [D(float(v[d][i])) for d in range(3)]
    for j in range(n):
        if j == i:
            continue
        r = [D(float(x[d][j])) - xi[d] for d in range(3)]
        w = [D(float(v[d][j])) - vi[d] for d in range(3)]
        s = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + e2
        rs = s.sqrt()
        mj = D(float(m[j]))
        mq3 = mj / (s * rs)
        rv = r[0] * w[0] + r[1] * w[1] + r[2] * w[2]
        for d in range(3):
            ax[d] += mq3 * r[d]
            jx[d] += mq3 * (w[d] - 3 * rv / s * r[d])
        ph -= mj / rs
    return ax, jx, ph
