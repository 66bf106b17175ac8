"""Writes tests/golden/pair_sums.json: 50-digit values of equations (acc),
(jrk), (pot) (Section 2) for three tiny seeded configurations.

Calls only the oracle package (its decimal brute force).  Run from the
repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import decimal_ref  # noqa: E402


def main():
    cases = []
    for n, seed, eps2 in ((2, 101, 0.0), (3, 102, 1e-3), (6, 103, 2.5e-5)):
        rng = np.random.default_rng(seed)
        x = rng.normal(size=(3, n))
        v = rng.normal(size=(3, n))
        m = rng.uniform(0.1, 1.0, size=n)
        acc = [[None] * n for _ in range(3)]
        jerk = [[None] * n for _ in range(3)]
        pot = [None] * n
        for i in range(n):
            a, j, p = decimal_ref.pair_sums(x, v, m, eps2, i)
            for d in range(3):
                acc[d][i] = str(a[d])
                jerk[d][i] = str(j[d])
            pot[i] = str(p)
        cases.append({"n": n, "seed": seed, "eps2": eps2, "x": x.tolist(),
                      "v": v.tolist(), "m": m.tolist(), "acc": acc,
                      "jerk": jerk, "pot": pot,
                      "cite": "Section 2, equations (acc), (jrk), (pot)"})
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pair_sums.json")
    with open(out, "w") as f:
        json.dump(cases, f, indent=1)


if __name__ == "__main__":
    main()
