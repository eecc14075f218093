"""Writes tests/golden/tiny_exact.json: tiny integer GLS problems and their
exact b_i (Eq. (1) of the paper), computed only with oracle/exact.py.

The paper prints no worked numerical example, so these fixtures hold exact
rational values of the definition instead.  Rerun with
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.exact import gls_exact  # noqa: E402


def case(seed, n, p_L, p_R, m, t):
    rng = np.random.default_rng(seed)
    A = rng.integers(-3, 4, (n, n))
    M = A @ A.T + n * np.eye(n, dtype=np.int64)          # SPD, integer
    XL = np.hstack([np.ones((n, 1), np.int64), rng.integers(-3, 4, (n, p_L - 1))])
    XR = rng.integers(0, 3, (n, m * p_R))                 # genotypes in {0,1,2}
    Y = rng.integers(-9, 10, (n, t))
    b = gls_exact(M, XL, XR, Y, p_R)
    return {
        "seed": seed, "n": n, "p_L": p_L, "p_R": p_R, "m": m, "t": t,
        "M": M.tolist(), "XL": XL.tolist(), "XR": XR.tolist(), "Y": Y.tolist(),
        "b": [[[f"{v.numerator}/{v.denominator}" for v in bj] for bj in bi] for bi in b],
    }


def main():
    cases = [case(1, 6, 2, 1, 4, 1), case(2, 8, 3, 1, 5, 2), case(3, 9, 2, 2, 3, 1),
             case(4, 11, 4, 1, 3, 3), case(5, 12, 3, 3, 2, 1)]
    doc = {"about": "Exact rational b_i = (X_i^T M^-1 X_i)^-1 X_i^T M^-1 y (paper Sec. 1, Eq. (1)) "
                    "for tiny integer inputs; written by tests/golden/make_golden.py from oracle/exact.py.",
           "cases": cases}
    with open(os.path.join(HERE, "tiny_exact.json"), "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
