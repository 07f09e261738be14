"""Writes eq1_exact_tiny.json: exact rational solutions of Eq. 1 (Sec. 1.3).

The inputs are small integers chosen by hand (an SPD tridiagonal M, an
intercept plus a 0/1 covariate, three SNP columns of 0/1/2 dosages).  The
expected values come from oracle.exact (Fraction arithmetic, explicit
inverses), nothing else.  Run from the repository root:
    python tests/golden/make_eq1_exact.py
"""
import json
import os
import sys

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))
from oracle.exact import gls_exact  # noqa: E402

n = 7
M = [[0] * n for _ in range(n)]
for i in range(n):
    M[i][i] = 4
    if i + 1 < n:
        M[i][i + 1] = M[i + 1][i] = 1
M[0][n - 1] = M[n - 1][0] = 1          # a wrap-around relation keeps it dense-ish, still SPD
XL = [[1, s] for s in (0, 1, 1, 0, 1, 0, 0)]
y = [3, -1, 2, 0, 5, -2, 1]
XR = [[0, 1, 2, 1, 0, 2, 1],
      [2, 2, 1, 0, 0, 1, 0],
      [1, 0, 0, 1, 2, 2, 1]]

res = gls_exact(M, XL, y, XR)
fx = lambda q: f"{q.numerator}/{q.denominator}"
doc = {
    "citation": "Eq. 1, Sec. 1.3 (GLS sequence); values exact (Fraction arithmetic)",
    "n": n, "p": 3, "M": M, "XL": XL, "y": y, "XR_cols": XR,
    "b": [[fx(v) for v in b] for b, _, _ in res],
    "sigma2": [fx(s) for _, s, _ in res],
    "v": [fx(v) for _, _, v in res],
}
with open(os.path.join(os.path.dirname(__file__), "eq1_exact_tiny.json"), "w") as f:
    json.dump(doc, f, indent=1)
print("wrote eq1_exact_tiny.json")
