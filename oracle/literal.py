"""Literal transcription of Algorithm 1 for tiny inputs (n <= 12).

TEST INFRASTRUCTURE ONLY.  A second, independent reading of Section 2 in
pure Python: every max and sum runs over exactly the index set printed in
Eqs. (2)-(4) (k' != k; i' not in {i,k}; i' != k), with no top-2 or
column-sum rewriting, so it cross-checks the O(n^2) oracle in apo.c.
"""
from __future__ import annotations

import math


def iterate(S, lam, n_iter, A=None, R=None):
    """Run n_iter damped iterations; returns (R, A, decisions) as lists."""
    n = len(S)
    R = [[0.0] * n for _ in range(n)] if R is None else [row[:] for row in R]
    A = [[0.0] * n for _ in range(n)] if A is None else [row[:] for row in A]
    dec = [0] * n
    for _ in range(n_iter):
        # Step 2, Eq. (2), damped
        Rn = [[0.0] * n for _ in range(n)]
        for i in range(n):
            for k in range(n):
                m = -math.inf
                for kp in range(n):
                    if kp != k:
                        m = max(m, A[i][kp] + S[i][kp])
                Rn[i][k] = lam * R[i][k] + (1.0 - lam) * (S[i][k] - m)
        R = Rn
        # Step 3, Eqs. (3) and (4), damped
        An = [[0.0] * n for _ in range(n)]
        for i in range(n):
            for k in range(n):
                if i == k:
                    tot = 0.0
                    for ip in range(n):
                        if ip != k:
                            tot += max(0.0, R[ip][k])
                    upd = tot
                else:
                    tot = 0.0
                    for ip in range(n):
                        if ip != i and ip != k:
                            tot += max(0.0, R[ip][k])
                    upd = min(0.0, R[k][k] + tot)
                An[i][k] = lam * A[i][k] + (1.0 - lam) * upd
        A = An
        for i in range(n):
            best, bk = -math.inf, 0
            for k in range(n):
                v = A[i][k] + R[i][k]
                if v > best:
                    best, bk = v, k
            dec[i] = bk
    return R, A, dec
