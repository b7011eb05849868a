"""Brute-force optimum of the AP energy for tiny inputs (n <= 10).

TEST INFRASTRUCTURE ONLY.  Enumerates every non-empty exemplar set E, forms
the valid configuration (exemplars label themselves, other points take the
exemplar of largest similarity) and returns the one of largest net
similarity, i.e. least energy E(c) = -sum_i s(i,c_i) of Section 2.
"""
from __future__ import annotations

import itertools

import numpy as np


def labels_for(S: np.ndarray, E) -> np.ndarray:
    n = S.shape[0]
    E = sorted(E)
    idx = np.empty(n, dtype=np.int64)
    for i in range(n):
        if i in E:
            idx[i] = i
        else:
            best, bk = -np.inf, E[0]
            for k in E:
                if S[i, k] > best:
                    best, bk = S[i, k], k
            idx[i] = bk
    return idx


def netsim(S: np.ndarray, E) -> float:
    idx = labels_for(S, E)
    return float(sum(S[i, idx[i]] for i in range(S.shape[0])))


def optimum(S: np.ndarray):
    """(best netsim, best exemplar set as a tuple) over all 2^n - 1 sets."""
    n = S.shape[0]
    assert n <= 12
    best, best_E = -np.inf, None
    for size in range(1, n + 1):
        for E in itertools.combinations(range(n), size):
            v = netsim(S, E)
            if v > best:
                best, best_E = v, E
    return best, best_E
