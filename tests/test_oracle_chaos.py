"""At the paper's damping (0.5) the iteration on the 2-D workload amplifies
rounding: two FP64 runs of the oracle that differ only in the order of their
column sums (the same points, relabelled) drift apart to O(range) within
100 iterations and mostly end on different exemplar sets.  So no exemplar
parity between an FP32 GPU run and the FP64 oracle can be asked for on that
workload at damping 0.5 (the GPU tests compare messages there for the
first iterations only, and use damping 0.9 for longer runs).  At damping 0.9
the same relabelled runs agree.

The relabelling is checked to be exact where rounding has not yet grown
(after 10 iterations the two runs agree to 1e-12 of the range), so the later
divergence is the iteration's own sensitivity, not a mistake in the test.
"""
import numpy as np
import pytest

import oracle
import synth

SEEDS = range(1001, 1011)   # the ten 2-D workload seeds (n = 1000, 10 components)


def _pair(seed):
    pts = synth.gaussian_2d(n=1000, k=10, seed=seed)
    S = oracle.prepare(oracle.similarity(pts.X), "median", seed=seed).S
    P = np.random.default_rng(seed).permutation(S.shape[0])
    return S, P, np.ascontiguousarray(S[np.ix_(P, P)])


def _msg_gap(S, P, Sp, lam, T):
    inv = np.argsort(P)
    a = oracle.ap(S, lam, T, 0, finalize_labels=False)
    b = oracle.ap(Sp, lam, T, 0, finalize_labels=False)
    rng = S.max() - S.min()
    return max(np.abs(a.R - b.R[np.ix_(inv, inv)]).max(), np.abs(a.A - b.A[np.ix_(inv, inv)]).max()) / rng


@pytest.fixture(scope="module")
def runs():
    out = {}
    for seed in SEEDS:
        S, P, Sp = _pair(seed)
        g10 = _msg_gap(S, P, Sp, 0.5, 10)
        g100 = _msg_gap(S, P, Sp, 0.5, 100)
        a = oracle.ap(S, 0.5, 200, 15, finalize_labels=False)
        b = oracle.ap(Sp, 0.5, 200, 15, finalize_labels=False)
        same = set(a.exemplars.tolist()) == set(P[b.exemplars].tolist())
        out[seed] = (g10, g100, same)
    return out


def test_relabelled_runs_agree_early(runs):
    assert all(g10 <= 1e-12 for g10, _, _ in runs.values())


def test_relabelled_runs_diverge_at_damping_half(runs):
    far = [s for s, (_, g100, _) in runs.items() if g100 > 1e-4]
    assert len(far) >= 8, runs
    differ = [s for s, (_, _, same) in runs.items() if not same]
    assert len(differ) >= 5, runs


def test_relabelled_runs_agree_at_damping_0_9():
    S, P, Sp = _pair(1001)
    a = oracle.ap(S, 0.9, 1000, 15)
    b = oracle.ap(Sp, 0.9, 1000, 15)
    assert a.converged and b.converged and a.iterations == b.iterations
    assert set(a.exemplars.tolist()) == set(P[b.exemplars].tolist())
    assert _msg_gap(S, P, Sp, 0.9, 100) <= 1e-9
