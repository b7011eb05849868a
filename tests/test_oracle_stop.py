"""Pins of the oracle's stop rules (Algorithm 1, Step 4) other than the
exemplar-set rule: the fixed iteration count and the message-change
threshold.

The message changes are measured here independently of the oracle's own
bookkeeping: two fixed-count runs from zero messages, t-1 and t iterations
(runs compose, so the second equals one more iteration after the first),
differenced with numpy.  A stop one iteration early or late, a test on only
one of the two messages, or a test before the second iteration fails one of
these.
"""
import numpy as np
import pytest

import oracle
import synth


def _S(n=120, seed=1007):
    pts = synth.gaussian_2d(n=n, k=5, seed=seed)
    return oracle.prepare(oracle.similarity(pts.X), "median", seed=seed).S


def _changes(S, lam, T):
    """delta_R[t], delta_A[t] = max |R_t - R_{t-1}|, max |A_t - A_{t-1}| for t = 1..T."""
    dR, dA = [np.inf], [np.inf]
    prev = oracle.ap(S, lam, 1, 0, finalize_labels=False)
    prevR, prevA = np.abs(prev.R).max(), np.abs(prev.A).max()   # t = 1 from zeros
    dR.append(prevR)
    dA.append(prevA)
    for t in range(2, T + 1):
        cur = oracle.ap(S, lam, t, 0, finalize_labels=False)
        dR.append(float(np.abs(cur.R - prev.R).max()))
        dA.append(float(np.abs(cur.A - prev.A).max()))
        prev = cur
    return np.asarray(dR), np.asarray(dA)


@pytest.fixture(scope="module")
def seq():
    S = _S()
    T = 120
    dR, dA = _changes(S, 0.9, T)
    return S, T, dR, dA


def test_runs_compose():
    """t iterations from zero equal t-1 iterations, then one more from their
    messages (the property the change measurement relies on)."""
    S = _S(60, 1009)
    a = oracle.ap(S, 0.9, 7, 0, finalize_labels=False)
    b = oracle.ap(S, 0.9, 6, 0, finalize_labels=False)
    c = oracle.ap(S, 0.9, 1, 0, A0=b.A, R0=b.R, finalize_labels=False)
    assert np.array_equal(a.R, c.R) and np.array_equal(a.A, c.A)


@pytest.mark.parametrize("frac", [0.3, 0.1, 0.03, 0.01, 0.003])
def test_message_threshold_stops_at_first_small_change(seq, frac):
    S, T, dR, dA = seq
    rng = S.max() - S.min()
    tol = frac * rng
    d = np.maximum(dR, dA)
    small = [t for t in range(2, T + 1) if d[t] <= tol]
    r = oracle.ap(S, 0.9, T, 0, msg_tol=tol, finalize_labels=False)
    if not small:
        assert not r.converged and r.iterations == T
        return
    assert r.converged and r.iterations == small[0]
    # the messages are those of that iteration
    ref = oracle.ap(S, 0.9, small[0], 0, finalize_labels=False)
    assert np.array_equal(r.R, ref.R) and np.array_equal(r.A, ref.A)


def test_threshold_needs_both_messages(seq):
    """A tolerance between the two changes of an iteration does not stop it."""
    S, T, dR, dA = seq
    # an iteration whose R and A changes are far apart
    t = next(t for t in range(2, T + 1) if max(dR[t], dA[t]) > 4 * min(dR[t], dA[t]))
    tol = np.sqrt(dR[t] * dA[t])
    r = oracle.ap(S, 0.9, t, 0, msg_tol=tol, finalize_labels=False)
    assert r.iterations == t
    earlier = [u for u in range(2, t) if max(dR[u], dA[u]) <= tol]
    assert r.converged == bool(earlier)


def test_threshold_not_tested_on_first_iteration():
    """A huge tolerance stops at t = 2, never at t = 1."""
    S = _S(40, 1011)
    r = oracle.ap(S, 0.9, 50, 0, msg_tol=1e30, finalize_labels=False)
    assert r.converged and r.iterations == 2


def test_zero_tolerance_runs_to_the_cap():
    S = _S(40, 1013)
    r = oracle.ap(S, 0.9, 30, 0, msg_tol=0.0, finalize_labels=False)
    assert not r.converged and r.iterations == 30


def test_exemplar_rule_takes_precedence_and_both_apply():
    """With both rules on, the run stops at the earlier of the two stops."""
    S = _S(100, 1015)
    a = oracle.ap(S, 0.9, 1000, 15)
    rng = S.max() - S.min()
    b = oracle.ap(S, 0.9, 1000, 0, msg_tol=1e-6 * rng, finalize_labels=False)
    c = oracle.ap(S, 0.9, 1000, 15, msg_tol=1e-6 * rng, finalize_labels=False)
    assert c.iterations == min(a.iterations, b.iterations)
