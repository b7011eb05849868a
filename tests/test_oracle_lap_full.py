"""Pins of the oracle's full landmark method (Algorithm 3, Steps 1-4).

* Step 2's threshold on a hand-worked 1-D example: every distance and
  max_distance is a small binary fraction, so the assigned and unassigned
  points follow by inspection (including a point exactly at its class's
  max_distance, which stays unassigned: "<" is strict).
* The medoid against the identity sum_i |x_i - x_k|^2 = sum_i |x_i - mu|^2
  + m |x_k - mu|^2 (the medoid is the member nearest the mean) and against
  a brute-force distance matrix.
* The landmark draw: the SplitMix64 stream against its published outputs,
  and a Fisher-Yates prefix is a set of distinct positions.
* With every point a landmark, Steps 2-3 have nothing to do and the centres
  before Step 4 are exactly Algorithm 1's exemplars.
* Recursion: when more than m0 points are left, the next level runs on
  exactly those points with min(L, m0) landmarks; the final labels are the
  nearest exemplars (brute force) and exemplars label themselves.
"""
import json
import os

import numpy as np

import oracle
import synth
from oracle import brute
from oracle import lap_full as LF


def _hand_case():
    # landmarks 0..5 form two classes {0,1,2} and {3,4,5} around 1.0 and 11.0
    x = np.array([0.0, 1.0, 2.0, 10.0, 11.0, 12.0,      # landmarks
                  0.5, 1.5, 3.5, 10.75, 20.0, 0.0],      # other points
                 dtype=np.float32)[:, None]
    return x, np.arange(6, dtype=np.int64)


def test_step2_threshold_hand_example():
    X, M = _hand_case()
    C1 = np.array([1, 4], dtype=np.int64)
    cls = np.array([1, 1, 1, 4, 4, 4], dtype=np.int64)
    Q = np.arange(6, 12, dtype=np.int64)
    assigned, U = LF.step2(X, Q, M, C1, cls)
    # max_distance is 1 for both classes; distances to the nearest centre:
    # 0.25, 0.25, 6.25, 0.0625, 81, 1 (the last equals max_distance)
    assert assigned.tolist() == [True, True, False, True, False, False]
    assert U.tolist() == [8, 10, 11]


def test_step1_on_the_hand_example_is_the_optimum():
    """The landmark AP of the hand example reaches the brute-force optimum
    {1, 4} (its preference set by hand), so the classes above are Step 1's."""
    X, M = _hand_case()
    S = oracle.similarity(X[M])
    np.fill_diagonal(S, -3.0)
    r = oracle.ap(S, 0.9, 500, 15)
    best, bestE = brute.optimum(S)
    assert tuple(r.exemplars.tolist()) == bestE == (1, 4)
    assert r.idx.tolist() == [1, 1, 1, 4, 4, 4]


def test_full_method_on_the_hand_example():
    X, M = _hand_case()
    r = LF.lap_full(X, M, 6, seed=1, lam=0.9, m0=10, pref=-3.0, noise_rel=0.0)
    top = r.levels[0]
    assert top.step1_centres == 2 and top.assigned == 3 and top.unassigned == 3 and top.step3 == "ap"
    assert np.all(r.idx[r.exemplars] == r.exemplars)
    _, d = oracle.nearest_of(X, np.arange(X.shape[0]), r.exemplars)
    assert np.all(d[r.idx != np.arange(X.shape[0])] >= 0)


def test_medoid_is_the_member_nearest_the_mean():
    rng = np.random.default_rng(3)
    for t in range(20):
        m = int(rng.integers(2, 60))
        X = rng.normal(size=(200, 5)).astype(np.float32)
        members = np.sort(rng.choice(200, size=m, replace=False))
        k = oracle.medoid(X, members)
        Y = X[members].astype(np.float64)
        D = ((Y[:, None, :] - Y[None, :, :]) ** 2).sum(-1).sum(0)
        assert k == members[np.argmin(D)]
        mu = Y.mean(0)
        assert k == members[np.argmin(((Y - mu) ** 2).sum(1))]


def test_splitmix64_stream_published_values(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "splitmix64.json")))
    s = LF.splitmix64_stream(g["state"])
    assert [str(next(s)) for _ in range(5)] == g["outputs"]


def test_sample_positions_distinct_and_reproducible():
    a = LF.sample_positions(1000, 37, 11)
    b = LF.sample_positions(1000, 37, 11)
    assert np.array_equal(a, b) and np.unique(a).size == 37 and a.min() >= 0 and a.max() < 1000
    assert np.array_equal(LF.sample_positions(40, 40, 5), np.arange(40))


def test_all_points_as_landmarks_reduces_to_ap():
    pts = synth.gaussian_2d(n=300, k=4, seed=8)
    n = pts.X.shape[0]
    calls = []
    orig = LF._ap_centres

    def spy(X, P, *a):
        r = orig(X, P, *a)
        calls.append((P.copy(), r[0].copy()))
        return r
    LF._ap_centres = spy
    try:
        r = LF.lap_full(pts.X, np.arange(n), n, seed=8, lam=0.9, m0=1000)
    finally:
        LF._ap_centres = orig
    assert len(calls) == 1                       # Step 1 only: Steps 2-3 have nothing to do
    prep = oracle.prepare(oracle.similarity(pts.X), "median", seed=8)
    ref = oracle.ap(prep.S, 0.9, 2000, 15)
    assert np.array_equal(calls[0][1], ref.exemplars)
    assert r.levels[0].assigned == 0 and r.levels[0].unassigned == 0
    assert r.exemplars.size == ref.exemplars.size


def test_recursion_and_final_labels():
    pts = synth.gaussian_2d(n=6000, k=8, seed=9)
    X = pts.X
    r = LF.lap_full(X, None, 300, seed=9, lam=0.9, m0=60)
    lv = {s.level: s for s in r.levels}
    assert lv[0].unassigned > 60 and lv[0].step3 == "lap"
    assert lv[1].points == lv[0].unassigned and lv[1].landmarks == 60
    for s in r.levels:
        assert s.assigned + s.unassigned + s.landmarks == s.points
    n = X.shape[0]
    assert np.all(r.idx[r.exemplars] == r.exemplars)
    Xd = X.astype(np.float64)
    E = r.exemplars
    for i in np.random.default_rng(2).choice(n, 300, replace=False):
        if r.idx[i] == i:
            continue
        d = ((Xd[E] - Xd[i]) ** 2).sum(1)
        assert d[np.searchsorted(E, r.idx[i])] <= d.min() * (1 + 1e-12)
    dp = -sum(((Xd[i] - Xd[r.idx[i]]) ** 2).sum() for i in range(n) if r.idx[i] != i)
    assert abs(dp - r.dpsim) <= 1e-9 * abs(dp)
    assert r.expref == r.pref * E.size
