"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test is chosen so that a plausible slip in the oracle (a dropped term,
a wrong sign or index, a transposed operand, damping on the wrong side, an
off-by-one in the stop rule) fails at least one of them:

* a hand-worked example of Algorithm 1 (exact binary fractions);
* a literal O(n^3) transcription of Eqs. (2)-(4) on tiny, asymmetric inputs;
* brute-force enumeration of exemplar sets (the energy of Section 2);
* closed forms (n=2 fixed points, very large preferences, the first
  iteration from zero messages);
* invariants (sign of the availabilities, exact power-of-two scaling, row
  shifts of S, fixed-point residual);
* library routines (scipy distances, numpy median) and published SplitMix64
  output values.
"""
import json
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
from oracle import brute, literal
import synth


def _rand_S(n, seed, asym=True):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, 2)).astype(np.float32)
    S = oracle.similarity(x)
    if asym:
        S = S + rng.uniform(-0.3, 0.3, size=(n, n))   # break symmetry on purpose
    np.fill_diagonal(S, np.median(S[~np.eye(n, dtype=bool)]) + rng.uniform(-0.5, 0.5, size=n))
    return S


# ---------------------------------------------------------------------------
# Hand-worked example
# ---------------------------------------------------------------------------
def test_four_point_example(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "four_points.json")))
    x = np.asarray(g["x"], dtype=np.float32)[:, None]
    S0 = oracle.similarity(x)
    assert oracle.median_offdiag(S0) == g["preference"]
    S = S0.copy()
    np.fill_diagonal(S, g["preference"])
    assert np.array_equal(S, np.asarray(g["S"], dtype=np.float64))
    for t, key in ((1, "iter1"), (2, "iter2")):
        r = oracle.ap(S, g["lambda"], t, 0)
        assert np.array_equal(r.R, np.asarray(g[key]["R"])), key
        assert np.array_equal(r.A, np.asarray(g[key]["A"])), key
        assert r.dec.tolist() == g[key]["decisions"]
        assert r.exemplars.tolist() == g[key]["exemplars"]
    c = g["converged"]
    r = oracle.ap(S, g["lambda"], 200, c["conv_iter"])
    assert r.converged and r.iterations == c["stop_iteration"]
    assert r.idx.tolist() == c["idx"]
    assert (r.netsim, r.dpsim, r.expref) == (c["netsim"], c["dpsim"], c["expref"])
    best, bestE = brute.optimum(S)
    assert best == c["brute_force_optimum"] and bestE == (1, 3)
    for key, val in c["other_sets_netsim"].items():
        assert brute.netsim(S, [int(v) for v in key.split(",")]) == val


def test_four_point_literal(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "four_points.json")))
    S = np.asarray(g["S"], dtype=np.float64)
    for t, key in ((1, "iter1"), (2, "iter2")):
        R, A, dec = literal.iterate(S.tolist(), g["lambda"], t)
        assert np.array_equal(np.asarray(R), np.asarray(g[key]["R"]))
        assert np.array_equal(np.asarray(A), np.asarray(g[key]["A"]))
        assert dec == g[key]["decisions"]


# ---------------------------------------------------------------------------
# Literal transcription (independent reading of Eqs. (2)-(4))
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(40))
def test_matches_literal_transcription(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 11))
    lam = float(rng.choice([0.5, 0.7, 0.9]))
    n_iter = int(rng.integers(1, 25))
    S = _rand_S(n, seed, asym=True)
    A0 = -np.abs(rng.normal(size=(n, n))) * (seed % 2)
    np.fill_diagonal(A0, np.abs(rng.normal(size=n)) * (seed % 2))
    R0 = rng.normal(size=(n, n)) * (seed % 3 == 0)
    r = oracle.ap(S, lam, n_iter, 0, A0=A0, R0=R0)
    Rl, Al, decl = literal.iterate(S.tolist(), lam, n_iter, A=A0.tolist(), R=R0.tolist())
    rng_S = S.max() - S.min()
    assert np.max(np.abs(r.R - np.asarray(Rl))) <= 1e-12 * rng_S
    assert np.max(np.abs(r.A - np.asarray(Al))) <= 1e-12 * rng_S
    E = np.asarray(Al) + np.asarray(Rl)
    srt = np.sort(E, axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 1e-9 * rng_S
    assert np.array_equal(r.dec[clear], np.asarray(decl)[clear])


def test_first_iteration_closed_form():
    """From A_0 = R_0 = 0 the first responsibilities are
    (1-lambda) * (s(i,k) - max_{k' != k} s(i,k')) and pin the damping side."""
    S = _rand_S(9, 123, asym=True)
    lam = 0.9
    r = oracle.ap(S, lam, 1, 0)
    n = S.shape[0]
    expect = np.empty_like(S)
    for i in range(n):
        for k in range(n):
            expect[i, k] = (1 - lam) * (S[i, k] - np.delete(S[i], k).max())
    assert np.allclose(r.R, expect, rtol=0, atol=1e-13)
    # availabilities after one step: columns of positive responsibilities
    pos = np.maximum(expect, 0)
    np.fill_diagonal(pos, 0)
    col = pos.sum(axis=0)
    for i in range(n):
        for k in range(n):
            if i == k:
                upd = col[k]
            else:
                upd = min(0.0, expect[k, k] + col[k] - pos[i, k])
            assert abs(r.A[i, k] - (1 - lam) * upd) < 1e-13


# ---------------------------------------------------------------------------
# Brute force over exemplar sets
# ---------------------------------------------------------------------------
def _separated_case(seed) -> bool:
    """On well-separated clusters AP reaches the optimum of the energy.
    Returns True when the exact exemplar set was compared (pinned)."""
    rng = np.random.default_rng(1000 + seed)
    k = int(rng.integers(2, 4))
    n = int(rng.integers(3 * k, 11))
    centres = rng.uniform(0, 40, size=(k, 2))
    lab = np.concatenate([np.repeat(np.arange(k), 3), rng.integers(0, k, size=n - 3 * k)])
    x = (centres[lab] + rng.normal(0, 1.0, size=(n, 2))).astype(np.float32)
    prep = oracle.prepare(oracle.similarity(x), "median", seed=seed)
    r = oracle.ap(prep.S, 0.5, 1000, 30)
    best, bestE = brute.optimum(prep.S)
    assert r.netsim <= best + 1e-9
    ex = r.exemplars
    assert np.all(r.idx[ex] == ex)                     # exemplars label themselves
    lab_bf = brute.labels_for(prep.S, ex.tolist())
    assert np.array_equal(r.idx, lab_bf)               # labels = argmax over E
    assert abs(r.netsim - oracle.netsim_of_labels(prep.S, r.idx)) < 1e-9
    if r.converged:
        assert abs(r.netsim - best) <= 1e-9 * abs(best)
        # the set itself is pinned when no other set comes within 1e-6 of it
        # (a two-point cluster gives two sets whose netsim differ only by noise)
        import itertools
        gap = min(best - brute.netsim(prep.S, E) for size in range(1, x.shape[0] + 1)
                  for E in itertools.combinations(range(x.shape[0]), size) if E != bestE)
        if gap > 1e-6 * abs(best):
            assert tuple(ex.tolist()) == bestE
            return True
    return False


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_separated(seed):
    _separated_case(seed)


def test_brute_force_pins_some_sets():
    # the cases above must compare exact exemplar sets, not only netsim
    # (recomputed here, so the count does not depend on test order or workers)
    assert sum(_separated_case(seed) for seed in range(12)) >= 6


@pytest.mark.parametrize("seed", range(8))
def test_brute_force_bound_random(seed):
    """AP's net similarity never exceeds the brute-force optimum."""
    S = _rand_S(8, 77 + seed, asym=False)
    r = oracle.ap(S, 0.5, 500, 15)
    best, _ = brute.optimum(S)
    if r.n_exemplars:
        assert r.netsim <= best + 1e-9
        assert np.all(r.idx[r.exemplars] == r.exemplars)


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------
def test_two_points_high_preference():
    p, s = -1.0, -3.0
    S = np.array([[p, s], [s, p]])
    r = oracle.ap(S, 0.5, 400, 0)
    assert np.allclose(r.A, 0.0, atol=1e-12)
    assert np.allclose(r.R, [[p - s, s - p], [s - p, p - s]], atol=1e-12)
    r = oracle.ap(S, 0.5, 400, 15)
    assert r.exemplars.tolist() == [0, 1] and r.netsim == 2 * p


def test_two_points_low_preference():
    p, s = -5.0, -1.0
    S = np.array([[p, s], [s, p]])
    r = oracle.ap(S, 0.5, 400, 0)
    h = (s - p) / 2
    assert np.allclose(r.A, [[h, -h], [-h, h]], atol=1e-9)
    assert np.allclose(r.R, [[-h, h], [h, -h]], atol=1e-9)
    fin = oracle.finalize(S, r.dec)
    assert fin["n_exemplars"] == 1 and fin["netsim"] == p + s


def test_preference_above_all_similarities():
    rng = np.random.default_rng(5)
    x = rng.normal(size=(30, 3)).astype(np.float32)
    S = oracle.similarity(x)
    p = S[~np.eye(30, dtype=bool)].max() + 1.0
    np.fill_diagonal(S, p)
    r = oracle.ap(S, 0.5, 400, 15)
    assert r.n_exemplars == 30 and abs(r.netsim - 30 * p) < 1e-9


def test_single_point():
    r = oracle.ap(np.array([[-2.5]]), 0.5, 10, 15)
    assert r.iterations == 0 and r.converged
    assert r.idx.tolist() == [0] and r.netsim == -2.5 and r.expref == -2.5


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------
def test_availability_signs_every_iteration():
    S = _rand_S(40, 9, asym=True)
    A = np.zeros_like(S)
    R = np.zeros_like(S)
    off = ~np.eye(40, dtype=bool)
    for _ in range(30):
        r = oracle.ap(S, 0.5, 1, 0, A0=A, R0=R)
        A, R = r.A, r.R
        assert np.all(A[off] <= 0.0)
        assert np.all(np.diag(A) >= 0.0)


def test_power_of_two_scaling_is_exact():
    S = _rand_S(50, 10, asym=True)
    a = oracle.ap(S, 0.7, 25, 0)
    b = oracle.ap(S * 8.0, 0.7, 25, 0)
    assert np.array_equal(b.R, a.R * 8.0) and np.array_equal(b.A, a.A * 8.0)
    assert np.array_equal(a.dec, b.dec)


def test_row_shift_invariance():
    """Adding c_i to every entry of row i (diagonal included) leaves R, A and
    the decisions unchanged; catches any transposed use of S."""
    S = _rand_S(60, 11, asym=True)
    c = np.random.default_rng(3).uniform(-50, 50, size=(60, 1))
    a = oracle.ap(S, 0.9, 60, 0)
    b = oracle.ap(S + c, 0.9, 60, 0)
    scale = np.abs(S + c).max()
    assert np.max(np.abs(a.R - b.R)) < 1e-11 * scale
    assert np.max(np.abs(a.A - b.A)) < 1e-11 * scale
    assert np.array_equal(a.dec, b.dec)


def test_fixed_point_residual():
    pts = synth.gaussian_2d(n=10, k=3, seed=44, std=0.2)
    prep = oracle.prepare(oracle.similarity(pts.X), "median", seed=44)
    r = oracle.ap(prep.S, 0.9, 1000, 0)
    # one undamped step of the literal transcription from the final state
    Rn, An, _ = literal.iterate(prep.S.tolist(), 0.0, 1, A=r.A.tolist(), R=r.R.tolist())
    rng_S = prep.S.max() - prep.S.min()
    assert np.max(np.abs(np.asarray(Rn) - r.R)) < 1e-9 * rng_S
    assert np.max(np.abs(np.asarray(An) - r.A)) < 1e-9 * rng_S


# ---------------------------------------------------------------------------
# Similarity, median, noise
# ---------------------------------------------------------------------------
def test_similarity_matches_scipy():
    pts = synth.gaussian_mixture(n=300, d=17, k=5, seed=8)
    S = oracle.similarity(pts.X)
    ref = -cdist(pts.X.astype(np.float64), pts.X.astype(np.float64), "sqeuclidean")
    np.fill_diagonal(ref, 0.0)
    assert np.max(np.abs(S - ref)) <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(S, S.T)


@pytest.mark.parametrize("n", [2, 3, 7, 50])
def test_median_matches_numpy(n):
    S = _rand_S(n, n, asym=True)
    assert oracle.median_offdiag(S) == np.median(S[~np.eye(n, dtype=bool)])


def test_splitmix64_published_values(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "splitmix64.json")))
    # counter c = i*n+k+1 at (i,k)=(0,c-1) with n large: u = (z >> 11) * 2^-53
    for c, z in enumerate(g["outputs"], start=1):
        u = oracle.noise_u(g["state"], 1 << 20, 0, c - 1)
        assert u == (int(z) >> 11) * 2.0 ** -53


def test_noise_range_and_scale():
    S0 = _rand_S(30, 1, asym=False)
    prep = oracle.prepare(S0, "median", seed=99, noise_rel=1e-12)
    np.fill_diagonal(S0, oracle.median_offdiag(S0))
    d = prep.S - S0
    assert prep.noise_scale == pytest.approx(1e-12 * (S0.max() - S0.min()))
    assert np.all(d >= -1e-13 * np.abs(S0).max()) and np.all(d <= prep.noise_scale * 1.01 + 1e-13 * np.abs(S0).max())


# ---------------------------------------------------------------------------
# Algorithms 2 and 3 special cases
# ---------------------------------------------------------------------------
def test_pap_with_singleton_parts_is_cold_ap():
    S = _rand_S(25, 4, asym=True)
    cold = oracle.ap(S, 0.5, 200, 15)
    p = oracle.pap(S, 25, lam=0.5, max_iter=200, conv_iter=15)
    assert np.array_equal(p.A_prime, np.zeros_like(S))
    assert np.array_equal(p.full.R, cold.R) and np.array_equal(p.full.A, cold.A)
    assert p.full.iterations == cold.iterations


def test_pap_even_offsets():
    assert oracle.even_offsets(10, 3).tolist() == [0, 3, 6, 10]
    assert oracle.even_offsets(9, 4).tolist() == [0, 2, 4, 6, 9]


def test_pap_blocks_are_sub_ap():
    S = _rand_S(30, 6, asym=True)
    perm = np.random.default_rng(1).permutation(30)
    off = np.array([0, 7, 19, 30])
    p = oracle.pap(S, 3, perm, off, lam=0.5, max_iter=100, conv_iter=15)
    for j in range(3):
        m = perm[off[j]:off[j + 1]]
        sub = oracle.ap(np.ascontiguousarray(S[np.ix_(m, m)]), 0.5, 100, 15)
        assert np.array_equal(p.A_prime[np.ix_(m, m)], sub.A)
    mask = np.ones((30, 30), dtype=bool)
    for j in range(3):
        m = perm[off[j]:off[j + 1]]
        mask[np.ix_(m, m)] = False
    assert np.all(p.A_prime[mask] == 0.0)


def test_lap_all_landmarks_is_ap():
    pts = synth.gaussian_2d(n=120, k=4, seed=31)
    M = np.arange(120)
    lr = oracle.lap(pts.X, M, seed=31, lam=0.5, max_iter=400)
    prep = oracle.prepare(oracle.similarity(pts.X), "median", seed=31)
    ar = oracle.ap(prep.S, 0.5, 400, 15)
    assert np.array_equal(lr.exemplars, ar.exemplars)
    assert np.array_equal(lr.idx, ar.idx)


def test_lap_assignment_is_nearest_exemplar():
    pts = synth.gaussian_mixture(n=400, d=8, k=5, seed=12, centre_std=4.0)
    M = synth.landmarks(400, 80, 12)
    lr = oracle.lap(pts.X, M, seed=12, lam=0.9, max_iter=1000)
    ex = lr.exemplars
    D = cdist(pts.X.astype(np.float64), pts.X[ex].astype(np.float64), "sqeuclidean")
    want = ex[np.argmin(D, axis=1)]
    want[ex] = ex
    assert np.array_equal(lr.idx, want)


def test_row_pieces_match_full_iteration():
    """The row-wise oracle pieces reproduce one full iteration exactly."""
    S = _rand_S(30, 21, asym=True)
    a = oracle.ap(S, 0.7, 5, 0)
    b = oracle.ap(S, 0.7, 6, 0)
    rows = np.array([0, 3, 17, 29])
    Rn = oracle.resp_rows(S, a.A, a.R, 0.7, np.arange(30))
    assert np.array_equal(Rn, b.R)
    An = oracle.avail_rows(b.R, a.A, 0.7, rows)
    assert np.array_equal(An, b.A[rows])
