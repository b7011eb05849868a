"""Pins for the warm-start oracle (oracle/warm.py) against facts that do not
come from the oracle itself: textbook values (the normal CDF, bfloat16 round
to nearest even), brute-force order statistics by counting, central finite
differences, Adam's closed-form first steps, a hand-worked feature example,
the hand-worked column sums of Algorithm 1 iteration 1, and the fixed-point
form of Eqs. (3)-(4)."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import warm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# bfloat16
# --------------------------------------------------------------------------
def _bf16_by_neighbours(f: np.float32) -> float:
    """Nearest of the two bfloat16 neighbours of a finite float32, ties to the
    one whose last kept bit is 0."""
    b = int(np.array([f], dtype=np.float32).view(np.uint32)[0])
    lo = b & 0xFFFF0000
    hi = lo + 0x10000
    vals = [np.array([x], dtype=np.uint32).view(np.float32)[0] for x in (lo, hi & 0xFFFFFFFF)]
    x = Fraction(float(f))
    d0, d1 = abs(Fraction(float(vals[0])) - x), abs(Fraction(float(vals[1])) - x)
    if d0 < d1 or (d0 == d1 and (lo >> 16) % 2 == 0):
        return float(vals[0])
    return float(vals[1])


def test_bf16_round_matches_neighbour_search():
    rng = np.random.default_rng(5)
    f = rng.normal(0, 10, 4000).astype(np.float32)
    # plant exact ties: low 16 bits = 0x8000
    bits = f.view(np.uint32).copy()
    bits[:500] = (bits[:500] & 0xFFFF0000) | 0x8000
    f = bits.view(np.float32)
    got = warm.bf16_round(f)
    want = np.array([_bf16_by_neighbours(x) for x in f])
    assert np.array_equal(got, want)


def test_bf16_round_worked_values():
    cases = {
        1.0: 1.0,
        1.0 + 2**-8: 1.0,                            # tie, 1.0 is even
        1.0 + 3 * 2**-8: 1.0 + 2**-6,                # tie, 1+2^-6 is even
        -(1.0 + 2**-8 + 2**-20): -(1.0 + 2**-7),     # above the tie
        0.1: 0.10009765625,                          # 0x3DCCCCCD -> 0x3DCD
        65504.0: 65536.0,
    }
    for x, want in cases.items():
        assert warm.bf16_round(np.float32(x)) == want, x
    assert np.isnan(warm.bf16_round(np.float32("nan")))


# --------------------------------------------------------------------------
# GELU, Huber
# --------------------------------------------------------------------------
def test_gelu_textbook_values():
    # Phi(1) = 0.8413447460685429 (standard normal table), gelu(z) = z Phi(z)
    assert warm.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, abs=1e-15)
    assert warm.gelu(np.array([0.0]))[0] == 0.0
    assert warm.gelu(np.array([2.0]))[0] == pytest.approx(2 * 0.9772498680518208, abs=1e-15)
    z = np.random.default_rng(1).normal(0, 3, 200)
    # Phi(z) + Phi(-z) = 1  =>  gelu(z) - gelu(-z) = z
    assert np.allclose(warm.gelu(z) - warm.gelu(-z), z, atol=1e-14, rtol=0)


def test_gelu_grad_central_differences():
    z = np.random.default_rng(2).normal(0, 3, 200)
    h = 1e-6
    fd = (warm.gelu(z + h) - warm.gelu(z - h)) / (2 * h)
    assert np.allclose(warm.gelu_grad(z), fd, atol=1e-8, rtol=0)


def test_huber_values():
    e = np.array([0.0, 0.5, -0.5, 1.0, 2.0, -3.0])
    assert np.array_equal(warm.huber(e), [0.0, 0.125, 0.125, 0.5, 1.5, 2.5])
    assert np.array_equal(warm.huber_grad(e), [0.0, 0.5, -0.5, 1.0, 1.0, -1.0])


# --------------------------------------------------------------------------
# Network gradient
# --------------------------------------------------------------------------
def _fd_setup(seed=3, count=24):
    theta = synth.mlp_params(seed).astype(np.float64)
    X, T, w = synth.mlp_batch(count, seed + 1)
    return theta, X.astype(np.float64), T.astype(np.float64), w.astype(np.float64)


def test_backward_matches_central_differences_per_coordinate():
    theta, X, T, w = _fd_setup()
    L, g, _ = warm.backward(theta, X, T, w, bf16=False)
    assert L == pytest.approx(warm.loss(theta, X, T, w, bf16=False), rel=1e-15)
    rng = np.random.default_rng(4)
    # every bias of the last layer, then samples from each tensor
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in warm.SHAPES])
    coords = list(range(offs[5], offs[6]))
    for t in range(6):
        size = min(25, offs[t + 1] - offs[t])
        coords += list(rng.choice(np.arange(offs[t], offs[t + 1]), size=size, replace=False))
    h = 1e-5
    for c in coords:
        tp, tm = theta.copy(), theta.copy()
        tp[c] += h
        tm[c] -= h
        fd = (warm.loss(tp, X, T, w, bf16=False) - warm.loss(tm, X, T, w, bf16=False)) / (2 * h)
        assert abs(fd - g[c]) <= 1e-6 * max(1e-3, abs(g[c])) + 1e-10, c


def test_backward_matches_central_differences_directional():
    theta, X, T, w = _fd_setup(seed=7, count=40)
    _, g, _ = warm.backward(theta, X, T, w, bf16=False)
    rng = np.random.default_rng(8)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in warm.SHAPES])
    dirs = [rng.normal(size=theta.size) for _ in range(4)]
    for t in range(6):                      # one direction inside each tensor
        d = np.zeros(theta.size)
        d[offs[t]:offs[t + 1]] = rng.normal(size=offs[t + 1] - offs[t])
        dirs.append(d)
    h = 1e-6
    for d in dirs:
        d = d / np.linalg.norm(d)
        fd = (warm.loss(theta + h * d, X, T, w, bf16=False)
              - warm.loss(theta - h * d, X, T, w, bf16=False)) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * abs(g @ d) + 1e-10


def test_bf16_forward_rounds_inputs_and_stays_close():
    theta, X, T, w = _fd_setup(seed=9, count=64)
    y16, c = warm.forward(theta, X, bf16=True)
    y64, _ = warm.forward(theta, X, bf16=False)
    # inputs enter through bfloat16: a perturbation far below half an ulp of
    # every input leaves the output unchanged
    Xp = X * (1 + 2.0**-14)
    Xp[warm.bf16_round(Xp) != warm.bf16_round(X)] = X[warm.bf16_round(Xp) != warm.bf16_round(X)]
    assert np.array_equal(warm.forward(theta, Xp, bf16=True)[0], y16)
    # every stored operand is on the bfloat16 grid
    for key in ("x", "W1", "W2", "W3", "h1", "h2"):
        assert np.array_equal(warm.bf16_round(c[key]), c[key]), key
    # relative error of a few bfloat16 roundings, in the abs-sum scale
    scale = np.abs(c["h2"]) @ np.abs(c["W3"]) + 1.0
    assert np.max(np.abs(y16 - y64) / scale) < 2**-5


# --------------------------------------------------------------------------
# Adam
# --------------------------------------------------------------------------
def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(10)
    theta0 = rng.normal(size=500)
    g = rng.normal(size=500) * 10.0 ** rng.uniform(-4, 2, 500)
    m = v = np.zeros(500)
    lr, eps = 1e-3, 1e-8
    t1, m, v = warm.adam_step(theta0, m, v, g, 1, lr, eps=eps)
    # bias correction makes m_hat = g and v_hat = g^2 on the first step ...
    assert np.allclose(t1, theta0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    # ... and on every step while the gradient stays constant
    t2, m, v = warm.adam_step(t1, m, v, g, 2, lr, eps=eps)
    assert np.allclose(t2, theta0 - 2 * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)


# --------------------------------------------------------------------------
# Features
# --------------------------------------------------------------------------
def test_features_four_point_example():
    d = json.load(open(os.path.join(GOLDEN, "four_points_features.json")))
    S = np.array(d["S"], dtype=np.float64)
    F, sigma = warm.features(S)
    assert sigma == d["sigma"]
    for k, row in enumerate(d["features"]):
        want = [np.float32(float(Fraction(v))) for v in row] + [np.float32(math.log(4) / 10)]
        assert np.array_equal(F[k], np.array(want, dtype=np.float32)), k


def _count_rank(vals, r):
    """The value v with #{x < v} <= r < #{x <= v} (ascending rank r)."""
    for v in vals:
        lt = sum(1 for x in vals if x < v)
        le = sum(1 for x in vals if x <= v)
        if lt <= r < le:
            return v
    raise AssertionError


@pytest.mark.parametrize("n", [2, 3, 9, 40])
def test_features_by_counting(n):
    rng = np.random.default_rng(100 + n)
    S = rng.integers(-30, 3, size=(n, n)).astype(np.float64)   # many ties
    F, sigma = warm.features(S)
    mus = []
    for k in range(n):
        off = [S[k, j] for j in range(n) if j != k]
        mus.append(_count_rank(off, (len(off) - 1) // 2))
    s = abs(_count_rank(mus, (n - 1) // 2))
    assert sigma == (s if s > 0 else 1.0)
    for k in range(n):
        off = [S[k, j] for j in range(n) if j != k]
        m = len(off)
        desc = [_count_rank(off, m - 1 - min(j, m - 1)) for j in (0, 1, 3, 7, 15, 31)]
        top = [_count_rank(off, m - 1 - j) for j in range(min(32, m))]
        tm = math.fsum(top) / len(top)
        qs = [_count_rank(off, (q * (m - 1)) // 100) for q in (1, 10, 25, 50, 75)]
        want = [x / sigma for x in desc] + [tm / sigma] + [x / sigma for x in qs]
        want += [(S[k, k] - mus[k]) / sigma, (S[k, k] - tm) / sigma,
                 sum(1 for x in off if x > S[k, k]) / m, math.log(n) / 10]
        assert np.array_equal(F[k], np.array(want, dtype=np.float32)), k


def test_features_scale_invariant_and_permutation_equivariant():
    pts = synth.gaussian_2d(n=120, k=4, seed=11)
    S = oracle.prepare(oracle.similarity(pts.X), "median", seed=11).S
    F, sigma = warm.features(S)
    F2, sigma2 = warm.features(S * 8.0)
    assert sigma2 == 8.0 * sigma and np.array_equal(F, F2)
    perm = np.random.default_rng(12).permutation(120)
    F3, sigma3 = warm.features(S[np.ix_(perm, perm)])
    assert sigma3 == sigma and np.array_equal(F3, F[perm])


def test_features_sampled_rows_equal_full():
    pts = synth.gaussian_2d(n=90, k=3, seed=13)
    S = oracle.prepare(oracle.similarity(pts.X), "median", seed=13).S
    F, sigma = warm.features(S)
    rows = np.array([0, 5, 89, 44])
    Fr, _ = warm.features(S, rows=rows, sigma=sigma)
    assert np.array_equal(Fr, F[rows])


# --------------------------------------------------------------------------
# Targets and A_0
# --------------------------------------------------------------------------
def test_column_state_matches_hand_worked_iteration():
    d = json.load(open(os.path.join(GOLDEN, "four_points.json")))
    R1 = np.array(d["iter1"]["R"])
    t, c = warm.column_state(R1)
    assert np.array_equal(c, d["iter1"]["column_sums"])
    assert np.array_equal(t, [-4.25, 0.75, -4.25, 1.75])   # r(k,k) + c_k


def test_a0_from_exact_targets_is_the_fixed_point_availability():
    """At a fixed point of Eqs. (3)-(4), a(i,k) = min(0, t_k) wherever
    r(i,k) <= 0 and a(k,k) = c_k; A_0 built from the exact targets equals it."""
    pts = synth.gaussian_2d(n=150, k=5, seed=14)
    prep = oracle.prepare(oracle.similarity(pts.X), "median", seed=14)
    ref = oracle.ap(prep.S, 0.9, 3000, 0)
    sigma = 7.0
    Y = warm.targets(ref.R, sigma)
    A0 = warm.warm_a0(Y, sigma)
    n = 150
    rng = prep.S.max() - prep.S.min()
    off = ~np.eye(n, dtype=bool) & (ref.R <= 0)
    assert np.max(np.abs(A0[off] - ref.A[off])) <= 1e-6 * rng
    assert np.max(np.abs(np.diag(A0) - np.diag(ref.A))) <= 1e-6 * rng
    assert np.all(A0[~np.eye(n, dtype=bool)] <= 0) and np.all(np.diag(A0) >= 0)


# ---------------------------------------------------------------------------
# The straight-through gradient of the bfloat16 network, pinned against
# central differences of a surrogate written here: the forward pass with
# every bfloat16 rounding replaced by a fixed offset, the rounding error it
# makes at the expansion point.  At that point the surrogate equals the
# rounded network; its derivative treats each rounding as the identity,
# which is the gradient the backward pass defines.  A slip in which operand
# of a product the backward pass takes rounded (or unrounded) changes the
# derivative by the rounding error times the other factor, which these
# differences resolve.
# ---------------------------------------------------------------------------
def _st_surrogate(theta0, X):
    rnd = warm.bf16_round
    p0 = warm.unpack(theta0)
    off = {k: rnd(p0[k]) - p0[k] for k in ("W1", "W2", "W3")}
    x = rnd(X)
    z1_0 = x @ rnd(p0["W1"]) + p0["b1"]
    g1 = warm.gelu(z1_0)
    o1 = rnd(g1) - g1
    z2_0 = rnd(g1) @ rnd(p0["W2"]) + p0["b2"]
    g2 = warm.gelu(z2_0)
    o2 = rnd(g2) - g2

    def f(theta, T, w):
        p = warm.unpack(theta)
        z1 = x @ (p["W1"] + off["W1"]) + p["b1"]
        h1 = warm.gelu(z1) + o1
        z2 = h1 @ (p["W2"] + off["W2"]) + p["b2"]
        h2 = warm.gelu(z2) + o2
        y = h2 @ (p["W3"] + off["W3"]) + p["b3"]
        return float(np.sum(w[:, None] * warm.huber(y - T)))
    return f


def test_bf16_backward_is_the_straight_through_gradient():
    theta, X, T, w = _fd_setup(seed=11, count=32)
    # weights large enough that their rounding errors are far above the FD error
    theta = theta * 4.0
    L, g, _ = warm.backward(theta, X, T, w, bf16=True)
    f = _st_surrogate(theta, X)
    assert f(theta, T, w) == pytest.approx(warm.loss(theta, X, T, w, bf16=True), rel=1e-13)
    assert L == pytest.approx(f(theta, T, w), rel=1e-13)
    rng = np.random.default_rng(12)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in warm.SHAPES])
    dirs = [rng.normal(size=theta.size) for _ in range(3)]
    for t in range(6):
        d = np.zeros(theta.size)
        d[offs[t]:offs[t + 1]] = rng.normal(size=offs[t + 1] - offs[t])
        dirs.append(d)
    h = 1e-6
    for d in dirs:
        d = d / np.linalg.norm(d)
        fd = (f(theta + h * d, T, w) - f(theta - h * d, T, w)) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * abs(g @ d) + 1e-9


def test_bf16_backward_differs_from_the_unrounded_gradient():
    """The same check distinguishes the rounded network: the FP64 network's
    gradient misses the surrogate's differences by far more than their error."""
    theta, X, T, w = _fd_setup(seed=11, count=32)
    theta = theta * 4.0
    _, g64, _ = warm.backward(theta, X, T, w, bf16=False)
    _, g16, _ = warm.backward(theta, X, T, w, bf16=True)
    rel = np.abs(g64 - g16).max() / np.abs(g16).max()
    assert rel > 1e-4
