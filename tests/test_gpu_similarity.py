"""GPU similarity build (ap_similarity) against the FP64 oracle and exact
order statistics."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0910_1650_amd as apx  # noqa: E402

EPS32 = 2.0 ** -24


def run(X, pref="median", seed=0, noise=0.0):
    Xd = torch.from_numpy(X).cuda()
    S, p = apx.ap_similarity(Xd, pref=pref, noise_seed=seed, noise_rel=noise)
    torch.cuda.synchronize()
    return S.cpu().numpy().astype(np.float64), p


@pytest.mark.parametrize("n,d", [(2, 1), (3, 2), (129, 3), (1000, 2), (777, 64), (300, 100), (513, 128)])
def test_similarity_matches_oracle(n, d):
    print(f"similarity n={n} d={d}", flush=True)
    pts = synth.gaussian_mixture(n=n, d=d, k=5, seed=n + d)
    S, p = run(pts.X, pref=0.0)
    ref = oracle.similarity(pts.X)
    nrm = (pts.X.astype(np.float64) ** 2).sum(1)
    bound = 4 * (d + 4) * EPS32 * (nrm[:, None] + nrm[None, :]) + 1e-30
    off = ~np.eye(n, dtype=bool)
    assert np.all(np.abs(S - ref)[off] <= bound[off])
    assert np.array_equal(S, S.T)                        # exactly symmetric
    assert np.all(np.diag(S) == 0.0) and p == 0.0


@pytest.mark.parametrize("n", [2, 3, 4, 5, 100, 1001, 2048])
def test_median_is_exact(n):
    pts = synth.gaussian_2d(n=n, k=3, seed=n)
    S, p = run(pts.X, pref="median")
    off = ~np.eye(n, dtype=bool)
    assert p == np.median(S[off])
    assert np.all(np.diag(S) == np.float32(p))


@pytest.mark.parametrize("n", [2050, 9001])
def test_median_is_exact_with_noise_on_long_rows(n):
    # The first digit is counted by the GEMM, the second by a row walk with
    # eight 16-byte loads per thread in flight (8192 entries a step: n = 9001
    # takes a full step and a ragged one), the third by the noise pass (two
    # loads, 2048 entries a step); the median is of the entries before the
    # noise, whichever entries the noise then moves.
    print(f"median with noise n={n}", flush=True)
    pts = synth.gaussian_mixture(n=n, d=16, k=12, seed=n)
    S0, p0 = run(pts.X, pref="median")
    off = ~np.eye(n, dtype=bool)
    want = np.median(S0[off])
    S1, p1 = run(pts.X, pref="median", seed=n, noise=1e-6)
    assert p0 == want and p1 == want
    moved = (S1 != S0) & off
    assert moved.any()                                   # the noise changed entries


def test_median_with_many_ties():
    # integer grid: many exactly equal distances
    g = np.array([[i % 7, i // 7] for i in range(70)], dtype=np.float32)
    S, p = run(g, pref="median")
    off = ~np.eye(70, dtype=bool)
    assert p == np.median(S[off])


def test_preference_vector_and_scalar():
    pts = synth.gaussian_2d(n=300, k=4, seed=3)
    pv = torch.linspace(-5, -1, 300, device="cuda")
    S, _ = run(pts.X, pref=pv)
    assert np.array_equal(np.diag(S), pv.cpu().numpy().astype(np.float64))
    S, p = run(pts.X, pref=-2.5)
    assert np.all(np.diag(S) == -2.5) and p == -2.5


def test_noise_matches_counter_definition():
    n, seed, rel = 400, 77, 1e-6          # a large rel makes every entry move
    pts = synth.gaussian_2d(n=n, k=5, seed=seed)
    S0, p = run(pts.X, pref="median")
    S1, _ = run(pts.X, pref="median", seed=seed, noise=rel)
    scale = rel * (S0.max() - S0.min())
    rng = np.random.default_rng(0)
    for i, k in rng.integers(0, n, size=(500, 2)):
        # the added noise is scale * u(seed, i, k) up to the final FP32 rounding
        added = float(np.float32(S1[i, k])) - float(np.float32(S0[i, k]))
        want = scale * oracle.noise_u(seed, n, int(i), int(k))
        half_ulp = float(np.spacing(np.float32(abs(S1[i, k])))) / 2
        assert abs(added - want) <= half_ulp + 1e-12 * scale, (i, k)


def test_c1_preference_close_to_oracle():
    pts = synth.gaussian_2d(n=1000, k=10, seed=1001)
    S, p = run(pts.X, pref="median", seed=1001, noise=1e-12)
    prep = oracle.prepare(oracle.similarity(pts.X), "median", seed=1001)
    rng = prep.S.max() - prep.S.min()
    assert abs(p - prep.pref) <= 1e-6 * rng
    assert np.max(np.abs(S - prep.S)) <= 1e-5 * rng
