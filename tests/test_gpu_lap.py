"""Landmark AP (Algorithm 3, Steps 1-2) on the GPU against the FP64 oracle.

The GPU builds the landmark similarity on matrix cores; the oracle builds
its own in FP64 from the same points.  Exemplar sets and every label must
match (the GPU assignment is certified against FP32 error and rechecked in
FP64), iteration counts of the landmark AP must match, and the net
similarity must agree to rounding."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0910_1650_amd as apx  # noqa: E402


def run_case(n, d, k, L, seed, lam=0.9):
    pts = synth.gaussian_mixture(n=n, d=d, k=k, seed=seed, centre_std=1.0, std=1.0, clip=3.0)
    M = synth.landmarks(n, L, seed)
    print(f"lap n={n} d={d} L={L}", flush=True)
    X = torch.from_numpy(pts.X).cuda()
    idx, res, ex = apx.lap_solve(X, L, landmarks=M, seed=seed, damping=lam, max_iter=2000, conv_iter=15)
    ref = oracle.lap(pts.X, M, seed=seed, lam=lam, max_iter=2000, conv_iter=15)
    assert ref.landmark.converged and res.converged
    assert res.iterations == ref.landmark.iterations
    assert np.array_equal(ex, ref.exemplars)
    assert np.array_equal(idx.cpu().numpy(), ref.idx)
    assert abs(res.dpsim - ref.dpsim) <= 1e-9 * abs(ref.dpsim)
    assert abs(res.netsim - ref.netsim) <= 1e-6 * abs(ref.netsim)


def test_lap_moderate():
    run_case(20000, 32, 20, 1000, 4101)


def test_lap_image_features_full_size():
    """200000 points in 128-D, 10000 landmarks: the n x n matrix (160 GB) is
    never formed."""
    run_case(200000, 128, 20, 10000, 4001)


def test_lap_sampled_landmarks_valid():
    n = 5000
    pts = synth.gaussian_2d(n=n, k=6, seed=5)
    X = torch.from_numpy(pts.X).cuda()
    idx, res, ex = apx.lap_solve(X, 400, landmarks=None, seed=123, damping=0.9)
    lab = idx.cpu().numpy()
    assert res.n_exemplars == ex.size > 0
    assert np.all(np.isin(lab, ex))
    assert np.all(lab[ex] == ex)
    # every point's label is a nearest exemplar (FP64 check on a sample)
    for i in np.random.default_rng(1).choice(n, 200, replace=False):
        dd = ((pts.X[ex].astype(np.float64) - pts.X[i].astype(np.float64)) ** 2).sum(1)
        if lab[i] != i:
            assert dd[np.searchsorted(ex, lab[i])] == dd.min()


def test_lap_rejects_bad_landmarks():
    X = torch.from_numpy(synth.gaussian_2d(n=100, k=3, seed=1).X).cuda()
    with pytest.raises(ValueError):
        apx.lap_solve(X, 10, landmarks=np.arange(9))
    with pytest.raises(apx.ApxError):
        apx.lap_solve(X, 3, landmarks=np.array([1, 1, 2]))
