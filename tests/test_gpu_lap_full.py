"""Landmark AP, Algorithm 3 Steps 1-4, on the GPU against the FP64 oracle
(oracle/lap_full.py) with the same landmarks, m0 and seeds.  The GPU builds
each AP's similarity on matrix cores; the oracle builds its own in FP64.
Compared: the top level's counts (Step 1 centres, Step 2 assigned and
unassigned points, merged centres, Step 3's mode, recursion depth), the
final exemplars and every label, and the net similarity."""
import numpy as np
import pytest

import synth
from oracle import lap_full as LF

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0910_1650_amd as apx  # noqa: E402


def run_case(pts, L, m0, seed, sampled=False, pref="median"):
    n = pts.X.shape[0]
    M = None if sampled else synth.landmarks(n, L, seed)
    print(f"lap_full n={n} d={pts.X.shape[1]} L={L} m0={m0}", flush=True)
    X = torch.from_numpy(pts.X).cuda()
    idx, res, ex, st = apx.lap_full_solve(X, L, m0=m0, landmarks=M, seed=seed, damping=0.9, pref=pref)
    ref = LF.lap_full(pts.X, M, L, seed=seed, lam=0.9, m0=m0, pref=pref)
    top = {s.level: s for s in ref.levels}[0]
    print(f"  gpu {st}; oracle top {top}, levels {len(ref.levels)}", flush=True)
    assert st["step1_centres"] == top.step1_centres
    assert st["assigned"] == top.assigned and st["unassigned"] == top.unassigned
    assert st["merged_centres"] == top.merged
    assert st["step3_mode"] == {"none": 0, "ap": 1, "lap": 2}[top.step3]
    assert st["levels"] == max(s.level for s in ref.levels) + 1
    assert np.array_equal(ex, ref.exemplars)
    assert np.array_equal(idx.cpu().numpy(), ref.idx)
    assert abs(res.dpsim - ref.dpsim) <= 1e-9 * abs(ref.dpsim)
    assert abs(res.netsim - ref.netsim) <= 1e-6 * abs(ref.netsim)
    return st


def test_lap_full_step3_ap():
    st = run_case(synth.gaussian_2d(n=12000, k=10, seed=4201), 600, 2000, 4201)
    assert st["step3_mode"] == 1


def test_lap_full_recursion():
    st = run_case(synth.gaussian_2d(n=12000, k=10, seed=4201), 600, 100, 4201)
    assert st["step3_mode"] == 2 and st["levels"] >= 2


def test_lap_full_high_dimensional_sampled_landmarks():
    pts = synth.gaussian_mixture(n=20000, d=32, k=20, seed=4203, centre_std=1.0, std=1.0, clip=3.0)
    run_case(pts, 1000, 1500, 4203, sampled=True)


def test_lap_full_scalar_preference():
    run_case(synth.gaussian_2d(n=5000, k=6, seed=4205), 400, 500, 4205, pref=-30.0)


def test_lap_full_rejects():
    X = torch.from_numpy(synth.gaussian_2d(n=200, k=3, seed=1).X).cuda()
    with pytest.raises(apx.ApxError):
        apx.lap_full_solve(X, 20, m0=1)
    Xb = X.clone()
    Xb[7, 0] = float("nan")
    with pytest.raises(apx.ApxError):
        apx.lap_full_solve(Xb, 20, m0=50)
    with pytest.raises(apx.ApxError):
        apx.lap_solve(Xb, 20)
