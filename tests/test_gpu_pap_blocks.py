"""Partition AP (Algorithm 2) with the paper's contiguous split, whose
Step 4 keeps its availabilities implicit: A' is block-diagonal, so an
element whose responsibility was never positive has a_t = acol_t(k) +
lambda^t a'(i,k) (the damped Eq. (3) unrolled from a_0 = a'), and the pass
reads a' only inside the row's block.

N = 12000 points of the C2 family in 32-D, k = 4 parts of 3000: after 60
fixed iterations (sub-problems and Step 4) every message of Step 4 equals
the oracle's within 1e-4 of the range of S, and to the stop rules the
parts' and Step 4's stop iterations, exemplar set and labels equal the
oracle's.  Step 4 runs every iteration with implicit R and A.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0910_1650_amd as apx  # noqa: E402

N, K, TOL, SEED = 12000, 4, 1e-4, 3041


@pytest.fixture(scope="module")
def S32():
    pts = synth.gaussian_mixture(n=N, d=32, k=30, seed=SEED)
    print(f"pap blocks n={N}: oracle similarity", flush=True)
    return oracle.prepare(oracle.similarity(pts.X), "median", seed=SEED).S.astype(np.float32)


def test_step4_messages_after_60(S32):
    S64 = S32.astype(np.float64)
    rng = S64.max() - S64.min()
    R, A = apx.empty_matrix(N), apx.empty_matrix(N)
    Sd = apx.to_matrix(torch.from_numpy(S32))
    print(f"pap blocks n={N}: 60 fixed iterations", flush=True)
    idx, res, sub = apx.pap_solve(Sd, R, A, K, None, None, damping=0.9, max_iter=60, conv_iter=0)
    imp, exp, ia = apx.apx_last_solve_info()
    assert res.iterations == 60 and (imp, exp, ia) == (60, 0, 60)
    del Sd
    ref = oracle.pap(S64, K, None, None, lam=0.9, max_iter=60, conv_iter=0)
    dR = np.abs(R.cpu().numpy() - ref.full.R).max()
    dA = np.abs(A.cpu().numpy() - ref.full.A).max()
    print(f"  max|dR| = {dR / rng:.3e} range, max|dA| = {dA / rng:.3e} range", flush=True)
    assert dR <= TOL * rng and dA <= TOL * rng


def test_step4_converged_exemplars(S32):
    S64 = S32.astype(np.float64)
    rng = S64.max() - S64.min()
    R, A = apx.empty_matrix(N), apx.empty_matrix(N)
    Sd = apx.to_matrix(torch.from_numpy(S32))
    print(f"pap blocks n={N}: to the stop rules", flush=True)
    idx, res, sub = apx.pap_solve(Sd, R, A, K, None, None, damping=0.9, max_iter=2000, conv_iter=15)
    imp, exp, ia = apx.apx_last_solve_info()
    print(f"  step 4: {res.iterations} iterations (implicit R {imp}, explicit {exp}, implicit A {ia})", flush=True)
    assert (imp, exp, ia) == (res.iterations, 0, res.iterations)
    del Sd, R, A
    ref = oracle.pap(S64, K, None, None, lam=0.9, max_iter=2000, conv_iter=15)
    for j, (sr, so) in enumerate(zip(sub, ref.subs)):
        assert sr.iterations == so.iterations and sr.n_exemplars == so.n_exemplars, j
    assert res.converged and ref.full.converged
    assert res.iterations == ref.full.iterations
    assert np.array_equal(idx.cpu().numpy(), ref.full.idx)
    assert abs(res.netsim - ref.full.netsim) <= N * 1e-6 * rng
