"""Partition AP (Algorithm 2) at a size whose code paths are the benchmark's:
N = 24000 points on a union of subspaces (the PAP workload's family), six
random uneven parts of 3000-7000 points, so the batched sub-problem pass
runs with several chunks per thread (J = 3..7) and Step 4 runs the long-row
implicit-R pass (rows too long for S to sit in LDS next to the partials).

Both sides use the oracle's S rounded once to FP32 and the same partition:
* 100 fixed iterations in every sub-problem and in Step 4: every message of
  Step 4 against the oracle within 1e-4 of the range;
* to the stop rules: every part's iteration count and exemplar count, then
  Step 4's stop iteration, exemplar set and labels, and the net similarity.
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

TOL = 1e-4
N, PARTS, SEED = 24000, 6, 3011


@pytest.fixture(scope="module")
def case():
    pts = synth.subspaces(n=N, d=100, n_sub=20, dim=5, seed=SEED)
    print(f"pap n={N}: oracle similarity", flush=True)
    S32 = oracle.prepare(oracle.similarity(pts.X), "median", seed=SEED).S.astype(np.float32)
    perm, offsets = synth.random_partition(N, parts=PARTS, lo=3000, hi=7000, seed=SEED)
    sizes = np.diff(offsets)
    assert sizes.min() >= 2000 and sizes.max() > 2 * 1024   # several chunks per thread
    return S32, perm, offsets


def test_pap_messages_after_100(case):
    S32, perm, offsets = case
    S64 = S32.astype(np.float64)
    rng = S64.max() - S64.min()
    print(f"pap n={N}: 100 fixed iterations, sizes {np.diff(offsets).tolist()}", flush=True)
    R, A = apx.empty_matrix(N), apx.empty_matrix(N)
    Sd = apx.to_matrix(torch.from_numpy(S32))
    idx, res, sub = apx.pap_solve(Sd, R, A, PARTS, perm, offsets, damping=0.9, max_iter=100, conv_iter=0)
    imp, exp, ia = apx.apx_last_solve_info()
    assert res.iterations == 100 and imp == 100 and exp == 0
    assert all(s.iterations == 100 for s in sub)
    del Sd
    ref = oracle.pap(S64, PARTS, perm, offsets, lam=0.9, max_iter=100, conv_iter=0)
    dR = np.abs(R.cpu().numpy() - ref.full.R).max()
    dA = np.abs(A.cpu().numpy() - ref.full.A).max()
    print(f"  max|dR| = {dR / rng:.3e} range, max|dA| = {dA / rng:.3e} range", flush=True)
    assert dR <= TOL * rng and dA <= TOL * rng


def test_pap_converged_exemplars(case):
    S32, perm, offsets = case
    S64 = S32.astype(np.float64)
    rng = S64.max() - S64.min()
    print(f"pap n={N}: to the stop rules", flush=True)
    R, A = apx.empty_matrix(N), apx.empty_matrix(N)
    Sd = apx.to_matrix(torch.from_numpy(S32))
    idx, res, sub = apx.pap_solve(Sd, R, A, PARTS, perm, offsets, damping=0.9, max_iter=2000, conv_iter=15)
    del Sd, R, A
    ref = oracle.pap(S64, PARTS, perm, offsets, lam=0.9, max_iter=2000, conv_iter=15)
    for j, (sr, so) in enumerate(zip(sub, ref.subs)):
        assert sr.iterations == so.iterations and sr.n_exemplars == so.n_exemplars, j
    assert res.converged and ref.full.converged
    assert res.iterations == ref.full.iterations
    assert np.array_equal(idx.cpu().numpy(), ref.full.idx)
    assert abs(res.netsim - ref.full.netsim) <= N * 1e-6 * rng
