"""Implicit R and A on rows longer than the LDS partials allow (Algorithm 1,
Eqs. (2)-(4), damping 0.9).

Above about 32k points the column partials of max(0, R_{t+1}) live in the
workgroup's global partial row instead of LDS; the same threads add to them
in the same order, so the two forms give bit-identical messages.  At
N = 28000 (seven float4 chunks per thread, where both forms fit) the global
form is forced and compared with the LDS form bit for bit, and both with
the oracle after 40 fixed iterations within 1e-4 of the range of S.
"""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0910_1650_amd as apx  # noqa: E402

N, ITERS, TOL, SEED = 28000, 40, 1e-4, 3021


@pytest.fixture(scope="module")
def S32():
    pts = synth.subspaces(n=N, d=100, n_sub=20, dim=5, seed=SEED)
    print(f"long rows n={N}: oracle similarity", flush=True)
    return oracle.prepare(oracle.similarity(pts.X), "median", seed=SEED).S.astype(np.float32)


def _solve(S32, global_partials: bool):
    os.environ["APX_IMPLICIT_A_GP"] = "1" if global_partials else "0"
    try:
        Sd = apx.to_matrix(torch.from_numpy(S32))
        R, A = apx.empty_matrix(N), apx.empty_matrix(N)
        idx, res = apx.ap_solve(Sd, R, A, damping=0.9, max_iter=ITERS, conv_iter=0)
        info = apx.apx_last_solve_info()
        return R.cpu().numpy(), A.cpu().numpy(), idx.cpu().numpy(), res, info
    finally:
        os.environ.pop("APX_IMPLICIT_A_GP", None)


def test_global_partials_match_lds_and_oracle(S32):
    print(f"long rows n={N}: {ITERS} iterations, LDS partials", flush=True)
    R0, A0, i0, r0, info0 = _solve(S32, False)
    print(f"long rows n={N}: {ITERS} iterations, global partials", flush=True)
    R1, A1, i1, r1, info1 = _solve(S32, True)
    assert info0 == info1 == (ITERS, 0, ITERS)
    assert np.array_equal(R0, R1) and np.array_equal(A0, A1) and np.array_equal(i0, i1)
    assert r0.netsim == r1.netsim
    S64 = S32.astype(np.float64)
    rng = S64.max() - S64.min()
    print(f"long rows n={N}: oracle", flush=True)
    ref = oracle.ap(S64, 0.9, ITERS, 0)
    dR = np.abs(R1 - ref.R).max()
    dA = np.abs(A1 - ref.A).max()
    print(f"  max|dR| = {dR / rng:.3e} range, max|dA| = {dA / rng:.3e} range", flush=True)
    assert dR <= TOL * rng and dA <= TOL * rng
