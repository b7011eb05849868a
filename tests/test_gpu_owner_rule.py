"""Implicit availabilities with row lists that the implicit-R-only pass
could not hold: the responsibility lists of the implicit-A pass have no
per-thread limit (listed columns are handled by the lanes holding the list
entries), so a row whose ever-argmax columns k (Eq. (2)'s maximiser) share
one owner thread, (k / 4) mod 1024 at N > 4096, keeps running implicitly.

Twelve points of one cluster sit at the columns {4m..4m+3} + {0, 4096,
8192} (one owner thread per cluster at N = 12288), so every row's argmax
moves between columns of one owner.  After 60 fixed iterations every message
equals the oracle's (Algorithm 1, Eqs. (2)-(4), damping 0.9) within 1e-4 of
the range of S, and no iteration left the implicit forms.  (The clusters are
spread enough for the case to be well conditioned: one-ulp changes of S move
the oracle's messages by ~1e-5 of the range after 60 iterations, where
near-duplicate points moved them by ~3e-3.)
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0910_1650_amd as apx  # noqa: E402

N, D, ITERS, TOL = 12288, 8, 60, 1e-4


def owner_clusters(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-5.0, 5.0, size=(1024, D))
    X = np.empty((N, D))
    for m in range(1024):
        idx = np.array([4 * m + e + 4096 * j for j in range(3) for e in range(4)])
        X[idx] = centres[m] + rng.normal(0.0, 1.0, size=(12, D))
    return X.astype(np.float32)


def test_owner_rule_lists_stay_implicit():
    X = owner_clusters(4242)
    print(f"owner-rule case n={N}: oracle similarity", flush=True)
    S32 = oracle.prepare(oracle.similarity(X), "median", seed=4242).S.astype(np.float32)
    S64 = S32.astype(np.float64)
    rng = S64.max() - S64.min()
    Sd = apx.to_matrix(torch.from_numpy(S32))
    R, A = apx.empty_matrix(N), apx.empty_matrix(N)
    print(f"owner-rule case n={N}: {ITERS} fixed iterations on the GPU", flush=True)
    idx, res = apx.ap_solve(Sd, R, A, damping=0.9, max_iter=ITERS, conv_iter=0)
    imp, exp, ia = apx.apx_last_solve_info()
    why = apx.apx_last_fallback()
    assert res.iterations == ITERS
    assert (imp, exp, ia) == (ITERS, 0, ITERS)
    assert why & (apx.APX_FALLBACK_R_LIST | apx.APX_FALLBACK_A_LIST | apx.APX_FALLBACK_R_OWNER) == 0
    assert why & apx.APX_NOTE_R_OWNER            # the case does break the owner rule
    del Sd
    print(f"owner-rule case n={N}: oracle", flush=True)
    ref = oracle.ap(S64, 0.9, ITERS, 0)
    dR = np.abs(R.cpu().numpy() - ref.R).max()
    dA = np.abs(A.cpu().numpy() - ref.A).max()
    print(f"  max|dR| = {dR / rng:.3e} range, max|dA| = {dA / rng:.3e} range", flush=True)
    assert dR <= TOL * rng and dA <= TOL * rng
