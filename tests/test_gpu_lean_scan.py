"""The lean implicit-A scan changes no bit (Algorithm 1, Eqs. (2)-(4) and
the exemplar decision argmax_k a(i,k) + r(i,k), lowest index on ties).

It leaves the ordinary columns out of the decision where they cannot change
it and tests positivity of al*s - beta against a per-row threshold.  Switched
off, positivity is fl(al*s) > beta and every row is decided over its ordinary
columns after the reduction.  Solves to the stop rule both ways give
identical R, A, labels, iteration counts and net similarity: cold starts in
the LDS form (N = 6000, 20000) and with global partials (N = 33000), and a
column-structured warm start whose column values are partly positive, where
every row that the listed columns do not decide is tested again."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0910_1650_amd as apx  # noqa: E402


def _both(S, n, warm=apx.APX_COLD, A0=None):
    out = []
    try:
        for on in (True, False):
            apx.apx_set_lean_scan(on)
            apx.apx_profile(True)
            apx.apx_profile_read()
            R = apx.empty_matrix(n)
            A = apx.empty_matrix(n)
            if A0 is not None:
                A.copy_(A0)
            idx, res = apx.ap_solve(S, R, A, 0.9, 2000, 15, warm=warm)
            launches, ms = apx.apx_profile_read()
            apx.apx_profile(False)
            info = apx.apx_last_solve_info()
            resc = apx.apx_last_lean_rescans()
            print(f"  lean {on}: {res.iterations} iterations {info}, rows decided again {resc}, "
                  f"{ms / max(launches, 1):.4f} ms per pass", flush=True)
            out.append((R, A, idx, res, info, resc))
    finally:
        apx.apx_set_lean_scan(True)
        apx.apx_profile(False)
    return out


@pytest.mark.parametrize("n,d,k,seed", [(6000, 16, 20, 6101), (20000, 64, 50, 2001), (33000, 32, 40, 6103)])
def test_lean_scan_is_bit_identical(n, d, k, seed):
    print(f"lean scan n={n}", flush=True)
    pts = synth.gaussian_mixture(n=n, d=d, k=k, seed=seed)
    X = torch.from_numpy(pts.X).cuda()
    S, _ = apx.ap_similarity(X, pref="median", noise_seed=seed, noise_rel=1e-12)
    (R1, A1, i1, r1, f1, c1), (R0, A0, i0, r0, f0, c0) = _both(S, n)
    assert f1 == f0 and f1[2] == r1.iterations                 # implicit A throughout
    assert c0 >= c1                                            # off: every row is decided again
    assert r1.iterations == r0.iterations and r1.netsim == r0.netsim
    assert torch.equal(i1, i0) and torch.equal(R1, R0) and torch.equal(A1, A0)


def test_lean_scan_positive_column_values():
    """A column-structured A_0 with positive column values voids the sign
    argument: rows that no listed column decides are scanned again."""
    n, seed = 6000, 6107
    print(f"lean scan, positive column values, n={n}", flush=True)
    pts = synth.gaussian_mixture(n=n, d=16, k=20, seed=seed)
    X = torch.from_numpy(pts.X).cuda()
    S, _ = apx.ap_similarity(X, pref="median", noise_seed=seed, noise_rel=1e-12)
    rng = np.random.default_rng(seed)
    col = rng.uniform(-0.5, 0.05, n).astype(np.float32)       # about 1 in 11 positive
    dia = rng.uniform(-0.5, 0.5, n).astype(np.float32)
    A0 = np.repeat(col[None, :], n, axis=0)
    np.fill_diagonal(A0, dia)
    A0 = apx.to_matrix(torch.from_numpy(A0).cuda())
    (R1, A1, i1, r1, f1, c1), (R0, A0_, i0, r0, f0, c0) = _both(S, n, apx.APX_WARM_COLUMNS, A0)
    assert f1 == f0 and f1[2] >= 1                             # implicit A ran
    assert c1 > 0 and c0 >= c1
    assert r1.iterations == r0.iterations and r1.netsim == r0.netsim
    assert torch.equal(i1, i0) and torch.equal(R1, R0) and torch.equal(A1, A0_)
