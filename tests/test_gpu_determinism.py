"""Run-to-run determinism of the iteration kernels in every launch shape.

The row pass keeps no floating-point atomics on the result path, so repeated
runs from the same state must agree bit for bit.  Sizes cover the 256- and
1024-thread row passes with 1 to 5 column chunks per thread and both the
LDS-resident and register variants (n = 24000 exceeds the LDS budget)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0910_1650_amd as apx  # noqa: E402


@pytest.mark.parametrize("n", [1000, 3000, 4097, 9000, 14000, 20000, 24000])
def test_one_iteration_repeats_bit_identical(n):
    print(f"determinism n={n}", flush=True)
    pts = synth.gaussian_mixture(n=n, d=32, k=40, seed=5)
    X = torch.from_numpy(pts.X).cuda()
    S, _ = apx.ap_similarity(X, pref="median", noise_seed=5, noise_rel=1e-12)
    R0, A0 = apx.empty_matrix(n, fill=0.0), apx.empty_matrix(n, fill=0.0)
    apx.ap_iterate(S, R0, A0, 0.9, 5)
    outs = []
    for _ in range(3):
        R, A = apx.empty_matrix(n), apx.empty_matrix(n)
        R.copy_(R0)
        A.copy_(A0)
        apx.ap_iterate(S, R, A, 0.9, 2)
        outs.append((R, A))
    torch.cuda.synchronize()
    for R, A in outs[1:]:
        assert torch.equal(R, outs[0][0]) and torch.equal(A, outs[0][1])


def test_solve_repeats_bit_identical():
    n = 20000
    print(f"solve determinism n={n}", flush=True)
    pts = synth.gaussian_mixture(n=n, d=64, k=50, seed=2001)
    X = torch.from_numpy(pts.X).cuda()
    S, _ = apx.ap_similarity(X, pref="median", noise_seed=2001, noise_rel=1e-12)
    res = []
    for _ in range(3):
        R, A = apx.empty_matrix(n), apx.empty_matrix(n)
        idx, r = apx.ap_solve(S, R, A, 0.9, 300, 0)
        res.append((R, A, idx, r.iterations))
    for R, A, idx, it in res[1:]:
        assert it == res[0][3]
        assert torch.equal(idx, res[0][2]) and torch.equal(R, res[0][0]) and torch.equal(A, res[0][1])


def test_largest_lds_row_pass_solve_repeats_bit_identical():
    """The largest N whose implicit-A pass keeps its column partials in LDS
    (31844: the next row prefetched across the per-row barrier with eight
    float4 chunks per thread) and the global-partials form just above it
    (31848): three solves of 40 iterations each agree bit for bit."""
    for n in (31844, 31848):
        print(f"solve determinism n={n}", flush=True)
        pts = synth.gaussian_mixture(n=n, d=32, k=40, seed=7)
        X = torch.from_numpy(pts.X).cuda()
        S, _ = apx.ap_similarity(X, pref="median", noise_seed=7, noise_rel=1e-12)
        res = []
        for _ in range(3):
            R, A = apx.empty_matrix(n), apx.empty_matrix(n)
            idx, r = apx.ap_solve(S, R, A, 0.9, 40, 0)
            res.append((R, A, idx, apx.apx_last_solve_info()))
        assert res[0][3] == (40, 0, 40)
        for R, A, idx, info in res[1:]:
            assert info == res[0][3]
            assert torch.equal(idx, res[0][2]) and torch.equal(R, res[0][0]) and torch.equal(A, res[0][1])
        del S, X, res
        torch.cuda.empty_cache()
