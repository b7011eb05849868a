"""ap_solve with implicit responsibilities against explicit R and the oracle.

With R_0 = 0 the damped Eq. (2) unrolls to R_t = (1 - lambda^t) S - beta_t 1^T
+ gamma_t with gamma_t sparse per row; the library keeps only beta and the
list.  Same arithmetic, other rounding order: messages agree with explicit R
and with the FP64 oracle within the message tolerance, exemplar sets and
labels are identical.  A tiny list capacity forces the overflow hand-over
(R made explicit mid-run), which must give the same exemplars.
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


def say(msg):
    print(msg, flush=True)


def host(M):
    return M.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(autouse=True)
def restore():
    yield
    apx.apx_set_implicit(16, 8192)
    apx.apx_set_implicit_a(1024, 4096)
    apx.apx_set_graphs(True)


def mixture(n, seed, d=8, k=12):
    pts = synth.gaussian_mixture(n=n, d=d, k=k, seed=seed)
    S = oracle.prepare(oracle.similarity(pts.X), "median", seed=seed).S
    return S.astype(np.float32).astype(np.float64)


def solve(Sd, cap, lam=0.9, max_iter=2000, conv_iter=15, warm=apx.APX_COLD, A0=None):
    apx.apx_set_implicit(cap, 0)     # every size: these tests use small problems
    apx.apx_set_implicit_a(0, 0)     # explicit A (implicit A: test_gpu_implicit_a.py)
    n = Sd.shape[0]
    R, A = apx.empty_matrix(n), apx.empty_matrix(n)
    if A0 is not None:
        A.copy_(A0)
    idx, res = apx.ap_solve(Sd, R, A, lam, max_iter, conv_iter, warm=warm)
    torch.cuda.synchronize()
    return R, A, idx, res


@pytest.mark.parametrize("n", [300, 1000, 4097, 6000])
def test_implicit_matches_explicit_and_oracle(n):
    say(f"implicit vs explicit n={n}")
    S = mixture(n, 1300 + n)
    Sd = apx.to_matrix(torch.from_numpy(S.astype(np.float32)))
    Ri, Ai, ii, ri = solve(Sd, 16)
    Re, Ae, ie, re = solve(Sd, 0)
    ref = oracle.ap(S, 0.9, 2000, 15)
    rng = S.max() - S.min()
    assert ri.converged and re.converged and ref.converged
    assert ri.iterations == re.iterations == ref.iterations
    assert torch.equal(ii, ie)
    assert np.array_equal(ii.cpu().numpy(), ref.idx)
    assert np.max(np.abs(host(Ri) - host(Re))) <= TOL * rng
    assert np.max(np.abs(host(Ai) - host(Ae))) <= TOL * rng
    assert abs(ri.netsim - ref.netsim) <= n * 1e-6 * rng


def test_fixed_count_messages_against_oracle():
    n = 2000
    say(f"implicit fixed count n={n}")
    S = mixture(n, 77)
    Sd = apx.to_matrix(torch.from_numpy(S.astype(np.float32)))
    R, A, _, res = solve(Sd, 16, max_iter=37, conv_iter=0)
    assert res.iterations == 37
    ref = oracle.ap(S, 0.9, 37, 0)
    rng = S.max() - S.min()
    assert np.max(np.abs(host(R) - ref.R)) <= TOL * rng
    assert np.max(np.abs(host(A) - ref.A)) <= TOL * rng


@pytest.mark.parametrize("cap", [1, 2])
def test_list_overflow_hands_over_to_explicit(cap):
    n = 1500
    say(f"implicit overflow with list capacity {cap}")
    S = mixture(n, 91)
    Sd = apx.to_matrix(torch.from_numpy(S.astype(np.float32)))
    R, A, idx, res = solve(Sd, cap)
    Re, Ae, ie, re = solve(Sd, 0)
    rng = S.max() - S.min()
    assert res.converged and res.iterations == re.iterations
    assert torch.equal(idx, ie)
    assert np.max(np.abs(host(R) - host(Re))) <= TOL * rng
    assert np.max(np.abs(host(A) - host(Ae))) <= TOL * rng


def test_warm_a_start_matches_explicit():
    n = 2400
    say(f"implicit warm start (PAP) n={n}")
    S = mixture(n, 55)
    Sd = apx.to_matrix(torch.from_numpy(S.astype(np.float32)))
    out = {}
    for cap in (16, 0):
        apx.apx_set_implicit(cap, 0)
        apx.apx_set_implicit_a(0, 0)
        R, A = apx.empty_matrix(n), apx.empty_matrix(n)
        idx, res, _ = apx.pap_solve(Sd, R, A, 4, damping=0.9, max_iter=2000, conv_iter=15)
        torch.cuda.synchronize()
        out[cap] = (idx.clone(), res, host(R), host(A))
    (i1, r1, R1, A1), (i0, r0, R0, A0) = out[16], out[0]
    rng = S.max() - S.min()
    assert r1.iterations == r0.iterations and torch.equal(i1, i0)
    assert np.max(np.abs(R1 - R0)) <= TOL * rng and np.max(np.abs(A1 - A0)) <= TOL * rng


def test_graph_and_repeat_bit_identical():
    n = 3000
    say(f"implicit graph vs host launches n={n}")
    S = mixture(n, 66)
    Sd = apx.to_matrix(torch.from_numpy(S.astype(np.float32)))
    apx.apx_set_graphs(False)
    ref = solve(Sd, 16)
    apx.apx_set_graphs(True)
    for _ in range(2):
        got = solve(Sd, 16)
        for a, b in zip(got[:3], ref[:3]):
            assert torch.equal(a, b)
        assert got[3].netsim == ref[3].netsim
