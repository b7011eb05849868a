"""ap_solve with implicit availabilities (cold start) against explicit
messages and the FP64 oracle.

With A_0 = 0, Eq. (3) with damping keeps every off-diagonal a(i,k) whose
responsibility was never positive equal to one value per column, and Eq. (4)
makes the diagonal a column vector; each row keeps the other elements in a
list.  A is the explicit update element for element, R is implicit as in
test_gpu_implicit.py: messages agree with explicit messages and with the
oracle within the message tolerance, exemplar sets and labels are identical.
Tiny list capacities force the hand-over to explicit A mid-run.
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
    os.environ.pop("APX_IMPLICIT_A_GP", None)


def mixture(n, seed, d=8, k=12):
    pts = synth.gaussian_mixture(n=n, d=d, k=k, seed=seed)
    S = oracle.prepare(oracle.similarity(pts.X), "median", seed=seed).S
    return S.astype(np.float32).astype(np.float64)


def solve(Sd, cap_r, cap_a, lam=0.9, max_iter=2000, conv_iter=15):
    apx.apx_set_implicit(cap_r, 0)     # every size: these tests use small problems
    apx.apx_set_implicit_a(cap_a, 0)
    n = Sd.shape[0]
    R, A = apx.empty_matrix(n), apx.empty_matrix(n)
    idx, res = apx.ap_solve(Sd, R, A, lam, max_iter, conv_iter)
    torch.cuda.synchronize()
    return R, A, idx, res, apx.apx_last_solve_info()


@pytest.mark.parametrize("n", [300, 1000, 4097, 6000])
def test_implicit_a_matches_explicit_and_oracle(n):
    say(f"implicit A vs explicit n={n}")
    S = mixture(n, 2300 + n)
    Sd = apx.to_matrix(torch.from_numpy(S.astype(np.float32)))
    Ri, Ai, ii, ri, info = solve(Sd, 16, 1024)
    Rr, Ar, ir, rr, _ = solve(Sd, 16, 0)       # implicit R, explicit A
    Re, Ae, ie, re, _ = solve(Sd, 0, 0)        # explicit R and A
    ref = oracle.ap(S, 0.9, 2000, 15)
    rng = S.max() - S.min()
    assert info[2] == ri.iterations, info        # A implicit for the whole run
    assert ri.converged and re.converged and ref.converged
    assert ri.iterations == rr.iterations == re.iterations == ref.iterations
    assert torch.equal(ii, ie) and torch.equal(ii, ir)
    assert np.array_equal(ii.cpu().numpy(), ref.idx)
    # same R arithmetic as implicit R with explicit A: A differs at most in zero signs
    assert torch.equal(Ri, Rr) and torch.equal(Ai, Ar)
    assert np.max(np.abs(host(Ai) - host(Ae))) <= TOL * rng
    assert np.max(np.abs(host(Ri) - host(Re))) <= TOL * rng
    assert np.max(np.abs(host(Ai) - ref.A)) <= TOL * rng
    assert abs(ri.netsim - ref.netsim) <= n * 1e-6 * rng


def test_fixed_count_messages_against_oracle():
    n = 2000
    say(f"implicit A fixed count n={n}")
    S = mixture(n, 177)
    Sd = apx.to_matrix(torch.from_numpy(S.astype(np.float32)))
    R, A, _, res, info = solve(Sd, 16, 1024, max_iter=37, conv_iter=0)
    assert res.iterations == 37 and info[2] == 37
    ref = oracle.ap(S, 0.9, 37, 0)
    rng = S.max() - S.min()
    assert np.max(np.abs(host(R) - ref.R)) <= TOL * rng
    assert np.max(np.abs(host(A) - ref.A)) <= TOL * rng


@pytest.mark.parametrize("cap_r,cap_a", [(16, 1), (16, 3), (1, 2)])
def test_list_overflow_hands_over_to_explicit(cap_r, cap_a):
    n = 1500
    say(f"implicit A overflow with capacities R {cap_r}, A {cap_a}")
    S = mixture(n, 191)
    Sd = apx.to_matrix(torch.from_numpy(S.astype(np.float32)))
    R, A, idx, res, info = solve(Sd, cap_r, cap_a)
    Re, Ae, ie, re, _ = solve(Sd, 0, 0)
    rng = S.max() - S.min()
    say(f"  iterations {res.iterations}, implicit A for {info[2]}, implicit R for {info[0]}")
    assert info[2] < res.iterations              # the hand-over happened
    assert res.converged and res.iterations == re.iterations
    assert torch.equal(idx, ie)
    assert np.max(np.abs(host(R) - host(Re))) <= TOL * rng
    assert np.max(np.abs(host(A) - host(Ae))) <= TOL * rng


def test_warm_start_keeps_explicit_a():
    n = 2400
    say(f"implicit A off for a warm start n={n}")
    S = mixture(n, 155)
    Sd = apx.to_matrix(torch.from_numpy(S.astype(np.float32)))
    apx.apx_set_implicit(16, 0)
    R, A = apx.empty_matrix(n), apx.empty_matrix(n)
    apx.pap_solve(Sd, R, A, 4, damping=0.9, max_iter=2000, conv_iter=15)
    torch.cuda.synchronize()
    assert apx.apx_last_solve_info()[2] == 0


def test_graph_and_repeat_bit_identical():
    n = 3000
    say(f"implicit A graph vs host launches n={n}")
    S = mixture(n, 166)
    Sd = apx.to_matrix(torch.from_numpy(S.astype(np.float32)))
    apx.apx_set_graphs(False)
    ref = solve(Sd, 16, 1024)
    apx.apx_set_graphs(True)
    for _ in range(2):
        got = solve(Sd, 16, 1024)
        for a, b in zip(got[:3], ref[:3]):
            assert torch.equal(a, b)
        assert got[3].netsim == ref[3].netsim


def test_long_rows_global_partials():
    # rows of 7 float4 chunks per thread (n in (24576, 25312] still fits
    # the LDS variant): the LDS and the global-partials variants give
    # identical messages; both agree with explicit messages
    n = 25000
    say(f"implicit A long rows n={n}")
    pts = synth.gaussian_mixture(n=n, d=16, k=30, seed=2601)
    X = torch.from_numpy(pts.X).cuda()
    Sd, _ = apx.ap_similarity(X, pref="median", noise_seed=2601, noise_rel=1e-12)
    out = {}
    for gp in ("0", "1"):
        os.environ["APX_IMPLICIT_A_GP"] = gp
        R, A, idx, res, info = solve(Sd, 16, 1024, max_iter=25, conv_iter=0)
        assert info[2] == 25
        out[gp] = (R.clone(), A.clone(), idx.clone())
        del R, A
    os.environ.pop("APX_IMPLICIT_A_GP", None)
    for a, b in zip(out["0"], out["1"]):
        assert torch.equal(a, b)
    Re, Ae, ie, re, _ = solve(Sd, 0, 0, max_iter=25, conv_iter=0)
    rng = float(Sd.max() - Sd.min())
    assert float((out["0"][0] - Re).abs().max()) <= TOL * rng
    assert float((out["0"][1] - Ae).abs().max()) <= TOL * rng


def test_six_chunks_per_thread_against_explicit():
    # n = 22000: six float4 chunks per thread, the longest rows on which the
    # implicit-A pass bounds each hot thread's rereads per chunk and appends
    # a chunk's first positives one at a time; 25 fixed iterations through
    # the passes in which most entries turn positive, against the explicit
    # messages (checked against the oracle elsewhere)
    n = 22000
    say(f"implicit A six chunks n={n}")
    pts = synth.gaussian_mixture(n=n, d=64, k=50, seed=2701)
    X = torch.from_numpy(pts.X).cuda()
    Sd, _ = apx.ap_similarity(X, pref="median", noise_seed=2701, noise_rel=1e-12)
    R, A, idx, res, info = solve(Sd, 16, 1024, max_iter=25, conv_iter=0)
    assert info[2] == 25                                   # implicit A throughout
    Re, Ae, ie, re, _ = solve(Sd, 0, 0, max_iter=25, conv_iter=0)
    rng = float(Sd.max() - Sd.min())
    assert float((R - Re).abs().max()) <= TOL * rng
    assert float((A - Ae).abs().max()) <= TOL * rng


def tie_matrix(n, dims, hi, seed, pref_q):
    """Duplicated integer points: S = -||x_i - x_k||^2 is integer and every
    column has a twin, so a+s and a+r are tied in many rows."""
    rng = np.random.default_rng(seed)
    base = rng.integers(0, hi, size=(n // 2, dims))
    X = np.concatenate([base, base])[rng.permutation(n)].astype(np.float64)
    S = -((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    off = S[~np.eye(n, dtype=bool)]
    np.fill_diagonal(S, np.floor(np.quantile(off, pref_q)))
    return S


def tied_rows(M):
    return int(((M == M.max(axis=1, keepdims=True)).sum(axis=1) > 1).sum())


def test_exact_ties_against_oracle():
    # damping 1/2 and a short fixed run on a small integer S: every message
    # is a short dyadic fraction, exact in FP32 and FP64, so ties survive and
    # the lowest-index rule decides them; all three forms equal the oracle
    n = 64
    say(f"exact ties n={n}")
    S = tie_matrix(n, 1, 6, 4306, 0.5)
    Sd = apx.to_matrix(torch.from_numpy(S.astype(np.float32)))
    ref = oracle.ap(S, 0.5, 10, 0)
    assert tied_rows(ref.A + ref.R) > 0
    for name, cr, ca in (("R and A", 16, 1024), ("R", 16, 0), ("explicit", 0, 0)):
        R, A, idx, res, info = solve(Sd, cr, ca, lam=0.5, max_iter=10, conv_iter=0)
        assert np.array_equal(idx.cpu().numpy(), ref.idx), name
        assert np.array_equal(host(R), ref.R) and np.array_equal(host(A), ref.A), name
        if name == "R and A":
            # twins put several R-listed columns on one thread: the run may
            # hand over to explicit messages before the end
            assert info[2] >= 1
            say(f"  implicit A for {info[2]} of 10 iterations")


def test_ties_implicit_a_equals_implicit_r():
    # 1024-thread rows: implicit A gives the same R, A and labels as implicit
    # R with explicit A, bit for bit, on a matrix full of exact ties
    n = 5000
    say(f"ties, implicit A vs implicit R, n={n}")
    S = tie_matrix(n, 2, 10, 4242 + n, 0.5)
    Sd = apx.to_matrix(torch.from_numpy(S.astype(np.float32)))
    Ra, Aa, ia, ra, info = solve(Sd, 16, 1024, lam=0.5, max_iter=30, conv_iter=0)
    Rr, Ar, ir, rr, _ = solve(Sd, 16, 0, lam=0.5, max_iter=30, conv_iter=0)
    say(f"  implicit A for {info[2]} of 30 iterations")
    assert info[2] >= 5          # (twins can overflow the R list: both runs hand over alike)
    assert tied_rows(host(Aa) + host(Ra)) > 0 and tied_rows(host(Aa) + S) > 0
    assert torch.equal(ia, ir) and torch.equal(Ra, Rr) and torch.equal(Aa, Ar)
