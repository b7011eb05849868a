"""The boundary's options, through the C ABI: raw labels, the finite check,
the message-change stop rule (Algorithm 1, Step 4), the empty exemplar
set, non-finite input to the similarity build, the caller-owned workspace
and lap_solve's preference modes.  Results are compared with the FP64
oracle on the same (FP32-rounded) S.
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
from paper_0910_1650_amd import ApxError  # noqa: E402

TOL = 1e-4


def say(msg):
    print(msg, flush=True)


def host(M):
    return M.detach().cpu().numpy().astype(np.float64)


def shared_S(pts, seed, pref="median"):
    """The oracle's S rounded once to FP32: (device matrix, FP64 copy of it)."""
    S32 = oracle.prepare(oracle.similarity(pts.X), pref, seed=seed).S.astype(np.float32)
    return apx.to_matrix(torch.from_numpy(S32)), S32.astype(np.float64)


@pytest.fixture(scope="module")
def c1():
    seed = 1021
    pts = synth.gaussian_2d(n=900, k=8, seed=seed)
    return shared_S(pts, seed)


@pytest.fixture(scope="module")
def c2():
    seed = 2021
    pts = synth.gaussian_mixture(n=5000, d=32, k=20, seed=seed)
    return shared_S(pts, seed)


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_raw_labels_equal_oracle_decisions(which, request):
    S, S64 = request.getfixturevalue(which)
    n = S.shape[0]
    say(f"raw labels n={n}")
    R, A = apx.empty_matrix(n), apx.empty_matrix(n)
    idx, res = apx.ap_solve(S, R, A, 0.9, 2000, 15, flags=apx.APX_RAW_LABELS)
    ref = oracle.ap(S64, 0.9, 2000, 15)
    assert res.converged and ref.converged and res.iterations == ref.iterations
    d = idx.cpu().numpy()
    assert np.array_equal(d, ref.dec)
    ex = d == np.arange(n)
    assert res.n_exemplars == int(ex.sum())
    dp = float(sum(S64[i, d[i]] for i in range(n) if d[i] != i))
    ep = float(np.diag(S64)[ex].sum())
    rng = S64.max() - S64.min()
    assert abs(res.dpsim - dp) <= n * 1e-6 * rng and abs(res.expref - ep) <= n * 1e-6 * rng


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), float("-inf")])
@pytest.mark.parametrize("call", ["ap_solve", "pap_solve", "ap_solve_batched"])
def test_check_finite_rejects_before_any_write(c1, bad, call):
    S0, _ = c1
    n = S0.shape[0]
    S = apx.empty_matrix(n)
    S.copy_(S0)
    S[17, 403] = bad
    R, A = apx.empty_matrix(n, fill=7.0), apx.empty_matrix(n, fill=9.0)
    say(f"finite check {call} {bad}")
    with pytest.raises(ApxError) as ei:
        if call == "ap_solve":
            apx.ap_solve(S, R, A, 0.9, 100, 15, flags=apx.APX_CHECK_FINITE)
        elif call == "pap_solve":
            apx.pap_solve(S, R, A, 3, damping=0.9, flags=apx.APX_CHECK_FINITE)
        else:
            apx.ap_solve_batched([S0, S], [apx.empty_matrix(n), R], [apx.empty_matrix(n), A],
                                 damping=0.9, flags=apx.APX_CHECK_FINITE)
    assert ei.value.status == apx.APX_EINVAL
    torch.cuda.synchronize()
    assert bool((R == 7.0).all()) and bool((A == 9.0).all())


def test_similarity_rejects_non_finite_points():
    pts = synth.gaussian_2d(n=300, k=4, seed=1023)
    S = apx.empty_matrix(300, fill=5.0)
    for bad in (float("nan"), float("inf")):
        X = torch.from_numpy(pts.X).cuda()
        X[11, 1] = bad
        with pytest.raises(ApxError) as ei:
            apx.ap_similarity(X, S, pref="median", noise_seed=1, noise_rel=1e-12)
        assert ei.value.status == apx.APX_EINVAL
        torch.cuda.synchronize()
        assert bool((S == 5.0).all())
    X = torch.from_numpy(pts.X).cuda()
    pv = torch.zeros(300, dtype=torch.float32, device="cuda")
    pv[5] = float("inf")
    with pytest.raises(ApxError):
        apx.ap_similarity(X, S, pref=pv)
    torch.cuda.synchronize()
    assert bool((S == 5.0).all())


def test_similarity_rejects_overflow():
    X = torch.full((64, 3), 1e20, dtype=torch.float32, device="cuda")
    X[::2] *= -1.0
    with pytest.raises(ApxError) as ei:
        apx.ap_similarity(X, pref="median")
    assert ei.value.status == apx.APX_EINVAL


@pytest.mark.parametrize("n", [600, 4200])
def test_empty_exemplar_set(n):
    """A preference far below every similarity: after one iteration no point
    chooses itself, so E is empty: labels -1 and netsim NaN, as the oracle."""
    pts = synth.gaussian_2d(n=n, k=5, seed=1025)
    S64 = oracle.prepare(oracle.similarity(pts.X), -1.0e6, seed=1025).S
    S32 = S64.astype(np.float32)
    S = apx.to_matrix(torch.from_numpy(S32))
    R, A = apx.empty_matrix(n), apx.empty_matrix(n)
    say(f"empty exemplar set n={n}")
    idx, res = apx.ap_solve(S, R, A, 0.9, 1, 15)
    ref = oracle.ap(S32.astype(np.float64), 0.9, 1, 15)
    assert ref.n_exemplars == 0 and np.all(ref.idx == -1)
    assert res.n_exemplars == 0 and not res.converged and res.iterations == 1
    assert np.all(idx.cpu().numpy() == -1)
    assert np.isnan(res.netsim) and np.isnan(res.dpsim) and np.isnan(res.expref)


def _msg_stop_cases(S64, lam, cap):
    """Tolerances (fractions of the range) whose oracle stop iteration does not
    move when the tolerance moves by 0.5%: far from a tie with a change."""
    rng = S64.max() - S64.min()
    out = []
    for frac in (3e-2, 1e-2, 3e-3):
        tol = frac * rng
        t0 = oracle.ap(S64, lam, cap, 0, msg_tol=tol, finalize_labels=False)
        lo = oracle.ap(S64, lam, cap, 0, msg_tol=tol * 0.995, finalize_labels=False)
        hi = oracle.ap(S64, lam, cap, 0, msg_tol=tol * 1.005, finalize_labels=False)
        if t0.converged and lo.iterations == t0.iterations == hi.iterations:
            out.append((tol, t0))
    return out


@pytest.mark.parametrize("n", [700, 5000])
def test_message_threshold_stop(n):
    seed = 1027
    pts = synth.gaussian_2d(n=n, k=6, seed=seed)
    S, S64 = shared_S(pts, seed)
    rng = S64.max() - S64.min()
    cases = _msg_stop_cases(S64, 0.9, 400)
    assert cases, "no well-separated tolerance"
    for tol, ref in cases:
        say(f"message threshold n={n} tol={tol / rng:.0e} range, oracle stops at {ref.iterations}")
        R, A = apx.empty_matrix(n), apx.empty_matrix(n)
        idx, res = apx.ap_solve(S, R, A, 0.9, 400, 0, flags=apx.APX_MSG_THRESHOLD, msg_tol=tol)
        assert res.converged and res.iterations == ref.iterations
        assert np.max(np.abs(host(R) - ref.R)) <= TOL * rng
        assert np.max(np.abs(host(A) - ref.A)) <= TOL * rng


def test_bad_flags_rejected(c1):
    S, _ = c1
    n = S.shape[0]
    R, A = apx.empty_matrix(n), apx.empty_matrix(n)
    with pytest.raises(ApxError):
        apx.ap_solve(S, R, A, 0.9, 10, 0, flags=64)
    with pytest.raises(ApxError):
        apx.ap_solve(S, R, A, 0.9, 10, 0, flags=apx.APX_MSG_THRESHOLD, msg_tol=-1.0)
    with pytest.raises(ApxError) as ei:
        apx.ap_solve_batched([S], damping=0.9, flags=apx.APX_RAW_LABELS)
    assert ei.value.status == apx.APX_ENOTIMPL


@pytest.fixture
def restore_workspace():
    yield
    apx.apx_set_workspace(None)


def test_caller_workspace_same_results(c2, restore_workspace):
    S, _ = c2
    n, ld = S.shape[0], S.stride(0)
    R0, A0 = apx.empty_matrix(n), apx.empty_matrix(n)
    idx0, res0 = apx.ap_solve(S, R0, A0, 0.9, 2000, 15)
    need = apx.apx_workspace_size(apx.APX_OP_SOLVE, n, ld)
    assert need > 0
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    apx.apx_set_workspace(buf)
    assert apx.apx_workspace_bytes() == need
    R1, A1 = apx.empty_matrix(n), apx.empty_matrix(n)
    say(f"caller workspace {need} bytes")
    idx1, res1 = apx.ap_solve(S, R1, A1, 0.9, 2000, 15)
    assert res1.iterations == res0.iterations and res1.netsim == res0.netsim
    assert torch.equal(idx0, idx1) and torch.equal(R0, R1) and torch.equal(A0, A1)
    # too small: ENOMEM, nothing written
    apx.apx_set_workspace(buf[: need - 4096])
    R2 = apx.empty_matrix(n, fill=3.0)
    with pytest.raises(ApxError) as ei:
        apx.ap_solve(S, R2, A1, 0.9, 2000, 15)
    assert ei.value.status == apx.APX_ENOMEM
    torch.cuda.synchronize()
    assert bool((R2 == 3.0).all())


def test_caller_workspace_sizes_cover_every_call(restore_workspace):
    seed = 1029
    pts = synth.gaussian_2d(n=1200, k=6, seed=seed)
    n, d = pts.X.shape
    X = torch.from_numpy(pts.X).cuda()
    ld = apx.round_ld(n)
    sizes = np.array([300, 500, 400], dtype=np.int64)
    need = max(apx.apx_workspace_size(apx.APX_OP_SIMILARITY, n),
               apx.apx_workspace_size(apx.APX_OP_ITERATE, n, ld),
               apx.apx_workspace_size(apx.APX_OP_SOLVE, n, ld),
               apx.apx_workspace_size(apx.APX_OP_PAP, n, ld, count=3, sizes=sizes),
               apx.apx_workspace_size(apx.APX_OP_LAP, n, d=d, count=400),
               apx.apx_workspace_size(apx.APX_OP_SOLVE_BATCHED, count=3, sizes=sizes))
    # reference results with the library's own workspace
    S, _ = apx.ap_similarity(X, pref="median", noise_seed=seed)
    R, A = apx.empty_matrix(n), apx.empty_matrix(n)
    off = np.concatenate([[0], np.cumsum(sizes)])
    i_pap, r_pap, _ = apx.pap_solve(S, R, A, 3, offsets=off, damping=0.9, max_iter=1000)
    i_lap, r_lap, _ = apx.lap_solve(X, 400, landmarks=np.arange(0, n, 3), seed=seed)
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    apx.apx_set_workspace(buf)
    S2, _ = apx.ap_similarity(X, pref="median", noise_seed=seed)
    assert torch.equal(S, S2)
    R2, A2 = apx.empty_matrix(n), apx.empty_matrix(n)
    apx.ap_iterate(S2, R2.fill_(0), A2.fill_(0), 0.9, 5)
    j_pap, q_pap, _ = apx.pap_solve(S2, R2, A2, 3, offsets=off, damping=0.9, max_iter=1000)
    j_lap, q_lap, _ = apx.lap_solve(X, 400, landmarks=np.arange(0, n, 3), seed=seed)
    assert torch.equal(i_pap, j_pap) and r_pap.netsim == q_pap.netsim
    assert torch.equal(i_lap, j_lap) and r_lap.netsim == q_lap.netsim


def test_lap_scalar_preference():
    seed = 1031
    pts = synth.gaussian_2d(n=3000, k=7, seed=seed)
    X = torch.from_numpy(pts.X).cuda()
    M = synth.landmarks(3000, 500, seed)
    p = -40.0
    idx, res, ex = apx.lap_solve(X, 500, landmarks=M, seed=seed, damping=0.9, pref=p)
    ref = oracle.lap(pts.X, M, seed=seed, lam=0.9, pref=p)
    assert np.array_equal(np.sort(ex), ref.exemplars)
    assert np.array_equal(idx.cpu().numpy(), ref.idx)
    assert abs(res.expref - p * len(ex)) <= 1e-9
    with pytest.raises(ApxError):
        apx.lap_solve(X, 500, landmarks=M, seed=seed, flags=apx.APX_RAW_LABELS)
