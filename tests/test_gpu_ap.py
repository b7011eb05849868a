"""GPU parity of the AP iteration (ap_iterate / ap_solve) against the FP64 oracle.

Tolerance: after a fixed iteration count, max|dR| and max|dA| must be within
1e-4 * (max S - min S); exemplar sets, labels and stop iterations must be
identical at convergence.  Inputs are the oracle's S (FP64, with the
tie-break noise) rounded once to FP32.
"""
import json
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


def dev(S64):
    return apx.to_matrix(torch.from_numpy(np.ascontiguousarray(S64, dtype=np.float32)))


def host(M):
    return M.detach().cpu().numpy().astype(np.float64)


def zeros(n):
    return apx.empty_matrix(n, fill=0.0)


def c1_S(seed, n=1000, k=10):
    pts = synth.gaussian_2d(n=n, k=k, seed=seed)
    return oracle.prepare(oracle.similarity(pts.X), "median", seed=seed).S


def say(msg):
    print(msg, flush=True)


def test_four_point_example_exact(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "four_points.json")))
    S = dev(np.asarray(g["S"]))
    for t, key in ((1, "iter1"), (2, "iter2")):
        R, A = zeros(4), zeros(4)
        d = torch.empty(4, dtype=torch.int32, device="cuda")
        apx.ap_iterate(S, R, A, g["lambda"], t, d)
        torch.cuda.synchronize()
        assert np.array_equal(host(R), np.asarray(g[key]["R"])), key
        assert np.array_equal(host(A), np.asarray(g[key]["A"])), key
        assert d.cpu().tolist() == g[key]["decisions"]
    R, A = zeros(4), zeros(4)
    idx, res = apx.ap_solve(S, R, A, g["lambda"], 200, 15)
    c = g["converged"]
    assert res.converged and res.iterations == c["stop_iteration"]
    assert idx.cpu().tolist() == c["idx"]
    assert (res.netsim, res.dpsim, res.expref) == (c["netsim"], c["dpsim"], c["expref"])


# Damping 0.5 (the 2-D configuration) is chaotic at rounding level: two FP64
# implementations that differ only in summation order drift apart by O(range)
# after ~50 iterations, so fixed-count parity at damping 0.5 is checked up to
# 10 iterations and longer runs use damping 0.9.
@pytest.mark.parametrize("seed", [1001, 1002, 1003])
@pytest.mark.parametrize("lam,t", [(0.5, 1), (0.5, 2), (0.5, 5), (0.5, 10), (0.9, 20), (0.9, 50),
                                   (0.9, 100)])
def test_c1_messages_fixed_count(seed, lam, t):
    say(f"c1 messages seed={seed} lambda={lam} t={t}")
    S64 = c1_S(seed)
    rng = S64.max() - S64.min()
    ref = oracle.ap(S64, lam, t, 0)
    S = dev(S64)
    R, A = zeros(1000), zeros(1000)
    d = torch.empty(1000, dtype=torch.int32, device="cuda")
    apx.ap_iterate(S, R, A, lam, t, d)
    torch.cuda.synchronize()
    assert np.max(np.abs(host(R) - ref.R)) <= TOL * rng
    assert np.max(np.abs(host(A) - ref.A)) <= TOL * rng


@pytest.mark.parametrize("n", [2, 3, 5, 64, 257, 1023, 4097, 5003])
def test_ragged_sizes_fixed_count(n):
    say(f"ragged n={n}")
    pts = synth.gaussian_mixture(n=n, d=8, k=max(1, min(12, n // 3)), seed=n)
    S64 = oracle.prepare(oracle.similarity(pts.X), "median", seed=n).S
    rng = S64.max() - S64.min()
    ref = oracle.ap(S64, 0.9, 12, 0)
    S = dev(S64)
    R, A = zeros(n), zeros(n)
    apx.ap_iterate(S, R, A, 0.9, 12)
    torch.cuda.synchronize()
    assert np.max(np.abs(host(R) - ref.R)) <= TOL * rng
    assert np.max(np.abs(host(A) - ref.A)) <= TOL * rng


@pytest.mark.parametrize("seed", [1001, 1002, 1003, 1004, 1005])
def test_c1_family_converged_exemplars(seed):
    """Exemplar sets, labels and the stop iteration equal the oracle's at
    convergence (damping 0.9)."""
    say(f"c1 lambda=0.9 converge seed={seed}")
    S64 = c1_S(seed)
    ref = oracle.ap(S64, 0.9, 1000, 15)
    S = dev(S64)
    R, A = zeros(1000), zeros(1000)
    idx, res = apx.ap_solve(S, R, A, 0.9, 1000, 15)
    assert ref.converged and res.converged
    assert res.iterations == ref.iterations
    assert res.n_exemplars == ref.n_exemplars
    assert np.array_equal(idx.cpu().numpy(), ref.idx)
    rng = S64.max() - S64.min()
    assert abs(res.netsim - ref.netsim) <= 1000 * 1e-6 * rng


def test_iterate_composes_bit_exact():
    S = dev(c1_S(1006, n=700))
    R1, A1, R2, A2 = zeros(700), zeros(700), zeros(700), zeros(700)
    apx.ap_iterate(S, R1, A1, 0.5, 7)
    apx.ap_iterate(S, R1, A1, 0.5, 5)
    apx.ap_iterate(S, R2, A2, 0.5, 12)
    torch.cuda.synchronize()
    assert torch.equal(R1, R2) and torch.equal(A1, A2)


def test_solve_matches_iterate_and_is_deterministic():
    S = dev(c1_S(1007, n=900))
    Ri, Ai = zeros(900), zeros(900)
    apx.ap_iterate(S, Ri, Ai, 0.5, 33)
    outs = []
    for _ in range(2):
        R, A = zeros(900), zeros(900)
        idx, res = apx.ap_solve(S, R, A, 0.5, 33, 0)
        assert res.iterations == 33 and not res.converged
        outs.append((R.clone(), A.clone(), idx.clone()))
    assert torch.equal(outs[0][0], Ri) and torch.equal(outs[0][1], Ai)
    assert all(torch.equal(a, b) for a, b in zip(outs[0], outs[1]))


def test_warm_start_resume_matches():
    """ap_solve from (R_t, A_t) continues exactly like an unsplit run."""
    S = dev(c1_S(1008, n=600))
    R, A = zeros(600), zeros(600)
    apx.ap_iterate(S, R, A, 0.5, 10)
    R2, A2 = zeros(600), zeros(600)
    apx.ap_iterate(S, R2, A2, 0.5, 25)
    _, res = apx.ap_solve(S, R, A, 0.5, 15, 0, warm=apx.APX_WARM_AR)
    assert res.iterations == 15
    assert torch.equal(R, R2) and torch.equal(A, A2)


def test_single_point():
    S = dev(np.array([[-3.5]]))
    idx, res = apx.ap_solve(S, zeros(1), zeros(1), 0.5, 10, 15)
    assert idx.cpu().tolist() == [0] and res.netsim == -3.5 and res.iterations == 0


def test_invalid_arguments_leave_outputs_untouched():
    S = dev(c1_S(1009, n=64))
    R, A = zeros(64), zeros(64)
    R.fill_(7.0)
    with pytest.raises(apx.ApxError) as e:
        apx.ap_iterate(S, R, A, 1.0, 3)
    assert e.value.status == apx.APX_EINVAL
    with pytest.raises(apx.ApxError):
        apx.ap_solve(S, R, A, 0.5, 0, 15)
    torch.cuda.synchronize()
    assert bool((R == 7.0).all()) and bool((A == 0.0).all())
