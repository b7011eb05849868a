"""Batched multi-instance AP and partition AP (Algorithm 2) on the GPU
against the FP64 oracle.

Inputs are the oracle's S (FP64 with tie noise) rounded once to FP32, so
the comparison isolates the batched iteration and the partition steps.
Damping 0.9 (exemplar sets are compared at convergence; at damping 0.5 the
iteration is chaotic at rounding level, see test_gpu_ap)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0910_1650_amd as apx  # noqa: E402


def dev(S64):
    return apx.to_matrix(torch.from_numpy(np.ascontiguousarray(S64, dtype=np.float32)))


def inst_S(pts, seed):
    return oracle.prepare(oracle.similarity(pts.X), "median", seed=seed).S


def test_batched_matches_oracle_per_instance():
    insts = synth.batch_instances(count=12, seed0=3101)
    Ss = [inst_S(p, p.seed) for p in insts]
    print("batched: sizes", [S.shape[0] for S in Ss], flush=True)
    idxs, res = apx.ap_solve_batched([dev(S) for S in Ss], damping=0.9, max_iter=1000, conv_iter=15)
    for S, idx, r in zip(Ss, idxs, res):
        ref = oracle.ap(S, 0.9, 1000, 15)
        assert r.converged == ref.converged
        assert r.iterations == ref.iterations
        assert np.array_equal(idx.cpu().numpy(), ref.idx)
        rng = S.max() - S.min()
        assert abs(r.netsim - ref.netsim) <= S.shape[0] * 1e-6 * rng


def test_batched_fixed_count_messages():
    insts = synth.batch_instances(count=5, seed0=3301)
    Ss = [inst_S(p, p.seed) for p in insts]
    Rs = [apx.empty_matrix(S.shape[0]) for S in Ss]
    As = [apx.empty_matrix(S.shape[0]) for S in Ss]
    apx.ap_solve_batched([dev(S) for S in Ss], Rs, As, damping=0.9, max_iter=40, conv_iter=0)
    for S, R, A in zip(Ss, Rs, As):
        ref = oracle.ap(S, 0.9, 40, 0)
        rng = S.max() - S.min()
        assert np.max(np.abs(R.cpu().numpy() - ref.R)) <= 1e-4 * rng
        assert np.max(np.abs(A.cpu().numpy() - ref.A)) <= 1e-4 * rng


def test_batched_512_instances():
    """The 512-instance workload (n in [100, 2000], 2-20 clusters): every
    instance valid, a sample against the oracle, and deterministic."""
    insts = synth.batch_instances(count=512, seed0=3101)
    print("batched 512 instances, sum n^2 =", sum(len(p.X) ** 2 for p in insts), flush=True)
    Ss = [inst_S(p, p.seed) for p in insts]
    Sd = [dev(S) for S in Ss]
    idxs, res = apx.ap_solve_batched(Sd, damping=0.9, max_iter=1000, conv_iter=15)
    idxs2, res2 = apx.ap_solve_batched(Sd, damping=0.9, max_iter=1000, conv_iter=15)
    for a, b, ra, rb in zip(idxs, idxs2, res, res2):
        assert torch.equal(a, b) and ra.iterations == rb.iterations and ra.netsim == rb.netsim
    for S, idx, r in zip(Ss, idxs, res):
        lab = idx.cpu().numpy()
        ex = np.flatnonzero(lab == np.arange(lab.size))
        assert ex.size == r.n_exemplars > 0
        assert np.all(lab[lab] == lab)                 # every label is an exemplar
        # reported net similarity = sum_i s(i, idx(i)) on the matrix the GPU used
        S32 = S.astype(np.float32).astype(np.float64)
        assert abs(S32[np.arange(lab.size), lab].sum() - r.netsim) <= 1e-6 * abs(r.netsim) + 1e-3
    for j in np.random.default_rng(0).choice(512, size=16, replace=False):
        ref = oracle.ap(Ss[j], 0.9, 1000, 15)
        assert res[j].iterations == ref.iterations, j
        assert np.array_equal(idxs[j].cpu().numpy(), ref.idx), j


@pytest.mark.parametrize("k", [2, 4])
def test_pap_matches_oracle(k):
    n = 1500
    pts = synth.subspaces(n=n, d=20, n_sub=6, dim=3, seed=3001 + k)
    S = inst_S(pts, pts.seed)
    perm, offsets = synth.random_partition(n, parts=k, lo=200, hi=600, seed=pts.seed)
    print(f"pap n={n} k={k} sizes={np.diff(offsets).tolist()}", flush=True)
    ref = oracle.pap(S, k, perm, offsets, lam=0.9, max_iter=1000, conv_iter=15)
    R, A = apx.empty_matrix(n), apx.empty_matrix(n)
    idx, res, sub = apx.pap_solve(dev(S), R, A, k, perm, offsets, damping=0.9, max_iter=1000, conv_iter=15)
    for sr, so in zip(sub, ref.subs):
        assert sr.iterations == so.iterations and sr.n_exemplars == so.n_exemplars
    assert res.iterations == ref.full.iterations
    assert np.array_equal(idx.cpu().numpy(), ref.full.idx)


def test_pap_even_split_default():
    n = 1200
    pts = synth.gaussian_2d(n=n, k=8, seed=77)
    S = inst_S(pts, 77)
    ref = oracle.pap(S, 3, lam=0.9, max_iter=1000, conv_iter=15)
    idx, res, sub = apx.pap_solve(dev(S), apx.empty_matrix(n), apx.empty_matrix(n), 3,
                                  damping=0.9, max_iter=1000, conv_iter=15)
    assert res.iterations == ref.full.iterations
    assert np.array_equal(idx.cpu().numpy(), ref.full.idx)


def test_pap_singleton_parts_equal_cold_ap():
    n = 300
    S = dev(inst_S(synth.gaussian_2d(n=n, k=5, seed=9), 9))
    R1, A1 = apx.empty_matrix(n), apx.empty_matrix(n)
    i1, r1 = apx.ap_solve(S, R1, A1, 0.9, 500, 15)
    R2, A2 = apx.empty_matrix(n), apx.empty_matrix(n)
    i2, r2, _ = apx.pap_solve(S, R2, A2, n, damping=0.9, max_iter=500, conv_iter=15)
    assert r1.iterations == r2.iterations
    assert torch.equal(i1, i2) and torch.equal(R1, R2) and torch.equal(A1, A2)


def test_pap_rejects_bad_partition():
    S = dev(inst_S(synth.gaussian_2d(n=50, k=3, seed=1), 1))
    with pytest.raises(apx.ApxError):
        apx.pap_solve(S, apx.empty_matrix(50), apx.empty_matrix(50), 2, perm=np.zeros(50, dtype=np.int64))
    with pytest.raises(apx.ApxError):
        apx.pap_solve(S, apx.empty_matrix(50), apx.empty_matrix(50), 2, offsets=[0, 60, 50])


def test_more_instances_than_workgroups():
    """1300 small instances (more than the persistent grid holds): one-
    workgroup teams each solve a queue of instances; every instance equals
    its own oracle run."""
    rng = np.random.default_rng(5)
    Ss = []
    for j in range(1300):
        n = int(rng.integers(12, 48))
        pts = synth.gaussian_2d(n=n, k=3, seed=7000 + j)
        Ss.append(inst_S(pts, 7000 + j))
    print("batched: 1300 instances", flush=True)
    idxs, res = apx.ap_solve_batched([dev(S) for S in Ss], damping=0.9, max_iter=500, conv_iter=15)
    for j, (S, idx, r) in enumerate(zip(Ss, idxs, res)):
        ref = oracle.ap(S, 0.9, 500, 15)
        assert r.iterations == ref.iterations and r.converged == ref.converged, j
        assert np.array_equal(idx.cpu().numpy(), ref.idx), j


def test_one_large_instance_runs_as_a_team():
    """A batch whose instances are far from equal: one large instance takes a
    team of many workgroups (device barriers between its passes) next to
    small ones; messages after a fixed count and the converged exemplars
    against the oracle."""
    sizes = [6000, 300, 450]
    Ss = [inst_S(synth.gaussian_2d(n=n, k=6, seed=7900 + n), 7900 + n) for n in sizes]
    print("batched: team instance", sizes, flush=True)
    Rs = [apx.empty_matrix(n) for n in sizes]
    As = [apx.empty_matrix(n) for n in sizes]
    apx.ap_solve_batched([dev(S) for S in Ss], Rs, As, damping=0.9, max_iter=60, conv_iter=0)
    for S, R, A in zip(Ss, Rs, As):
        ref = oracle.ap(S, 0.9, 60, 0)
        rng = S.max() - S.min()
        assert np.max(np.abs(R.cpu().numpy() - ref.R)) <= 1e-4 * rng
        assert np.max(np.abs(A.cpu().numpy() - ref.A)) <= 1e-4 * rng
    idxs, res = apx.ap_solve_batched([dev(S) for S in Ss], damping=0.9, max_iter=1000, conv_iter=15)
    idxs2, res2 = apx.ap_solve_batched([dev(S) for S in Ss], damping=0.9, max_iter=1000, conv_iter=15)
    for S, idx, r, idx2, r2 in zip(Ss, idxs, res, idxs2, res2):
        ref = oracle.ap(S, 0.9, 1000, 15)
        assert r.iterations == ref.iterations
        assert np.array_equal(idx.cpu().numpy(), ref.idx)
        assert torch.equal(idx, idx2) and r.netsim == r2.netsim


def test_tuned_batched_plan_matches_oracle():
    """apx_autotune_batched picks a plan for the batch's shape from the
    timed candidates; the batch solved with it still matches the oracle."""
    insts = synth.batch_instances(count=12, seed0=3151)
    Ss = [inst_S(p, p.seed) for p in insts]
    sizes = [S.shape[0] for S in Ss]
    apx.apx_tune_clear()
    try:
        pick = apx.apx_autotune_batched(sizes)
        print("batched plan pick:", pick, flush=True)
        assert 1 <= pick["wpc"] <= 4 and pick["min_rows"] in (2, 8, 32) and pick["ms"] > 0
        idxs, res = apx.ap_solve_batched([dev(S) for S in Ss], damping=0.9, max_iter=1000, conv_iter=15)
    finally:
        apx.apx_tune_clear()
    for S, idx, r in zip(Ss, idxs, res):
        ref = oracle.ap(S, 0.9, 1000, 15)
        assert r.converged == ref.converged and r.iterations == ref.iterations
        assert np.array_equal(idx.cpu().numpy(), ref.idx)
