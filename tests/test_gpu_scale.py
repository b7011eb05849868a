"""Full-size run of the partition workload: 40000 points on a union of 20
random 5-D subspaces of R^100 (noise 0.05), split into 8 random parts of
3000-7000 points (Section 3, Algorithm 2), against cold-start AP on the same
S.  Checks what holds at any size (every sub-problem and the full run
stopped by the rule, exemplars label themselves, sampled labels are the most
similar exemplar) and prints wall time, iterations, net similarity and the
true/false association rates on the ground-truth subspaces (the pair
metrics of Section 5)."""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0910_1650_amd as apx  # noqa: E402


def say(msg):
    print(msg, flush=True)


def association_rates(truth, lab):
    """(true, false) association rates: the share of same-class pairs put in
    one cluster, and of different-class pairs put in one cluster."""
    _, t = np.unique(truth, return_inverse=True)
    _, c = np.unique(lab, return_inverse=True)
    table = np.zeros((t.max() + 1, c.max() + 1), dtype=np.int64)
    np.add.at(table, (t, c), 1)
    pairs = lambda x: (x * (x - 1) // 2).sum()      # noqa: E731
    same_both = pairs(table)
    same_truth = pairs(table.sum(axis=1))
    same_clust = pairs(table.sum(axis=0))
    n = len(truth)
    total = n * (n - 1) // 2
    return same_both / same_truth, (same_clust - same_both) / (total - same_truth)


def check_labels(S, lab, rows):
    ex = np.flatnonzero(lab == np.arange(lab.size))
    assert ex.size > 0 and np.all(lab[ex] == ex)
    Sr = S[torch.from_numpy(rows).cuda()].cpu().numpy()
    for r, i in enumerate(rows):
        if lab[i] != i:
            assert lab[i] == ex[np.argmax(Sr[r, ex])]


def test_c3_partition_ap_full_size():
    n, seed = 40000, 3001
    pts = synth.subspaces(n=n, d=100, n_sub=20, dim=5, noise=0.05, seed=seed)
    X = torch.from_numpy(pts.X).cuda()
    S, p = apx.ap_similarity(X, pref="median", noise_seed=seed, noise_rel=1e-12)
    perm, offsets = synth.random_partition(n, 8, 3000, 7000, seed=seed)
    R, A = apx.empty_matrix(n), apx.empty_matrix(n)
    rows = np.random.default_rng(1).choice(n, size=300, replace=False)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx, res, subs = apx.pap_solve(S, R, A, 8, perm, offsets, damping=0.9, max_iter=2000, conv_iter=15)
    t_pap = (time.perf_counter() - t0) * 1e3
    lab_pap = idx.cpu().numpy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx_c, res_c = apx.ap_solve(S, R, A, 0.9, 2000, 15)
    t_cold = (time.perf_counter() - t0) * 1e3
    lab_cold = idx_c.cpu().numpy()

    tar_p, far_p = association_rates(pts.labels, lab_pap)
    tar_c, far_c = association_rates(pts.labels, lab_cold)
    say(f"C3 n={n}: parts {np.diff(offsets).tolist()}, sub-problem iterations "
        f"{[r.iterations for r in subs]}")
    say(f"  cold: {t_cold:.1f} ms, {res_c.iterations} iterations, |E|={res_c.n_exemplars}, "
        f"netsim {res_c.netsim:.3f}, TAR {tar_c:.4f} FAR {far_c:.5f}")
    say(f"  PAP : {t_pap:.1f} ms, {res.iterations} iterations (+ max {max(r.iterations for r in subs)} "
        f"in the parts), |E|={res.n_exemplars}, netsim {res.netsim:.3f}, TAR {tar_p:.4f} FAR {far_p:.5f}")
    assert all(r.converged for r in subs) and res.converged and res_c.converged
    check_labels(S, lab_pap, rows)
    check_labels(S, lab_cold, rows)
    # With the median preference AP finds ~2000 small clusters along the
    # subspaces (true association rate ~0.01): they must be nearly pure, i.e.
    # points of different subspaces are almost never put together.
    assert far_p < 0.001 and far_c < 0.001
