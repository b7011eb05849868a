"""Matrix-free AP (beyond the paper; Section 2's similarity and Algorithm 1)
against the stored-S solve and the FP64 oracle's stored result.

ap_solve_mf rebuilds S from the points one row panel at a time in every
iteration (no n x n buffer) with the values ap_similarity stores, and runs
the implicit message passes on those rows.  Checks:

* one panel (the stored path's grouping of the column sums): the same
  labels, stop iteration and net similarity as ap_similarity + ap_solve;
* several panels with a ragged last one (n = 3000 and 6000 with partials
  in LDS, n = 33000 with global partials): the same exemplar set, labels and
  stop iteration (the column sums group their rows per panel: rounding
  only), net similarity equal (it sums the same S entries in one order);
* the C2 configuration (N = 20000, 64-D mixture, damping 0.9): the oracle's
  exemplar set, labels and stop iteration from the stored golden file;
* errors: raw labels and the message-change rule (they need R and A), a
  panel below one row per workgroup, sizes outside the implicit passes.
"""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0910_1650_amd as apx  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "c2_n20000_d64_k50_seed2001.json")


def _stored(X, seed, lam, max_iter, conv_iter, pref="median"):
    """ap_similarity + ap_solve with implicit R and A at any size (the form
    the matrix-free solve runs)."""
    n = X.shape[0]
    S, p = apx.ap_similarity(X, pref=pref, noise_seed=seed, noise_rel=1e-12)
    R, A = apx.empty_matrix(n), apx.empty_matrix(n)
    try:
        apx.apx_set_implicit(16, 2)
        apx.apx_set_implicit_a(1024, 2)
        idx, res = apx.ap_solve(S, R, A, lam, max_iter, conv_iter)
        assert apx.apx_last_solve_info()[2] == res.iterations
    finally:
        apx.apx_set_implicit(16)
        apx.apx_set_implicit_a(1024)
    del S, R, A
    return idx.cpu().numpy(), res, p


@pytest.mark.parametrize("n,pref,rows_few", [(6000, "median", 1000), (6000, -300.0, 1000), (3000, "median", 700),
                                              (33000, "median", 4000)])
def test_matrix_free_matches_stored_path(n, pref, rows_few):
    seed = 6201
    print(f"matrix-free n={n} pref={pref}", flush=True)
    pts = synth.gaussian_mixture(n=n, d=16, k=20, seed=seed)
    X = torch.from_numpy(pts.X).cuda()
    lab0, res0, p0 = _stored(X, seed, 0.9, 1000, 15, pref)
    for rows in (n, rows_few):
        idx, res, p = apx.ap_solve_mf(X, pref=pref, noise_seed=seed, noise_rel=1e-12, damping=0.9,
                                      max_iter=1000, conv_iter=15, panel_rows=rows)
        lab = idx.cpu().numpy()
        print(f"  panel {rows}: {res.iterations} iterations (stored {res0.iterations}), "
              f"{res.n_exemplars} exemplars, netsim {res.netsim:.6f} (stored {res0.netsim:.6f}), "
              f"implicit passes {apx.apx_last_solve_info()}", flush=True)
        assert p == p0
        assert res.converged and res0.converged
        assert res.iterations == res0.iterations
        assert np.array_equal(lab, lab0)
        assert res.netsim == res0.netsim


def test_matrix_free_c2_oracle_exemplars():
    g = json.load(open(GOLDEN))
    n, seed = g["args"]["n"], g["args"]["seed"]
    print(f"matrix-free c2 n={n}", flush=True)
    pts = synth.gaussian_mixture(**g["args"])
    X = torch.from_numpy(pts.X).cuda()
    idx, res, p = apx.ap_solve_mf(X, pref="median", noise_seed=g["noise_seed"], noise_rel=g["noise_rel"],
                                  damping=g["damping"], max_iter=g["max_iter"], conv_iter=g["conv_iter"],
                                  panel_rows=3000)
    lab = idx.cpu().numpy()
    ex = np.flatnonzero(lab == np.arange(n))
    print(f"  {res.iterations} iterations (oracle {g['iterations']}), {len(ex)} exemplars, "
          f"netsim {res.netsim:.4f} (oracle {g['netsim']:.4f})", flush=True)
    assert abs(p - g["preference"]) <= 1e-6 * g["range"]
    assert res.converged and res.iterations == g["iterations"]
    assert np.array_equal(ex, np.asarray(g["exemplars"]))
    assert np.array_equal(lab, np.asarray(g["labels"], dtype=np.int32))
    assert abs(res.netsim - g["netsim"]) <= n * 1e-6 * g["range"]


def test_matrix_free_errors():
    n = 6000
    X = torch.from_numpy(synth.gaussian_mixture(n=n, d=8, k=5, seed=3).X).cuda()
    with pytest.raises(RuntimeError, match="R and A"):
        apx.ap_solve_mf(X, flags=apx.APX_RAW_LABELS)
    with pytest.raises(RuntimeError, match="R and A"):
        apx.ap_solve_mf(X, flags=apx.APX_MSG_THRESHOLD)
    with pytest.raises(RuntimeError, match="panel_rows"):
        apx.ap_solve_mf(X, panel_rows=16)
    Xs = torch.zeros((70000, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError, match="implicit passes"):
        apx.ap_solve_mf(Xs)


def test_matrix_free_caller_workspace():
    """apx_workspace_size(APX_OP_SOLVE_MF) covers the call: with a caller
    workspace of exactly that size it allocates nothing and gives the same
    result; one page less is APX_ENOMEM."""
    n, seed, rows = 6000, 6203, 1000
    X = torch.from_numpy(synth.gaussian_mixture(n=n, d=16, k=20, seed=seed).X).cuda()
    idx0, res0, _ = apx.ap_solve_mf(X, noise_seed=seed, damping=0.9, max_iter=1000, panel_rows=rows)
    need = apx.apx_workspace_size(apx.APX_OP_SOLVE_MF, n, count=rows)
    assert need > 0 and apx.apx_workspace_size(apx.APX_OP_SOLVE_MF, n, count=16) == 0
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    try:
        apx.apx_set_workspace(buf)
        idx1, res1, _ = apx.ap_solve_mf(X, noise_seed=seed, damping=0.9, max_iter=1000, panel_rows=rows)
        assert torch.equal(idx0, idx1) and res1.iterations == res0.iterations and res1.netsim == res0.netsim
        apx.apx_set_workspace(buf[: need - 4096])
        with pytest.raises(apx.ApxError) as ei:
            apx.ap_solve_mf(X, noise_seed=seed, damping=0.9, max_iter=1000, panel_rows=rows)
        assert ei.value.status == apx.APX_ENOMEM
    finally:
        apx.apx_set_workspace(None)
