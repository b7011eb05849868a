"""The evaluation protocols on the GPU: Table 2's PAP part-count sweep with
the paper's contiguous split (every k against the oracle's PAP with the same
split), the size sweep of the 2-D sets (a small instance of it against the
oracle), and landmark re-seeding (kept exemplars are landmarks again)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0910_1650_amd as apx  # noqa: E402
from paper_0910_1650_amd import experiments as ex  # noqa: E402


def shared(pts, seed):
    S64 = oracle.prepare(oracle.similarity(pts.X), "median", seed=seed).S
    S32 = S64.astype(np.float32)
    return apx.to_matrix(torch.from_numpy(S32)), S32.astype(np.float64)


def test_pap_k_sweep_matches_oracle():
    pts = synth.subspaces(n=3000, d=20, n_sub=8, dim=3, seed=3051)
    S, S64 = shared(pts, 3051)
    print("pap k sweep n=3000", flush=True)
    rows = ex.pap_k_sweep(S, ks=(2, 4, 8, 16), truth=pts.labels)
    ref = oracle.ap(S64, 0.9, 2000, 15)
    assert rows[0]["method"] == "AP" and rows[0]["iterations"] == ref.iterations
    assert rows[0]["classes"] == ref.n_exemplars
    for row in rows[1:]:
        r = oracle.pap(S64, row["k"], lam=0.9, max_iter=2000, conv_iter=15)
        assert row["iterations"] == r.full.iterations, row
        assert row["classes"] == r.full.n_exemplars, row
        assert row["part_iterations"] == max(s.iterations for s in r.subs), row
        tar, far = ex.association_rates(pts.labels, r.full.idx)
        assert row["TAR"] == tar and row["FAR"] == far


def test_size_sweep_small():
    print("size sweep", flush=True)
    out = ex.size_sweep(sizes=(200, 500), runs=2)
    assert [o["n"] for o in out] == [200, 500] and all(o["runs"] == 2 for o in out)
    assert all(o["ap_iterations"] > 0 and o["pap_iterations"] > 0 for o in out)


def test_lap_reseed_keeps_exemplars():
    pts = synth.gaussian_2d(n=8000, k=8, seed=4301)
    X = torch.from_numpy(pts.X).cuda()
    print("lap reseed", flush=True)
    rounds = ex.lap_reseed(X, 400, seed=4301, rounds=3)
    assert [r["round"] for r in rounds] == [0, 1, 2]
    assert rounds[0]["kept"] == 0 and rounds[1]["kept"] == rounds[0]["n_exemplars"]
    assert all(np.isfinite(r["netsim"]) for r in rounds)
    # the re-seeded landmark set holds the previous exemplars
    M0 = apx.apx_lap_landmarks(8000, 400, None, 4301)
    _, _, e0 = apx.lap_solve(X, 400, landmarks=M0, seed=4301)
    M1 = apx.apx_lap_landmarks(8000, 400, e0, 4302)
    assert np.all(np.isin(e0, M1))
