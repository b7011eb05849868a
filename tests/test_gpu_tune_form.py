"""Tuned message forms of a cold ap_solve (explicit; implicit R; implicit R
and A): each form, set by hand, runs as recorded by the solve and reaches
the oracle's stop iteration, exemplar set and labels (Algorithm 1, damping
0.9, stop after 15 unchanged sets); the timed pick is one of the three and
survives a JSON round trip."""
import json

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0910_1650_amd as apx  # noqa: E402

N, SEED = 6000, 6161


@pytest.fixture(autouse=True)
def clean_table():
    apx.apx_tune_clear()
    yield
    apx.apx_tune_clear()


@pytest.fixture(scope="module")
def case():
    pts = synth.gaussian_mixture(n=N, d=16, k=20, seed=SEED)
    S32 = oracle.prepare(oracle.similarity(pts.X), "median", seed=SEED).S.astype(np.float32)
    ref = oracle.ap(S32.astype(np.float64), 0.9, 2000, 15)
    return S32, ref


@pytest.mark.parametrize("form", [apx.APX_FORM_EXPLICIT, apx.APX_FORM_IMPLICIT_R, apx.APX_FORM_IMPLICIT_RA])
def test_each_form_matches_oracle(case, form):
    S32, ref = case
    apx.apx_tune_set_form(N, form)
    assert apx.apx_tune_get_form(N)["form"] == form
    Sd = apx.to_matrix(torch.from_numpy(S32))
    R, A = apx.empty_matrix(N), apx.empty_matrix(N)
    idx, res = apx.ap_solve(Sd, R, A, 0.9, 2000, 15)
    imp, exp, ia = apx.apx_last_solve_info()
    print(f"form {form}: iterations {res.iterations} (implicit R {imp}, explicit {exp}, implicit A {ia})",
          flush=True)
    T = res.iterations
    expect = {apx.APX_FORM_EXPLICIT: (0, T, 0), apx.APX_FORM_IMPLICIT_R: (T, 0, 0),
              apx.APX_FORM_IMPLICIT_RA: (T, 0, T)}[form]
    assert (imp, exp, ia) == expect
    assert res.converged and ref.converged and T == ref.iterations
    assert np.array_equal(idx.cpu().numpy(), ref.idx)
    rng = float(S32.max()) - float(S32.min())
    assert abs(res.netsim - ref.netsim) <= N * 1e-6 * rng


def test_timed_pick_and_round_trip(tmp_path):
    got = apx.apx_autotune_form(N)
    print(f"form timing n={N}: {got}", flush=True)
    assert got["form"] in (apx.APX_FORM_EXPLICIT, apx.APX_FORM_IMPLICIT_R, apx.APX_FORM_IMPLICIT_RA)
    assert all(m > 0 for m in got["ms"])
    assert got["ms"][got["form"] - 1] == min(got["ms"])
    path = str(tmp_path / "tune.json")
    apx.apx_tune_save(path)
    doc = json.load(open(path))
    assert doc["entries"][0]["form"] == got["form"]
    apx.apx_tune_clear()
    assert apx.apx_tune_get_form(N)["form"] == apx.APX_FORM_DEFAULT
    apx.apx_tune_load(path)
    back = apx.apx_tune_get_form(N)
    assert back["form"] == got["form"]
    assert np.allclose(back["ms"], got["ms"], atol=1e-6)
