"""Autotuner: every row-pass workgroup size and variant it may pick gives
bit-identical results to the default plan (same row -> workgroup map, same
sums in the same order); measured choices are valid and survive a JSON round
trip; a file tuned for another device is rejected."""
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


def say(msg):
    print(msg, flush=True)


@pytest.fixture(autouse=True)
def clean_table():
    apx.apx_tune_clear()
    yield
    apx.apx_tune_clear()


def solve(S, check_every=0):
    n = S.shape[0]
    R, A = apx.empty_matrix(n), apx.empty_matrix(n)
    idx, res = apx.ap_solve(S, R, A, 0.9, 2000, 15, check_every=check_every)
    torch.cuda.synchronize()
    return R, A, idx, res


@pytest.mark.parametrize("n", [1000, 3000, 6000, 12000])
def test_every_variant_is_bit_identical(n):
    pts = synth.gaussian_mixture(n=n, d=8, k=12, seed=900 + n)
    S = apx.to_matrix(torch.from_numpy(
        oracle.prepare(oracle.similarity(pts.X), "median", seed=900 + n).S.astype(np.float32)))
    R0, A0, i0, r0 = solve(S)
    tried = 0
    for threads in (256, 512, 1024):
        for lds in (True, False):
            try:
                apx.apx_tune_set(n, threads, lds, 6)
            except apx.ApxError:
                continue            # no row pass with this workgroup size for n
            got = apx.apx_tune_get(n)
            say(f"n={n}: threads {threads} lds {got['lds']}")
            R, A, idx, res = solve(S)
            assert torch.equal(R, R0) and torch.equal(A, A0) and torch.equal(idx, i0)
            assert (res.iterations, res.netsim) == (r0.iterations, r0.netsim)
            tried += 1
    assert tried >= 2


def test_autotune_choice_and_json_round_trip(tmp_path):
    picks = {}
    for n in (1000, 6000, 20000):
        e = apx.apx_autotune(n)
        say(f"autotune n={n}: {e}")
        assert e["threads"] in (256, 512, 1024)
        assert e["check_every"] >= 2 and e["check_every"] % 2 == 0
        assert e["ms_per_iter"] > 0
        picks[n] = e
    path = str(tmp_path / "tune.json")
    apx.apx_tune_save(path)
    doc = json.load(open(path))
    assert len(doc["entries"]) == 3
    apx.apx_tune_clear()
    assert apx.apx_tune_get(6000)["threads"] == 0
    apx.apx_tune_load(path)
    for n, e in picks.items():
        got = apx.apx_tune_get(n)
        assert abs(got.pop("ms_per_iter") - e.pop("ms_per_iter")) <= 1e-6   # printed to 1e-6 ms
        assert got == e


def test_foreign_or_malformed_file_is_rejected(tmp_path):
    apx.apx_autotune(3000)
    path = str(tmp_path / "t.json")
    apx.apx_tune_save(path)
    doc = open(path).read()
    other = tmp_path / "other.json"
    cus = json.loads(doc)["compute_units"]
    other.write_text(doc.replace(f'"compute_units": {cus}', f'"compute_units": {cus + 1}'))
    with pytest.raises(apx.ApxError):
        apx.apx_tune_load(str(other))
    bad = tmp_path / "bad.json"
    bad.write_text(doc.replace('"threads": ', '"threads": 7'))
    with pytest.raises(apx.ApxError):
        apx.apx_tune_load(str(bad))
    assert os.path.exists(path)


def test_autotuned_solve_matches_default():
    n = 4097
    pts = synth.gaussian_mixture(n=n, d=8, k=12, seed=4097)
    S = apx.to_matrix(torch.from_numpy(
        oracle.prepare(oracle.similarity(pts.X), "median", seed=4097).S.astype(np.float32)))
    R0, A0, i0, r0 = solve(S)
    apx.apx_set_autotune(True)
    try:
        R, A, idx, res = solve(S)
    finally:
        apx.apx_set_autotune(False)
    say(f"autotuned entry n={n}: {apx.apx_tune_get(n)}")
    assert torch.equal(R, R0) and torch.equal(A, A0) and torch.equal(idx, i0)
