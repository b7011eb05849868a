"""ap_solve with the iteration loop replayed as a captured HIP graph against
the same solve with every kernel launched from the host: bit-identical
messages, labels and results, over several replays of one cached graph with
other (eager) GPU work between them, with an odd poll interval, and a fixed
iteration count that ends inside a chunk; the timed path (host launches with
events) gives the same results."""
import time

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


def dev(S64):
    return apx.to_matrix(torch.from_numpy(np.ascontiguousarray(S64, dtype=np.float32)))


def solve(S, lam, max_iter, conv_iter, check_every=0):
    n = S.shape[0]
    R, A = apx.empty_matrix(n), apx.empty_matrix(n)
    idx, res = apx.ap_solve(S, R, A, lam, max_iter, conv_iter, check_every=check_every)
    torch.cuda.synchronize()
    return R.clone(), A.clone(), idx.clone(), res


def same(a, b):
    (Ra, Aa, ia, ra), (Rb, Ab, ib, rb) = a, b
    return (torch.equal(Ra, Rb) and torch.equal(Aa, Ab) and torch.equal(ia, ib)
            and ra.iterations == rb.iterations and ra.converged == rb.converged
            and ra.n_exemplars == rb.n_exemplars and ra.netsim == rb.netsim)


@pytest.fixture(autouse=True)
def graphs_back_on():
    yield
    apx.apx_set_graphs(True)


@pytest.mark.parametrize("n,lam,max_iter,conv_iter,check_every", [
    (1000, 0.9, 2000, 15, 0),
    (4097, 0.9, 2000, 15, 5),
    (3000, 0.9, 37, 0, 0),
])
def test_graph_replays_match_eager(n, lam, max_iter, conv_iter, check_every):
    say(f"graphs vs eager n={n} max_iter={max_iter} conv_iter={conv_iter} check_every={check_every}")
    pts = synth.gaussian_mixture(n=n, d=8, k=12, seed=500 + n)
    S = dev(oracle.prepare(oracle.similarity(pts.X), "median", seed=500 + n).S)
    apx.apx_set_graphs(False)
    ref = solve(S, lam, max_iter, conv_iter, check_every)
    apx.apx_set_graphs(True)
    other = dev(np.random.default_rng(1).normal(size=(300, 300)))
    for rep in range(3):
        got = solve(S, lam, max_iter, conv_iter, check_every)
        assert same(got, ref), f"replay {rep}"
        # eager work between replays on the same stream
        R2, A2 = apx.empty_matrix(300, fill=0.0), apx.empty_matrix(300, fill=0.0)
        apx.ap_iterate(other, R2, A2, 0.5, 3)
        _ = (other * 2.0).sum().item()


def test_timing_mode_matches_graph_mode():
    """Kernel timing launches the passes from the host; results do not change."""
    n = 2000
    say(f"graphs against the timed (host-launched) path n={n}")
    pts = synth.gaussian_mixture(n=n, d=8, k=12, seed=77)
    S = dev(oracle.prepare(oracle.similarity(pts.X), "median", seed=77).S)
    ref = solve(S, 0.9, 2000, 15)
    apx.apx_profile(True)
    apx.apx_profile_read()
    got = solve(S, 0.9, 2000, 15)
    launches, ms = apx.apx_profile_read()
    apx.apx_profile(False)
    assert same(got, ref)
    assert launches == got[3].iterations and ms > 0


def test_graph_speed_on_small_problem():
    n = 1000
    pts = synth.gaussian_2d(n=n, k=10, seed=1001)
    S = dev(oracle.prepare(oracle.similarity(pts.X), "median", seed=1001).S)
    out = {}
    for g in (False, True):
        apx.apx_set_graphs(g)
        solve(S, 0.9, 400, 0)
        t0 = time.perf_counter()
        solve(S, 0.9, 400, 0)
        out[g] = (time.perf_counter() - t0) * 1e3
    say(f"n={n}, 400 iterations: eager {out[False]:.2f} ms, graph {out[True]:.2f} ms")
