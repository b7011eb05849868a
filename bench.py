"""Benchmark: dense affinity propagation at N=20000 on one MI355X.

A step is one pass of the dense-AP hot path over the resident 64-D Gaussian
mixture (N=20000, 50 components): similarity build on FP32 matrix cores,
median preference with tie-break noise, AP (damping 0.9, stop after 15
unchanged exemplar sets, at most 2000 iterations) and the final labels and
net similarity.  Inputs are generated once and are resident in HBM before
the timed region starts.

After the timed steps (outside the timed region) the same resident S is
solved once each from a cold start, by PAP (Algorithm 2, 8 random uneven
parts) and from the learned warm start, reporting wall time to the stop rule
and whether the exemplar set is the FP64 oracle's ("time_to_exemplars").

Prints one JSON line (see the fields below).  `value` is the measured rate
of AP iterations over the whole step (similarity, preference, AP to the
stop rule, finalize): iterations per second.  `iteration_path` reports
which form of the iteration ran and the bytes that form moves per element
(cold start at this size: implicit R and A, an iteration reads S, 4 bytes
per element), with the executed GB/s of the step; the dense form's rate
(20 bytes per element and iteration: read S, R, A; write A, R) is reported
beside it, labelled as an equivalent, never as the value.  `roofline`
measures the dominant kernel against the HBM peak on its own bytes, from
HIP events on the solver's stream during the timed steps (the passes are
then launched one by one; `ms_per_step_graph` times the same step with the
iteration loop replayed as a HIP graph, outside the timed region).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N, D, K_MIX, SEED = 20000, 64, 50, 2001
LAMBDA, MAX_ITER, CONV_ITER = 0.9, 2000, 15
BYTES_EXPLICIT = 20               # explicit R and A: read S, R, A; write A, R (FP32)
BYTES_IMPLICIT = 12               # implicit R: read S, A; write A (FP32)
BYTES_IMPLICIT_A = 4              # implicit R and A: read S (FP32)
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=N)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=6)
    ap.add_argument("--no-warm-compare", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (PAP at N=40000, the 512-instance batch, LAP)")
    ap.add_argument("--counter-run", action="store_true",
                    help="sequence for rocprofv3 --pmc runs: one ap_solve at N as a step runs it "
                         "(to the stop rule), then a plain 1.6 GB device copy (the calibration "
                         "kernel); prints no JSON")
    return ap.parse_args()


def cpu_baseline(pts, n_iter: int) -> dict:
    """The FP64 oracle on the host: n_iter AP iterations on the same matrix."""
    import oracle
    S = oracle.prepare(oracle.similarity(pts.X), "median", seed=SEED).S
    oracle.ap(S, LAMBDA, 1, 0)                      # touch pages once
    t0 = time.perf_counter()
    oracle.ap(S, LAMBDA, n_iter, 0, finalize_labels=False)
    dt = time.perf_counter() - t0
    n = S.shape[0]
    it_s = n_iter / dt
    return {"value": round(it_s, 4), "unit": "iter/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "GBps": round(it_s * BYTES_EXPLICIT * n * n / 1e9, 3),
            "sample": f"{n_iter} FP64 oracle iterations of dense AP on the same N={n} matrix "
                      f"(similarity/preference setup untimed); GBps counts the "
                      f"{BYTES_EXPLICIT} B per element and iteration of the explicit form "
                      f"the oracle runs"}


GOLDEN = os.path.join(ROOT, "tests", "golden", "c2_n20000_d64_k50_seed2001.json")
CALIB_ELEMS = 400_000_000       # 1.6 GB FP32 copy: the counter calibration kernel

# HBM bytes moved per launch by the full row pass of the form that runs at
# N=20000 (averaged over the launches of one solve), from rocprofv3
# FETCH_SIZE and WRITE_SIZE runs of `bench.py --counter-run`, each scaled by
# what the same counter reads for the 1.6 GB copy (profiles/
# row_pass_n20000_hbm_counters.md).  Valid only for that form and the
# row-pass source with this SHA-256; otherwise the benchmark reports traffic
# as null.
ROW_PASS_SRC = "paper_0910_1650_amd/csrc/ap_iter.hip"
ROW_PASS_TRAFFIC = {"read": 1688642971, "write": 45899219, "path": "implicit_RA",
                    "sha256": "26823068bb96016525d0e0a14b2d86c187fcaf236554ec60c5d87ea3c66d543e"}
PAP_K = 8


def time_to_exemplars(apx, S, n, pts_seed):
    """Wall time from S resident in HBM to the stop rule for cold start, PAP
    (k = 8 random uneven parts of consecutive indices) and the learned warm
    start (features, network, column-structured A_0, cold fallback).  A run counts only if its exemplar set equals the
    FP64 oracle's (stored by tests/golden/make_oracle_exemplars.py) and its
    net similarity is within n * 1e-6 * (max S - min S) of the oracle's."""
    import numpy as np
    import torch

    from paper_0910_1650_amd import warmstart as ws

    ref = None
    if n == N and os.path.exists(GOLDEN):
        with open(GOLDEN) as f:
            ref = json.load(f)
    theta = ws.load_weights()
    out = {}
    runs = {
        "cold": lambda: ws.solve_cold(S, LAMBDA, MAX_ITER, CONV_ITER),
        "pap_k8": lambda: ws.solve_pap(S, PAP_K, pts_seed, LAMBDA, MAX_ITER, CONV_ITER),
        "learned": lambda: ws.solve_warm(S, theta, LAMBDA, MAX_ITER, CONV_ITER),
    }
    for name, fn in runs.items():
        r = fn()
        idx, res, ms = r[0], r[1], r[2]
        iters = r[3] if name == "learned" else res.iterations
        E = ws.exemplar_set(idx)
        rec = {"ms": round(ms, 2), "iterations": iters, "n_exemplars": res.n_exemplars,
               "netsim": res.netsim}
        if name == "pap_k8":
            rec["sub_iterations_max"] = max(x.iterations for x in r[3])
        if name == "learned":
            rec["fallback_to_cold"] = r[4]
        if ref is not None:
            same = bool(np.array_equal(E, np.asarray(ref["exemplars"])))
            close = abs(res.netsim - ref["netsim"]) <= n * 1e-6 * ref["range"]
            rec["same_exemplars_as_oracle"] = same
            rec["netsim_ratio_to_oracle"] = res.netsim / ref["netsim"]
            rec["time_to_oracle_exemplars_ms"] = round(ms, 2) if (same and close) else None
        out[name] = rec
        torch.cuda.synchronize()
    if ref is not None:
        out["oracle"] = {"iterations": ref["iterations"], "n_exemplars": ref["n_exemplars"],
                         "netsim": ref["netsim"]}
    return out


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, (time.perf_counter() - t0) * 1e3


def workload_extras(apx) -> dict:
    """The other workloads of the path, each timed once outside the timed
    region (inputs resident in HBM before each clock starts):

    * pap_c3: Algorithm 2 on 40000 points on a union of 20 random 5-D
      subspaces of R^100, 8 random parts of 3000-7000 points; the parts'
      sub-problems alone (one persistent batched launch) with their HBM rate
      (20 B per element and iteration of the explicit form those passes run,
      summed over the parts' own iteration counts), the whole pap_solve
      (parts of consecutive indices: Step 4 keeps A implicit; and the same
      sizes over a random permutation of the indices: Step 4 with implicit R
      only), and cold-start AP on the same S.
    * batch_512: 512 independent 2-D mixtures, n in [100, 2000], 2-20
      components, damping 0.5, at most 200 iterations: one ap_solve_batched
      call; instance-iterations per second and the same HBM rate.
    * lap_c4: Algorithm 3 (Steps 1-2) on 200000 points in 128-D, 10000
      landmarks: the landmark similarity and AP, then the assignment of every
      point; the whole lap_solve and the assignment's FP32 rate.
    * matrix_free_c2: ap_solve_mf on the benchmark's points (S rebuilt per
      iteration, no n x n buffer), against the oracle's exemplar set.
    * long_rows_n100000: ten explicit iterations (ap_iterate) at n = 100000,
      where every row is streamed twice per pass, with their HBM rate."""
    import numpy as np
    import torch

    import synth
    out = {}
    # ---- PAP, N = 40000
    n, seed = 40000, 3001
    pts = synth.subspaces(n=n, d=100, n_sub=20, dim=5, noise=0.05, seed=seed)
    X = torch.from_numpy(pts.X).cuda()
    S, _ = apx.ap_similarity(X, pref="median", noise_seed=seed, noise_rel=1e-12)
    # the points are drawn i.i.d., so parts of consecutive indices with random
    # sizes are a uniformly random partition; the same sizes with a random
    # permutation of the indices run the general path (no block structure
    # for Step 4)
    perm, offsets = synth.random_partition(n, 8, 3000, 7000, seed=seed)
    sizes = np.diff(offsets)
    blocks = []
    for j in range(8):
        a, b = int(offsets[j]), int(offsets[j + 1])
        Sj = apx.empty_matrix(int(sizes[j]))
        Sj.copy_(S[a:b, a:b])
        blocks.append(Sj)
    (idxs, subres), ms_sub = _timed(lambda: apx.ap_solve_batched(blocks, damping=0.9, max_iter=2000,
                                                                    conv_iter=15))
    sub_bytes = sum(20 * int(sizes[j]) ** 2 * subres[j].iterations for j in range(8))
    del blocks, idxs
    R, A = apx.empty_matrix(n), apx.empty_matrix(n)
    (idx, res, subs), ms_pap = _timed(lambda: apx.pap_solve(S, R, A, 8, None, offsets, damping=0.9,
                                                            max_iter=2000, conv_iter=15))
    step4_info = apx.apx_last_solve_info()
    (idx_p, res_p, subs_p), ms_pap_perm = _timed(lambda: apx.pap_solve(S, R, A, 8, perm, offsets, damping=0.9,
                                                                       max_iter=2000, conv_iter=15))
    del idx_p
    (idx_c, res_c), ms_cold = _timed(lambda: apx.ap_solve(S, R, A, 0.9, 2000, 15))
    sub_gbs = sub_bytes / (ms_sub * 1e-3) / 1e9
    out["pap_c3"] = {
        "workload": "40000 points, union of 20 random 5-D subspaces of R^100 (noise 0.05), "
                    "8 random parts of 3000-7000 points (consecutive indices of i.i.d. points), damping 0.9",
        "part_sizes": [int(x) for x in sizes],
        "parts_ms": round(ms_sub, 2), "parts_iterations": [r.iterations for r in subres],
        "parts_GBps": round(sub_gbs, 1), "parts_frac": round(sub_gbs / HBM_PEAK_GBS, 4),
        "parts_bytes_basis": "20 B per element and iteration (explicit form), each part's own iteration count",
        "pap_ms": round(ms_pap, 2), "pap_step4_iterations": res.iterations,
        "pap_step4_form": {"implicit_R_iterations": step4_info[0], "explicit_iterations": step4_info[1],
                           "implicit_A_iterations": step4_info[2]},
        "pap_netsim": res.netsim, "pap_n_exemplars": res.n_exemplars,
        "pap_permuted_parts_ms": round(ms_pap_perm, 2), "pap_permuted_step4_iterations": res_p.iterations,
        "cold_ms": round(ms_cold, 2), "cold_iterations": res_c.iterations,
        "cold_netsim": res_c.netsim, "cold_n_exemplars": res_c.n_exemplars,
        "same_exemplars": bool(torch.equal(idx, idx_c)),
    }
    del S, R, A, X, idx, idx_c
    torch.cuda.empty_cache()
    print("extras: pap done", file=sys.stderr, flush=True)

    # ---- 512 independent instances
    insts = synth.batch_instances(count=512, seed0=3101)
    Ss = []
    for p_ in insts:
        Xj = torch.from_numpy(p_.X).cuda()
        Sj, _ = apx.ap_similarity(Xj, pref="median", noise_seed=p_.seed, noise_rel=1e-12)
        Ss.append(Sj)
    Rs = [apx.empty_matrix(S_.shape[0]) for S_ in Ss]
    As = [apx.empty_matrix(S_.shape[0]) for S_ in Ss]
    apx.ap_solve_batched(Ss, Rs, As, damping=0.5, max_iter=200, conv_iter=15)      # warm-up
    (idxs, rs), ms_b = _timed(lambda: apx.ap_solve_batched(Ss, Rs, As, damping=0.5, max_iter=200,
                                                           conv_iter=15))
    it_sum = sum(r.iterations for r in rs)
    b_bytes = sum(20 * S_.shape[0] ** 2 * r.iterations for S_, r in zip(Ss, rs))
    b_gbs = b_bytes / (ms_b * 1e-3) / 1e9
    out["batch_512"] = {
        "workload": "512 independent 2-D Gaussian mixtures, n in [100, 2000], 2-20 components, "
                    "median preference, damping 0.5, at most 200 iterations, one launch",
        "sum_n2": int(sum(S_.shape[0] ** 2 for S_ in Ss)),
        "ms": round(ms_b, 2), "instance_iterations": it_sum,
        "instance_iterations_per_s": round(it_sum / (ms_b * 1e-3), 1),
        "converged": int(sum(r.converged for r in rs)),
        "GBps": round(b_gbs, 1), "frac": round(b_gbs / HBM_PEAK_GBS, 4),
        "bytes_basis": "20 B per element and iteration (explicit form), each instance's own count",
    }
    del Ss, Rs, As, idxs
    torch.cuda.empty_cache()
    print("extras: batch done", file=sys.stderr, flush=True)

    # ---- LAP, N = 200000
    n, d, L, seed = 200000, 128, 10000, 4001
    pts = synth.image_features(n=n, d=d, k=20, seed=seed)
    M = synth.landmarks(n, L, seed)
    X = torch.from_numpy(pts.X).cuda()
    apx.lap_solve(X, L, landmarks=M, seed=seed, damping=0.9)                        # warm-up
    (idx, res, ex), ms_lap = _timed(lambda: apx.lap_solve(X, L, landmarks=M, seed=seed, damping=0.9))
    XM = X[torch.from_numpy(M).cuda()].contiguous()

    def landmark_part():
        SL, _ = apx.ap_similarity(XM, pref="median", noise_seed=seed, noise_rel=1e-12)
        RL, AL = apx.empty_matrix(L), apx.empty_matrix(L)
        return apx.ap_solve(SL, RL, AL, 0.9, 2000, 15)
    landmark_part()
    (_, rl), ms_land = _timed(landmark_part)
    ms_assign = max(ms_lap - ms_land, 1e-3)
    flops = 2.0 * n * res.n_exemplars * d
    out["lap_c4"] = {
        "workload": "200000 points in 128-D (20-component mixture, clipped to [-3,3]), 10000 landmarks, "
                    "damping 0.9",
        "ms": round(ms_lap, 2), "landmark_ms": round(ms_land, 2), "landmark_iterations": rl.iterations,
        "n_exemplars": res.n_exemplars, "assign_ms": round(ms_assign, 2),
        "assign_TFLOPs": round(flops / (ms_assign * 1e-3) / 1e12, 2),
        "assign_frac_fp32": round(flops / (ms_assign * 1e-3) / 157.3e12, 4),
        "assign_basis": "2 n |E| d FP32 flops of the distances over the assignment time "
                        "(lap_solve minus the landmark similarity and AP)",
    }
    (idxf, rf, exf, stf), ms_full = _timed(lambda: apx.lap_full_solve(X, L, m0=20000, landmarks=M, seed=seed,
                                                                       damping=0.9))
    out["lap_full_c4"] = {
        "workload": "the same 200000 points and landmarks, Algorithm 3 Steps 1-4 with m0 = 20000",
        "ms": round(ms_full, 2), "n_exemplars": rf.n_exemplars, "netsim": rf.netsim,
        "netsim_steps_1_2": res.netsim, "stats": stf,
    }
    from paper_0910_1650_amd import experiments as ex
    out["lap_reseed_c4"] = {
        "workload": "the same points: LAP (Steps 1-2), then twice more with the landmarks re-seeded "
                    "from the previous run's exemplars plus a fresh uniform sample",
        "rounds": ex.lap_reseed(X, L, seed=seed, rounds=3),
    }
    print("extras: lap done", file=sys.stderr, flush=True)
    del X
    torch.cuda.empty_cache()
    # Table 2's protocol and the 2-D size sweep
    out["size_sweep_2d"] = {
        "workload": "2-D 10-component mixtures, N = 100..3000 step 100, 10 seeded runs each, "
                    "AP against PAP with k = 4 (contiguous split), damping 0.9",
        "rows": ex.size_sweep(),
    }
    print("extras: size sweep done", file=sys.stderr, flush=True)
    # matrix-free AP on the benchmark's points: S rebuilt per iteration
    import synth
    pts = synth.gaussian_mixture(n=N, d=D, k=K_MIX, seed=SEED)
    X = torch.from_numpy(pts.X).cuda()
    (idx, res, _), ms = _timed(lambda: apx.ap_solve_mf(X, pref="median", noise_seed=SEED, noise_rel=1e-12,
                                                       damping=LAMBDA, max_iter=MAX_ITER, conv_iter=CONV_ITER))
    rec = {
        "workload": f"ap_solve_mf on the benchmark's {N} points ({D}-D, {K_MIX}-component mixture): "
                    "S rebuilt from X one row panel at a time in every iteration (two panels of at "
                    "most 1 GiB, no n x n buffer), median preference by three panel sweeps, implicit "
                    "passes; wall time from X resident to labels",
        "ms": round(ms, 2), "iterations": res.iterations, "ms_per_iteration": round(ms / max(res.iterations, 1), 3),
        "n_exemplars": res.n_exemplars, "netsim": res.netsim,
        "s_bytes_not_allocated": 4 * N * N,
    }
    if os.path.exists(GOLDEN):
        with open(GOLDEN) as f:
            ref = json.load(f)
        lab = idx.cpu().numpy()
        rec["same_exemplars_as_oracle"] = bool(np.array_equal(np.flatnonzero(lab == np.arange(N)),
                                                              np.asarray(ref["exemplars"])))
    out["matrix_free_c2"] = rec
    del X
    torch.cuda.empty_cache()
    print("extras: matrix-free done", file=sys.stderr, flush=True)

    # explicit passes on rows too long to hold in registers: two sweeps per row
    n, seed, iters = 100000, 3201, 10
    pts = synth.gaussian_mixture(n=n, d=8, k=30, seed=seed)
    X = torch.from_numpy(pts.X).cuda()
    S, _ = apx.ap_similarity(X, pref="median", noise_seed=seed, noise_rel=1e-12)
    del X
    R, A = apx.empty_matrix(n, fill=0.0), apx.empty_matrix(n, fill=0.0)
    apx.ap_iterate(S, R, A, LAMBDA, 2)
    _, ms = _timed(lambda: apx.ap_iterate(S, R, A, LAMBDA, iters))
    gbs = 20.0 * n * n * iters / (ms * 1e-3) / 1e9
    out["long_rows_n100000"] = {
        "workload": f"ap_iterate on {n} points (8-D, 30-component mixture), damping {LAMBDA}: "
                    f"{iters} iterations of the explicit passes, each row streamed twice",
        "ms_per_iteration": round(ms / iters, 3),
        "GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
        "bytes_basis": "20 B per element and iteration (S, R_t, A_{t-1} read, R_{t+1}, A_t written); "
                       "the pass moves 28 B (S and R_t read twice)",
    }
    del S, R, A
    torch.cuda.empty_cache()
    print("extras: long rows done", file=sys.stderr, flush=True)
    return out


def counter_run(n: int) -> None:
    import torch

    import paper_0910_1650_amd as apx
    import synth
    pts = synth.gaussian_mixture(n=n, d=D, k=K_MIX, seed=SEED)
    X = torch.from_numpy(pts.X).cuda()
    S, _ = apx.ap_similarity(X, pref="median", noise_seed=SEED, noise_rel=1e-12)
    R, A = apx.empty_matrix(n), apx.empty_matrix(n)
    apx.ap_solve(S, R, A, LAMBDA, MAX_ITER, CONV_ITER)    # the solve of one benchmark step
    torch.cuda.synchronize()
    src = torch.ones(CALIB_ELEMS, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"counter run done: n={n}, copy of {CALIB_ELEMS * 4} bytes x2", file=sys.stderr, flush=True)


def source_sha256(rel: str) -> str:
    import hashlib
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def hbm_reference(torch, S, n: int, reps: int = 5) -> dict:
    """Rates of torch's reduction (reads the matrix) and copy (reads and
    writes it) over the resident n x n FP32 matrix: a reference for what a
    library streaming kernel reaches on this part, not the peak."""
    view = S[:, :n]
    dst = torch.empty((n, n), dtype=view.dtype, device=view.device)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    dst.copy_(view)
    torch.sum(dst)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        dst.copy_(view)
    ev[1].record()
    for _ in range(reps):
        torch.sum(dst)
    ev[2].record()
    torch.cuda.synchronize()
    nbytes = 4 * n * n
    copy_ms = ev[0].elapsed_time(ev[1]) / reps
    sum_ms = ev[1].elapsed_time(ev[2]) / reps
    del dst
    return {"read_GBps": round(nbytes / sum_ms / 1e6, 1),
            "read_kernel": "torch.sum over a contiguous copy of the matrix",
            "copy_GBps": round(2 * nbytes / copy_ms / 1e6, 1),
            "copy_kernel": "torch copy_ of the matrix (bytes read + written)",
            "note": "library streaming kernels on the same buffer, for context; the roofline's peak "
                    "stays the published 8 TB/s"}


def main():
    args = parse()
    if args.counter_run:
        counter_run(args.n)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (a sharded run "
              "would split the rows of S, R and A and all-reduce the column sums each "
              "iteration)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_0910_1650_amd as apx
    import synth

    n = args.n
    torch.cuda.set_device(0)
    pts = synth.gaussian_mixture(n=n, d=D, k=K_MIX, seed=SEED)
    X = torch.from_numpy(pts.X).cuda()
    S = apx.empty_matrix(n)
    R = apx.empty_matrix(n)
    A = apx.empty_matrix(n)
    idx = torch.empty(n, dtype=torch.int32, device="cuda")

    def step():
        apx.ap_similarity(X, S, pref="median", noise_seed=SEED, noise_rel=1e-12)
        return apx.ap_solve(S, R, A, LAMBDA, MAX_ITER, CONV_ITER, idx=idx)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    apx.apx_profile(True)
    apx.apx_profile_read()
    iters = 0
    alg_bytes = 0
    imp_iters = exp_iters = ia_iters = 0
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        _, res = step()
        iters += res.iterations
        ni, ne, na = apx.apx_last_solve_info()
        imp_iters += ni
        exp_iters += ne
        ia_iters += na
        results.append(res)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, pass_ms = apx.apx_profile_read()
    apx.apx_profile(False)
    print(f"timed {args.steps} steps in {dt:.3f}s", file=sys.stderr, flush=True)

    # the same step with graph replay (the library default), untimed above
    t1 = time.perf_counter()
    for _ in range(max(1, args.steps)):
        step()
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t1) * 1e3 / max(1, args.steps)

    # similarity build on its own (events on the current stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    apx.ap_similarity(X, S, pref="median", noise_seed=SEED, noise_rel=1e-12)
    e1.record()
    torch.cuda.synchronize()
    sim_ms = e0.elapsed_time(e1)

    # context for the roofline (outside the timed region): what torch's own
    # streaming kernels reach over the same n x n FP32 matrix on this part
    hbm_ref = hbm_reference(torch, S, n)

    elems = n * n
    ms_step = dt * 1e3 / args.steps
    ir_iters = imp_iters - ia_iters              # implicit R with explicit A
    exec_bytes = (ia_iters * BYTES_IMPLICIT_A + ir_iters * BYTES_IMPLICIT + exp_iters * BYTES_EXPLICIT) * elems
    gbs = iters * BYTES_EXPLICIT * elems / dt / 1e9
    avg_pass_ms = pass_ms / max(launches, 1)
    # the dominant row-pass kernel (profiled launches average over the form that ran)
    if ia_iters == iters:
        path, per_elem = "implicit_RA", BYTES_IMPLICIT_A
        kernel = "k_row_ia (full iteration pass, implicit R and A)"
    elif imp_iters == iters and ia_iters == 0:
        path, per_elem = "implicit_R", BYTES_IMPLICIT
        kernel = "k_row_imp (full iteration pass, implicit R)"
    elif exp_iters == iters:
        path, per_elem = "explicit", BYTES_EXPLICIT
        kernel = "k_row_pass (full iteration pass)"
    else:
        path, per_elem = "mixed", exec_bytes / max(iters, 1) / elems
        kernel = "row passes of mixed forms (hand-over during the run)"
    per_launch = int(per_elem * elems)
    achieved = per_launch / (avg_pass_ms * 1e-3) / 1e9
    r0 = results[-1]
    traffic = None
    if (ROW_PASS_TRAFFIC is not None and n == N and path == ROW_PASS_TRAFFIC["path"]
            and source_sha256(ROW_PASS_SRC) == ROW_PASS_TRAFFIC["sha256"]):
        traffic = round((ROW_PASS_TRAFFIC["read"] + ROW_PASS_TRAFFIC["write"]) / 1e9, 3)
    out = {
        "metric": "dense AP GB/s & iter/s at N=20k; time to oracle exemplars, plain vs warm-start",
        "value": round(iters / dt, 2),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"dense AP, {n} points in {D}-D from a {K_MIX}-component Gaussian "
                               f"mixture; MFMA similarity, median preference, damping {LAMBDA}, "
                               f"stop after {CONV_ITER} unchanged exemplar sets",
                   "n": n, "d": D, "damping": LAMBDA, "max_iter": MAX_ITER, "conv_iter": CONV_ITER},
        "iterations_per_step": r0.iterations,
        "ms_per_step_graph": round(ms_graph, 3),
        "converged": r0.converged,
        "n_exemplars": r0.n_exemplars,
        "netsim": r0.netsim,
        "similarity_ms": round(sim_ms, 3),
        "value_basis": "AP iterations per second over whole steps (similarity, preference, "
                       "AP to the stop rule, finalize)",
        "iteration_path": {"form": path,
                           "implicit_RA_iterations": ia_iters, "implicit_R_iterations": ir_iters,
                           "explicit_iterations": exp_iters,
                           "bytes_per_element": {"implicit_RA": BYTES_IMPLICIT_A, "implicit_R": BYTES_IMPLICIT,
                                                 "explicit": BYTES_EXPLICIT},
                           "executed_GBps": round(exec_bytes / dt / 1e9, 2),
                           "dense_form_equivalent_GBps": round(gbs, 2),
                           "dense_form_note": f"{BYTES_EXPLICIT} B per element and iteration of the explicit "
                                              f"form over the step time: the rate the explicit form would "
                                              f"need for the same iterations/s, not bytes moved"},
        "roofline": {"bound": "hbm", "kernel": kernel,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "launches": launches, "avg_launch_ms": round(avg_pass_ms, 4),
                     "bytes_per_launch": per_launch,
                     "traffic_unit": "GB per launch (HBM read + write, counter-measured)"},
        "hbm_reference": hbm_ref,
    }
    if not args.no_extras:
        print("other workloads: PAP N=40000, 512 instances, LAP N=200000 ...", file=sys.stderr, flush=True)
        out["workloads"] = workload_extras(apx)
        from paper_0910_1650_amd import experiments as ex
        out["workloads"]["pap_k_sweep"] = {
            "workload": f"the benchmark matrix (N={n}): AP, then PAP with the paper's contiguous split "
                        f"for k = 2, 4, 8, 16 (Table 2's protocol)",
            "rows": ex.pap_k_sweep(S, truth=pts.labels),
        }
    if not args.no_warm_compare:
        print("time to oracle exemplars: cold / PAP / learned ...", file=sys.stderr, flush=True)
        out["time_to_exemplars"] = time_to_exemplars(apx, S, n, SEED)
    if not args.no_cpu_baseline:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pts, args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
