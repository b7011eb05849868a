"""Experiment protocols of the paper's evaluation (Section 5) on this
library's GPU calls: the PAP part-count sweep of Table 2, the size sweep of
the 2-D random sets (AP against PAP with k = 4 over N = 100..3000, ten runs
each), the pair metrics of the face experiments, and landmark re-seeding
from a previous LAP run (Section 6 names better landmark choice as future
work).  Host-side orchestration only: every AP runs in libapx.

PAP here uses the paper's partition (Algorithm 2, Step 1): k-1 contiguous
parts of floor(N/k) points and a last part of the rest (pap_solve with no
permutation and no offsets).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import (ap_similarity, ap_solve, apx_lap_landmarks, empty_matrix, lap_full_solve, lap_solve,
               pap_solve)


def association_rates(truth, labels) -> tuple[float, float]:
    """(TAR, FAR) over point pairs: the share of same-class pairs put in one
    cluster and of different-class pairs put in one cluster."""
    truth = np.asarray(truth)
    labels = np.asarray(labels)
    _, t = np.unique(truth, return_inverse=True)
    _, c = np.unique(labels, return_inverse=True)
    table = np.zeros((t.max() + 1, c.max() + 1), dtype=np.int64)
    np.add.at(table, (t, c), 1)

    def pairs(x):
        return int((x * (x - 1) // 2).sum())
    same_both = pairs(table)
    same_truth = pairs(table.sum(axis=1))
    same_clust = pairs(table.sum(axis=0))
    n = truth.size
    total = n * (n - 1) // 2
    tar = same_both / same_truth if same_truth else float("nan")
    far = (same_clust - same_both) / (total - same_truth) if total > same_truth else float("nan")
    return tar, far


def _clock(fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) * 1e3


def pap_k_sweep(S: torch.Tensor, ks=(2, 4, 8, 16), damping: float = 0.9, max_iter: int = 2000,
                conv_iter: int = 15, truth=None) -> list[dict]:
    """Table 2's protocol on one similarity matrix: AP, then PAP with the
    paper's contiguous split for each k.  Rows: classes (|E|), iterations
    (Step 4's for PAP, with the largest part's count beside it), wall ms,
    net similarity and, with ground truth, TAR and FAR."""
    n = S.shape[0]
    R, A = empty_matrix(n), empty_matrix(n)
    rows = []
    (idx, res), ms = _clock(lambda: ap_solve(S, R, A, damping, max_iter, conv_iter))
    row = dict(method="AP", k=1, classes=res.n_exemplars, iterations=res.iterations, ms=round(ms, 2),
               netsim=res.netsim, converged=res.converged)
    if truth is not None:
        row["TAR"], row["FAR"] = association_rates(truth, idx.cpu().numpy())
    rows.append(row)
    for k in ks:
        (idx, res, subs), ms = _clock(lambda: pap_solve(S, R, A, k, None, None, damping, max_iter, conv_iter))
        row = dict(method="PAP", k=k, classes=res.n_exemplars, iterations=res.iterations,
                   part_iterations=max(r.iterations for r in subs), ms=round(ms, 2), netsim=res.netsim,
                   converged=res.converged)
        if truth is not None:
            row["TAR"], row["FAR"] = association_rates(truth, idx.cpu().numpy())
        rows.append(row)
    return rows


def size_sweep(sizes=tuple(range(100, 3001, 100)), runs: int = 10, k: int = 4, damping: float = 0.9,
               max_iter: int = 2000, conv_iter: int = 15, seed0: int = 1101, points=None) -> list[dict]:
    """The 2-D random-set protocol: for every N, `runs` seeded instances of
    `points(n, seed)` (default: 10-component 2-D mixtures), AP and PAP with
    k parts; mean iterations and wall ms of each, per N."""
    import synth
    points = points or (lambda n, seed: synth.gaussian_2d(n=n, k=10, seed=seed))
    out = []
    for n in sizes:
        it_ap, it_pap, ms_ap, ms_pap = [], [], [], []
        for r in range(runs):
            seed = seed0 + 1000 * r + n
            X = torch.from_numpy(points(n, seed).X).cuda()
            S, _ = ap_similarity(X, pref="median", noise_seed=seed, noise_rel=1e-12)
            R, A = empty_matrix(n), empty_matrix(n)
            (_, ra), ta = _clock(lambda: ap_solve(S, R, A, damping, max_iter, conv_iter))
            (_, rp, _), tp = _clock(lambda: pap_solve(S, R, A, k, None, None, damping, max_iter, conv_iter))
            it_ap.append(ra.iterations)
            it_pap.append(rp.iterations)
            ms_ap.append(ta)
            ms_pap.append(tp)
        out.append(dict(n=n, runs=runs, ap_iterations=float(np.mean(it_ap)),
                        pap_iterations=float(np.mean(it_pap)), ap_ms=round(float(np.mean(ms_ap)), 3),
                        pap_ms=round(float(np.mean(ms_pap)), 3)))
    return out


def lap_reseed(X: torch.Tensor, n_landmarks: int, seed: int, rounds: int = 2, full: bool = False,
               m0: int = 20000, damping: float = 0.9, max_iter: int = 2000, conv_iter: int = 15) -> list[dict]:
    """Landmark AP, then again with the landmarks re-seeded from the previous
    run's exemplars (kept) plus a fresh uniform sample of the other points.
    Per round: exemplars, net similarity, wall ms."""
    n = X.shape[0]
    keep = None
    out = []
    for r in range(rounds):
        M = apx_lap_landmarks(n, n_landmarks, keep, seed + r)
        if full:
            (idx, res, ex, _), ms = _clock(lambda: lap_full_solve(X, n_landmarks, m0=m0, landmarks=M, seed=seed,
                                                                   damping=damping, max_iter=max_iter,
                                                                   conv_iter=conv_iter))
        else:
            (idx, res, ex), ms = _clock(lambda: lap_solve(X, n_landmarks, landmarks=M, seed=seed, damping=damping,
                                                          max_iter=max_iter, conv_iter=conv_iter))
        out.append(dict(round=r, kept=0 if keep is None else int(keep.size), n_exemplars=res.n_exemplars,
                        netsim=res.netsim, ms=round(ms, 2)))
        keep = ex[: min(ex.size, n_landmarks)]
    return out
