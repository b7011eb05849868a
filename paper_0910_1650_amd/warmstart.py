"""Training and evaluation driver for the learned warm start.

The host holds the loop; every computation is a libapx call (similarity,
features, Algorithm 1, targets, network backward, Adam).  The paper has no
learned component: its Algorithm 1 starts from zero availabilities (Eq. (1))
and PAP warm-starts from merged sub-problem availabilities (Algorithm 2).

Training data: seeded synthetic instances of two families, alternating --
2-D Gaussian mixtures (10 components) and 64-D Gaussian mixtures (50
components) -- with n uniform in [n_lo, n_hi].  For each instance the
library builds S (median preference, tie noise), the features, runs
Algorithm 1 cold to its stop rule and, if it converged, takes the targets
(t_k, c_k)/sigma from the converged responsibilities.  Non-converged
instances are dropped and counted.

Training: Adam on the weighted Huber loss, every instance weighing the same
(point weight proportional to 1/n of its instance), minibatches drawn from a
seeded permutation of all points, cosine-decayed learning rate.

    python -m paper_0910_1650_amd.warmstart --instances 2000 --out weights.npy
"""
from __future__ import annotations

import argparse
import math
import os
import time

import numpy as np
import torch

from . import (APX_MLP_PARAMS, APX_WARM_COLUMNS, ap_similarity, ap_solve, ap_warmstart, apx_features,
               apx_mlp_adam, apx_mlp_backward, apx_targets, empty_matrix, pap_solve)

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "warmstart_weights.npy")
FAMILIES = ("mix2d", "mix64d")
SHAPES = ((16, 128), (128,), (128, 128), (128,), (128, 2), (2,))


def init_params(seed: int) -> np.ndarray:
    """Weights uniform in +-1/sqrt(fan_in), biases zero (FP32, flat layout)."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in SHAPES:
        if len(shape) == 2:
            b = 1.0 / math.sqrt(shape[0])
            parts.append(rng.uniform(-b, b, size=shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def load_weights(path: str = WEIGHTS, device="cuda") -> torch.Tensor:
    a = np.load(path, allow_pickle=False)
    if a.dtype != np.float32 or a.shape != (APX_MLP_PARAMS,):
        raise ValueError(f"{path}: expected {APX_MLP_PARAMS} float32 parameters")
    return torch.from_numpy(a).to(device)


def family_points(family: str, n: int, seed: int):
    import synth
    if family == "mix2d":
        return synth.gaussian_2d(n=n, k=10, seed=seed)
    if family == "mix64d":
        return synth.gaussian_mixture(n=n, d=64, k=50, seed=seed)
    raise ValueError(family)


def instance_spec(j: int, seed0: int, n_lo: int, n_hi: int):
    seed = seed0 + j
    n = int(np.random.default_rng(seed).integers(n_lo, n_hi + 1))
    return FAMILIES[j % 2], n, seed


def build_dataset(count: int, n_lo: int, n_hi: int, seed0: int, damping: float = 0.9,
                  max_iter: int = 1000, conv_iter: int = 15, log=print):
    """Features, targets and per-point instance weights of `count` instances."""
    Fs, Ys, ws = [], [], []
    dropped, iters = 0, []
    t0 = time.time()
    for j in range(count):
        family, n, seed = instance_spec(j, seed0, n_lo, n_hi)
        X = torch.from_numpy(family_points(family, n, seed).X).cuda()
        S, _ = ap_similarity(X, pref="median", noise_seed=seed, noise_rel=1e-12)
        F, sig = apx_features(S)
        R, A = empty_matrix(n), empty_matrix(n)
        _, res = ap_solve(S, R, A, damping, max_iter, conv_iter)
        if not res.converged:
            dropped += 1
            continue
        iters.append(res.iterations)
        Fs.append(F)
        Ys.append(apx_targets(R, sig))
        ws.append(torch.full((n,), 1.0 / n, dtype=torch.float32, device="cuda"))
        if (j + 1) % 100 == 0:
            log(f"instances {j + 1}/{count}: dropped {dropped}, mean iterations "
                f"{np.mean(iters):.1f}, {time.time() - t0:.1f} s")
    F = torch.cat(Fs)
    Y = torch.cat(Ys)
    w = torch.cat(ws) / len(Fs)
    return F, Y, w, dict(used=len(Fs), dropped=dropped, mean_iterations=float(np.mean(iters)),
                         points=int(F.shape[0]), seconds=time.time() - t0)


def train(F, Y, w, steps: int = 20000, batch: int = 8192, lr: float = 2e-3, seed: int = 0,
          log_every: int = 1000, log=print) -> torch.Tensor:
    """Adam on the weighted Huber loss; returns the FP32 parameters."""
    P = F.shape[0]
    wb = (w * (P / batch)).contiguous()      # batch loss estimates the instance-averaged loss
    theta = torch.from_numpy(init_params(seed)).cuda()
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    gen = torch.Generator().manual_seed(seed)
    perm, pos = None, P
    grad = torch.empty_like(theta)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    t0 = time.time()
    acc = 0.0
    for step in range(1, steps + 1):
        if pos + batch > P:
            perm = torch.randperm(P, generator=gen).cuda()
            pos = 0
        rows = perm[pos:pos + batch]
        pos += batch
        apx_mlp_backward(theta, F, Y, wb, rows=rows, grad=grad, loss=loss)
        lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / steps))
        apx_mlp_adam(theta, m, v, grad, step, lr_t)
        if step % 50 == 0:
            acc += loss.item()
        if step % log_every == 0:
            log(f"step {step}/{steps}: loss {acc / (log_every // 50):.5f}, {time.time() - t0:.1f} s")
            acc = 0.0
    return theta


def solve_cold(S, damping=0.9, max_iter=2000, conv_iter=15):
    n = S.shape[0]
    R, A = empty_matrix(n), empty_matrix(n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx, res = ap_solve(S, R, A, damping, max_iter, conv_iter)
    return idx, res, (time.perf_counter() - t0) * 1e3


def degenerate(res, n: int) -> bool:
    """A warm-started run that did not converge, found no exemplar, or made
    more than half the points exemplars is discarded for a cold run."""
    return (not res.converged) or res.n_exemplars == 0 or res.n_exemplars > n // 2


def solve_warm(S, theta, damping=0.9, max_iter=2000, conv_iter=15):
    """ap_warmstart then Algorithm 1 from (R_0, A_0), with cold start as the
    fallback; time includes the warm start (and the fallback, if taken).
    Returns (idx, result, ms, iterations of every run, fell_back)."""
    n = S.shape[0]
    R, A = empty_matrix(n), empty_matrix(n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ap_warmstart(S, theta, R, A)
    idx, res = ap_solve(S, R, A, damping, max_iter, conv_iter, warm=APX_WARM_COLUMNS)
    total = res.iterations
    fell_back = degenerate(res, n)
    if fell_back:
        idx, res = ap_solve(S, R, A, damping, max_iter, conv_iter)
        total += res.iterations
    return idx, res, (time.perf_counter() - t0) * 1e3, total, fell_back


def solve_pap(S, k: int, seed: int, damping=0.9, max_iter=2000, conv_iter=15):
    """Algorithm 2 with a random uneven partition into k parts (sizes drawn
    in [0.075 n, 0.175 n] before normalisation) of consecutive indices: the
    points are drawn i.i.d., so that is a uniformly random partition, and
    Step 4 can keep its availabilities implicit."""
    import synth
    n = S.shape[0]
    _, offsets = synth.random_partition(n, k, lo=max(1, (3 * n) // 40), hi=max(2, (7 * n) // 40), seed=seed)
    R, A = empty_matrix(n), empty_matrix(n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx, res, subs = pap_solve(S, R, A, k, None, offsets, damping, max_iter, conv_iter)
    return idx, res, (time.perf_counter() - t0) * 1e3, subs


def exemplar_set(idx: torch.Tensor) -> np.ndarray:
    lab = idx.cpu().numpy()
    return np.flatnonzero(lab == np.arange(lab.size))


def evaluate(theta, specs, damping=0.9, pap_k: int = 8, log=print):
    """Cold start against the learned warm start and PAP on (family, n, seed)
    instances: iterations, wall time, whether the exemplar set equals the
    cold run's, and net similarity relative to the cold run's."""
    rows = []
    for family, n, seed in specs:
        X = torch.from_numpy(family_points(family, n, seed).X).cuda()
        S, _ = ap_similarity(X, pref="median", noise_seed=seed, noise_rel=1e-12)
        ic, rc, tc = solve_cold(S, damping)
        E = exemplar_set(ic)
        iw, rw, tw, itw, fb = solve_warm(S, theta, damping)
        ip, rp, tp, subs = solve_pap(S, pap_k, seed, damping)
        row = dict(family=family, n=n, seed=seed, n_exemplars=rc.n_exemplars,
                   cold=dict(iterations=rc.iterations, ms=round(tc, 2), netsim=rc.netsim),
                   learned=dict(iterations=itw, ms=round(tw, 2), fallback=fb,
                                same_exemplars=bool(np.array_equal(exemplar_set(iw), E)),
                                netsim_ratio=rw.netsim / rc.netsim, n_exemplars=rw.n_exemplars),
                   pap=dict(iterations=rp.iterations, sub_iterations=max(r.iterations for r in subs),
                            ms=round(tp, 2), same_exemplars=bool(np.array_equal(exemplar_set(ip), E)),
                            netsim_ratio=rp.netsim / rc.netsim, n_exemplars=rp.n_exemplars))
        log(str(row))
        rows.append(row)
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--instances", type=int, default=2000)
    ap.add_argument("--n-lo", type=int, default=2000)
    ap.add_argument("--n-hi", type=int, default=10000)
    ap.add_argument("--seed0", type=int, default=50000)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval-n", type=int, nargs="*", default=[20000, 40000])
    ap.add_argument("--eval-seeds", type=int, default=4)
    ap.add_argument("--eval-json", default="")
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()

    def log(msg):
        print(msg, flush=True)

    F, Y, w, info = build_dataset(args.instances, args.n_lo, args.n_hi, args.seed0, log=log)
    log(f"dataset: {info}")
    theta = train(F, Y, w, args.steps, args.batch, args.lr, log=log)
    np.save(args.out, theta.cpu().numpy().astype(np.float32), allow_pickle=False)
    log(f"weights written to {args.out}")
    specs = [(FAMILIES[s % 2], n, 60000 + s) for n in args.eval_n for s in range(args.eval_seeds)]
    rows = evaluate(theta, specs, log=log)
    if args.eval_json:
        import json
        with open(args.eval_json, "w") as f:
            json.dump(dict(dataset=info, eval=rows), f, indent=1)


if __name__ == "__main__":
    main()
