"""Write the FP64 oracle's converged exemplar sets for the timed workloads.

Runs only the CPU oracle (Algorithm 1 to convergence from A=0, R=0) on the
seeded synthetic inputs and stores, per workload, the exemplar set E, the
labels (Algorithm 1's idx), the iteration at which the stop rule fired, the
preference and the net similarity.  The GPU runs (cold start and the warm
starts) are judged against these.

    python tests/golden/make_oracle_exemplars.py [name ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

# name -> (generator, kwargs, damping, max_iter, conv_iter, noise seed)
WORKLOADS = {
    "c2_n20000_d64_k50_seed2001": (
        "gaussian_mixture", dict(n=20000, d=64, k=50, seed=2001), 0.9, 2000, 15, 2001),
}


def run(name):
    gen, kw, lam, max_iter, conv_iter, seed = WORKLOADS[name]
    t0 = time.time()
    pts = getattr(synth, gen)(**kw)
    prep = oracle.prepare(oracle.similarity(pts.X), "median", seed=seed)
    t1 = time.time()
    res = oracle.ap(prep.S, lam, max_iter, conv_iter)
    t2 = time.time()
    out = {
        "workload": name,
        "generator": gen,
        "args": kw,
        "damping": lam,
        "max_iter": max_iter,
        "conv_iter": conv_iter,
        "noise_seed": seed,
        "noise_rel": 1e-12,
        "preference": prep.pref,
        "range": float(prep.S.max() - prep.S.min()),
        "iterations": res.iterations,
        "converged": bool(res.converged),
        "n_exemplars": int(res.n_exemplars),
        "exemplars": [int(e) for e in res.exemplars],
        "labels": [int(v) for v in res.idx],
        "netsim": res.netsim,
        "dpsim": res.dpsim,
        "expref": res.expref,
        "oracle_threads": oracle.num_threads(),
        "seconds": {"setup": round(t1 - t0, 1), "ap": round(t2 - t1, 1)},
    }
    labels = out.pop("labels")
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write(',\n')
    # the labels on one line, appended as the last key
    with open(os.path.join(HERE, name + ".json"), "r+") as f:
        body = f.read().rstrip().rstrip(",").rstrip()
        assert body.endswith("}")
        f.seek(0)
        f.write(body[:-1].rstrip() + ',\n "labels": ' + json.dumps(labels, separators=(",", ":")) + "\n}\n")
        f.truncate()
    print(name, out["iterations"], out["n_exemplars"], out["netsim"], out["seconds"], flush=True)
    del prep, res
    np.zeros(1)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(WORKLOADS):
        run(name)
