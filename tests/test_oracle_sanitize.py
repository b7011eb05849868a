"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code, CPU only): oracle/apo.c is built with -fsanitize=address,undefined
(errors fatal) into a temporary library, and a child process runs every entry
point the Python side uses on small inputs (similarity, preferences and
noise, Algorithm 1 with and without warm starts and with the message stop,
the row-wise pieces, Algorithm 2, Algorithm 3 Steps 1-2 and the full method's
distance helpers).  Any out-of-bounds access, use after free or undefined
operation aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle, synth
from oracle import lap_full
oracle._LIB_PATH = sys.argv[2]
pts = synth.gaussian_mixture(n=60, d=5, k=4, seed=3)
S0 = oracle.similarity(pts.X)
prep = oracle.prepare(S0, "median", seed=3)
S = prep.S
r = oracle.ap(S, 0.9, 300, 15)
r2 = oracle.ap(S, 0.5, 40, 0, A0=r.A, R0=r.R)
r3 = oracle.ap(S, 0.9, 300, 0, msg_tol=1e-6)
rows = np.arange(0, 60, 7)
oracle.resp_rows(S, r.A, r.R, 0.9, rows)
oracle.avail_rows(r.R, r.A, 0.9, rows)
oracle.column_sums(r.R)
oracle.decisions(r.A, r.R)
p = oracle.pap(S, 3, None, None, lam=0.9, max_iter=200, conv_iter=15)
perm = np.random.default_rng(0).permutation(60)
p2 = oracle.pap(S, 4, perm, np.array([0, 10, 25, 41, 60]), lam=0.9, max_iter=100, conv_iter=15)
big = synth.gaussian_mixture(n=400, d=6, k=5, seed=4)
M = np.sort(np.random.default_rng(1).choice(400, 60, replace=False))
l = oracle.lap(big.X, M, seed=4)
q = np.arange(400)
oracle.nearest_of(big.X, q, l.exemplars)
oracle.pair_dist(big.X, q[:50], q[50:100])
oracle.medoid(big.X, q[:30])
f = lap_full.lap_full(big.X, None, 60, seed=4, m0=100)
print("ok", r.iterations, r3.iterations, p.full.iterations, l.exemplars.size, f.exemplars.size)
'''


def _runtime(name):
    try:
        out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True, timeout=30)
    except (OSError, subprocess.TimeoutExpired):
        return None
    path = out.stdout.strip()
    return path if path and os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    lib = str(tmp_path / "libapo_san.so")
    src = os.path.join(ROOT, "oracle", "apo.c")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-o", lib, src, "-lm"], check=True, timeout=300)
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "4"
    out = subprocess.run([sys.executable, "-c", CHILD, ROOT, lib], capture_output=True, text=True, env=env,
                         timeout=600)
    assert out.returncode == 0, out.stderr[-4000:]
    assert "AddressSanitizer" not in out.stderr and "runtime error" not in out.stderr, out.stderr[-4000:]
    assert out.stdout.startswith("ok"), out.stdout
