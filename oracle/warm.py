"""FP64 oracle for the learned warm start of affinity propagation.

TEST INFRASTRUCTURE ONLY (like the rest of this package): the tests, the
smoke check and the benchmark's CPU leg may call it; the GPU library never
does and shares no code with it.

The paper has no learned component.  Its warm start is PAP's merged
availabilities (Section 3, Algorithm 2, steps 3-4); the learned warm start
replaces that merge with a per-point prediction made from the rows of S.
Everything here is therefore this project's own definition, written out
plainly so that the GPU kernels can be checked against it:

Features (16 per point k, from row k of S; n >= 2, m = n - 1 off-diagonal
values o_0 <= ... <= o_{m-1} in ascending order):
  row median      mu_k = o_{floor((m-1)/2)}
  scale           sigma = |lower median of (mu_0 .. mu_{n-1})|  (1 if that is 0)
  f0..f5          o_{m-1-min(j, m-1)} / sigma for j = 0, 1, 3, 7, 15, 31
                  (the 1st, 2nd, 4th, 8th, 16th, 32nd largest)
  f6              mean of the min(32, m) largest / sigma
  f7..f11         o_{floor(q (m-1) / 100)} / sigma for q = 1, 10, 25, 50, 75
  f12             (s(k,k) - mu_k) / sigma
  f13             (s(k,k) - f6 * sigma) / sigma
  f14             #{j != k : s(k,j) > s(k,k)} / m
  f15             ln(n) / 10
Each feature is evaluated in double from FP32 inputs and rounded once to FP32.

Network: 16 -> 128 -> 128 -> 2, GELU (erf form) after both hidden layers.
Mixed precision: the features, the three weight matrices and both hidden
activations are rounded to bfloat16 (round to nearest even, from the FP32
value); biases stay FP32; every product is exact and every sum is carried in
FP32 on the device (FP64 here).  The backward pass treats each rounding as
the identity (straight-through), so the gradient applies to the FP32 master
weights.

Targets (from a converged run of Algorithm 1): the column quantities of
Eqs. (3)-(4), c_k = sum_{i != k} max(0, r(i,k)) and t_k = r(k,k) + c_k, over
sigma: y0 -> t_k / sigma (its sign marks exemplars; min(0, t_k) is the level
of the off-diagonal availabilities in column k), y1 -> c_k / sigma (the self
availability of Eq. (4)).

Warm start: a0(i,k) = min(0, sigma * y0_k) for i != k and
a0(k,k) = max(0, sigma * y1_k), i.e. Eqs. (3)-(4) evaluated with the
predicted column quantities and R = 0, which keeps off-diagonal availabilities
non-positive and self availabilities non-negative as Algorithm 1 does.

Loss: Huber (delta 1) on both outputs, sum over outputs, weighted sum over
points with caller-given weights.  Optimiser: Adam (Kingma and Ba, 2015)
with bias correction, on the FP32 master weights.
"""
from __future__ import annotations

import math

import numpy as np

N_FEATURES = 16
HIDDEN = 128
N_OUT = 2
DESC_RANKS = (0, 1, 3, 7, 15, 31)
QUANT_PERCENT = (1, 10, 25, 50, 75)
TOP = 32

# name, shape; the flat parameter vector is these tensors row-major, in order.
SHAPES = (("W1", (N_FEATURES, HIDDEN)), ("b1", (HIDDEN,)),
          ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
          ("W3", (HIDDEN, N_OUT)), ("b3", (N_OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 18946


def unpack(theta: np.ndarray) -> dict:
    theta = np.asarray(theta, dtype=np.float64).ravel()
    assert theta.size == N_PARAMS
    out, o = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = theta[o:o + size].reshape(shape)
        o += size
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


# --------------------------------------------------------------------------
# bfloat16, GELU, Huber
# --------------------------------------------------------------------------
def bf16_round(x) -> np.ndarray:
    """Round to bfloat16 (8 significant bits, round to nearest, ties to even)
    after first rounding to FP32, returned as float64.  NaN stays NaN."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def _erf(z: np.ndarray) -> np.ndarray:
    return np.vectorize(math.erf, otypes=[np.float64])(z)


def gelu(z: np.ndarray) -> np.ndarray:
    """z * Phi(z) with Phi the standard normal CDF, Phi(z) = (1 + erf(z/sqrt2))/2."""
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z: np.ndarray) -> np.ndarray:
    """d/dz z*Phi(z) = Phi(z) + z*phi(z), phi the standard normal density."""
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def huber(e: np.ndarray) -> np.ndarray:
    a = np.abs(e)
    return np.where(a <= 1.0, 0.5 * e * e, a - 0.5)


def huber_grad(e: np.ndarray) -> np.ndarray:
    return np.clip(e, -1.0, 1.0)


# --------------------------------------------------------------------------
# Network
# --------------------------------------------------------------------------
def forward(theta: np.ndarray, X: np.ndarray, bf16: bool = True):
    """Outputs y (B x 2) and the intermediate values the backward pass needs."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(theta)
    x = rnd(X)
    W1, W2, W3 = rnd(p["W1"]), rnd(p["W2"]), rnd(p["W3"])
    z1 = x @ W1 + p["b1"]
    h1 = rnd(gelu(z1))
    z2 = h1 @ W2 + p["b2"]
    h2 = rnd(gelu(z2))
    y = h2 @ W3 + p["b3"]
    return y, dict(x=x, W1=W1, W2=W2, W3=W3, z1=z1, h1=h1, z2=z2, h2=h2)


def loss(theta, X, T, w, bf16: bool = True) -> float:
    y, _ = forward(theta, X, bf16)
    return float(np.sum(np.asarray(w, dtype=np.float64)[:, None] * huber(y - T)))


def backward(theta, X, T, w, bf16: bool = True):
    """Loss, its gradient with respect to the flat parameters, and y."""
    y, c = forward(theta, X, bf16)
    w = np.asarray(w, dtype=np.float64)
    e = y - np.asarray(T, dtype=np.float64)
    L = float(np.sum(w[:, None] * huber(e)))
    dy = w[:, None] * huber_grad(e)
    g = {"W3": c["h2"].T @ dy, "b3": dy.sum(axis=0)}
    dz2 = (dy @ c["W3"].T) * gelu_grad(c["z2"])
    g["W2"] = c["h1"].T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ c["W2"].T) * gelu_grad(c["z1"])
    g["W1"] = c["x"].T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return L, pack(g), y


def adam_step(theta, m, v, g, step: int, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step counts from 1).  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


# --------------------------------------------------------------------------
# Features, targets, warm start
# --------------------------------------------------------------------------
def row_stats(S: np.ndarray, k: int) -> dict:
    """Order statistics of the off-diagonal of row k (FP32 values as double)."""
    n = S.shape[0]
    row = np.asarray(S[k], dtype=np.float64)
    off = np.sort(np.delete(row, k))
    m = n - 1
    top = off[m - min(TOP, m):]
    return dict(
        mu=off[(m - 1) // 2],
        desc=[off[m - 1 - min(j, m - 1)] for j in DESC_RANKS],
        top_mean=math.fsum(top) / top.size,
        quant=[off[(q * (m - 1)) // 100] for q in QUANT_PERCENT],
        diag=row[k],
        above=int(np.count_nonzero(off > row[k])),
    )


def scale(S: np.ndarray) -> float:
    """sigma: absolute value of the lower median of the n row medians."""
    n = S.shape[0]
    m = n - 1
    mus = np.empty(n)
    for k in range(n):
        off = np.delete(np.asarray(S[k], dtype=np.float64), k)
        mus[k] = np.partition(off, (m - 1) // 2)[(m - 1) // 2]
    mus.sort()
    s = abs(float(mus[(n - 1) // 2]))
    return s if s > 0 and math.isfinite(s) else 1.0


def features(S: np.ndarray, rows=None, sigma: float | None = None):
    """Feature matrix (len(rows) x 16, FP32) and sigma."""
    n = S.shape[0]
    assert n >= 2
    if sigma is None:
        sigma = scale(S)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    F = np.empty((rows.size, N_FEATURES), dtype=np.float32)
    m = n - 1
    for r, k in enumerate(rows):
        st = row_stats(S, int(k))
        vals = [d / sigma for d in st["desc"]]
        vals.append(st["top_mean"] / sigma)
        vals += [q / sigma for q in st["quant"]]
        vals.append((st["diag"] - st["mu"]) / sigma)
        vals.append((st["diag"] - st["top_mean"]) / sigma)
        vals.append(st["above"] / m)
        vals.append(math.log(n) / 10.0)
        F[r] = np.asarray(vals, dtype=np.float64).astype(np.float32)
    return F, sigma


def column_state(R: np.ndarray):
    """c_k = sum_{i != k} max(0, r(i,k)) and t_k = r(k,k) + c_k (Eqs. (3)-(4))."""
    R = np.asarray(R, dtype=np.float64)
    P = np.maximum(R, 0.0)
    np.fill_diagonal(P, 0.0)
    c = P.sum(axis=0)
    return np.diag(R) + c, c


def targets(R: np.ndarray, sigma: float) -> np.ndarray:
    t, c = column_state(R)
    return np.stack([t / sigma, c / sigma], axis=1).astype(np.float32)


def warm_a0(Y: np.ndarray, sigma: float) -> np.ndarray:
    """A_0 from the predicted column quantities (FP32 products, as stored)."""
    Y = np.asarray(Y, dtype=np.float32)
    s = np.float32(sigma)
    lvl = np.minimum(np.float32(0), s * Y[:, 0])
    slf = np.maximum(np.float32(0), s * Y[:, 1])
    n = Y.shape[0]
    A0 = np.broadcast_to(lvl[None, :], (n, n)).astype(np.float64)
    A0[np.arange(n), np.arange(n)] = slf
    return A0


def warm_start(S: np.ndarray, theta: np.ndarray):
    """Features -> network -> A_0, all in the oracle.  Returns (A0, F, y, sigma)."""
    F, sigma = features(S)
    y, _ = forward(theta, F, bf16=True)
    y32 = y.astype(np.float32)
    return warm_a0(y32, sigma), F, y32, sigma

