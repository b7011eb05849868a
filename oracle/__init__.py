"""FP64 CPU oracle for dense affinity propagation, PAP and LAP.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the GPU library never
does, and the two share no code.  The arithmetic lives in ``apo.c`` (plain C,
IEEE double, OpenMP over rows/column chunks with a fixed summation order);
this wrapper marshals numpy arrays and composes the paper's algorithms:

* Algorithm 1 (affinity propagation), Section 2, Eqs. (1)-(4)
* Algorithm 2 (partition AP), Section 3
* Algorithm 3 (landmark AP) Steps 1-2 with the nearest-exemplar rule, Section 4
* the learned warm start (features, network, targets, A_0) in ``warm.py``,
  a definition of this project's own: the paper has no learned part

Readings of the paper that the oracle fixes:
R_0 = 0; R is updated and damped before A, and A uses the damped R; damping
weights the old value by lambda; ties go to the lowest index; the exemplar
set is E = {i : argmax_k a(i,k)+r(i,k) = i} and labels are the valid
configuration (exemplars label themselves, the rest take the most similar
exemplar); the stop rule counts consecutive iterations with the same E.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libapo.so")
_lib = None

_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_u64 = ctypes.c_uint64


def lib():
    """Load oracle/libapo.so, building it with gcc first if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    L = ctypes.CDLL(_LIB_PATH)
    L.apo_num_threads.restype = ctypes.c_int
    L.apo_similarity.argtypes = [_i64, _i64, _f32p, _i64, _f64p]
    L.apo_sqdist.argtypes = [_i64, _f32p, _f32p]
    L.apo_sqdist.restype = _dbl
    L.apo_noise_u.argtypes = [_u64, _i64, _i64, _i64]
    L.apo_noise_u.restype = _dbl
    L.apo_add_noise.argtypes = [_i64, _f64p, _u64, _dbl]
    L.apo_ap.argtypes = [_i64, _f64p, _dbl, _i32, _i32, _f64p, _f64p, _i32p,
                         ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.c_void_p]
    L.apo_ap.restype = ctypes.c_int
    L.apo_ap_tol.argtypes = [_i64, _f64p, _dbl, _i32, _i32, _dbl, _f64p, _f64p, _i32p,
                             ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.c_void_p]
    L.apo_ap_tol.restype = ctypes.c_int
    L.apo_decisions.argtypes = [_i64, _f64p, _f64p, _i32p]
    L.apo_finalize.argtypes = [_i64, _f64p, _i32p, _i32p, ctypes.POINTER(_dbl),
                               ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)]
    L.apo_finalize.restype = _i64
    L.apo_assign_nearest.argtypes = [_i64, _i64, _f32p, _i64, _i64, _i64p, _i32p,
                                     ctypes.POINTER(_dbl)]
    L.apo_nearest_of.argtypes = [_i64, _f32p, _i64, _i64, _i64p, _i64, _i64p, _i32p, _f64p]
    L.apo_pair_dist.argtypes = [_i64, _f32p, _i64, _i64, _i64p, _i64p, _f64p]
    L.apo_medoid.argtypes = [_i64, _f32p, _i64, _i64, _i64p]
    L.apo_medoid.restype = _i64
    L.apo_resp_rows.argtypes = [_i64, _f64p, _f64p, _f64p, _dbl, _i64p, _i64, _f64p]
    L.apo_column_sums.argtypes = [_i64, _f64p, _f64p]
    L.apo_avail_rows.argtypes = [_i64, _f64p, _f64p, _f64p, _dbl, _i64p, _i64, _f64p]
    _lib = L
    return L


def num_threads() -> int:
    return int(lib().apo_num_threads())


# --------------------------------------------------------------------------
# Similarity, preferences, tie noise (Section 2)
# --------------------------------------------------------------------------
def similarity(X: np.ndarray) -> np.ndarray:
    """S with s(i,k) = -||x_i - x_k||^2 (FP64, direct form), zero diagonal."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, d = X.shape
    S = np.empty((n, n), dtype=np.float64)
    lib().apo_similarity(n, d, X, d, S)
    return S


def median_offdiag(S: np.ndarray) -> float:
    """Median of the n(n-1) off-diagonal entries (mean of the two middle
    order statistics for an even count), selected with numpy's partition."""
    n = S.shape[0]
    if n < 2:
        return float("nan")
    vals = S[~np.eye(n, dtype=bool)]
    m = vals.size
    if m % 2:
        return float(np.partition(vals, m // 2)[m // 2])
    part = np.partition(vals, [m // 2 - 1, m // 2])
    return float((part[m // 2 - 1] + part[m // 2]) / 2.0)


def noise_u(seed: int, n: int, i: int, k: int) -> float:
    return float(lib().apo_noise_u(seed, n, i, k))


def add_noise(S: np.ndarray, seed: int, scale: float) -> None:
    assert S.dtype == np.float64 and S.flags.c_contiguous
    lib().apo_add_noise(S.shape[0], S, seed, scale)


@dataclass
class Prepared:
    S: np.ndarray       # diagonal = preferences, noise added
    pref: float | None  # scalar preference (None when a vector was given)
    noise_scale: float  # rel * (max S - min S) of the noiseless matrix


def prepare(S0: np.ndarray, pref="median", seed: int = 0, noise_rel: float = 1e-12) -> Prepared:
    """Set the preferences on the diagonal, then add the tie-break noise.

    pref: "median" (median of off-diagonal S), a float, or an (n,) vector.
    The noise scale is noise_rel * (max S - min S) of the matrix with the
    preferences set and no noise; noise goes to all n*n entries."""
    S = np.array(S0, dtype=np.float64, copy=True, order="C")
    n = S.shape[0]
    if isinstance(pref, str):
        assert pref == "median"
        p = median_offdiag(S0) if n > 1 else 0.0
        np.fill_diagonal(S, p)
        pscalar = p
    elif np.ndim(pref) == 0:
        np.fill_diagonal(S, float(pref))
        pscalar = float(pref)
    else:
        np.fill_diagonal(S, np.asarray(pref, dtype=np.float64))
        pscalar = None
    scale = 0.0
    if noise_rel > 0 and n > 0:
        scale = noise_rel * float(S.max() - S.min())
        add_noise(S, seed, scale)
    return Prepared(S, pscalar, scale)


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------
@dataclass
class APResult:
    R: np.ndarray
    A: np.ndarray
    dec: np.ndarray        # raw decisions of the last iteration
    iterations: int
    converged: bool
    trace_nex: np.ndarray  # |E_t| per iteration
    idx: np.ndarray | None = None
    n_exemplars: int = 0
    dpsim: float = float("nan")
    expref: float = float("nan")
    netsim: float = float("nan")

    @property
    def exemplars(self) -> np.ndarray:
        return np.flatnonzero(self.dec == np.arange(self.dec.size))


def ap(S: np.ndarray, lam: float = 0.5, max_iter: int = 200, conv_iter: int = 15,
       A0: np.ndarray | None = None, R0: np.ndarray | None = None,
       finalize_labels: bool = True, msg_tol: float | None = None) -> APResult:
    """Run Algorithm 1 on S (diagonal = preferences) from A0 (default 0, Eq. (1))
    and R0 (default 0).  conv_iter=0 runs exactly max_iter iterations.
    msg_tol (Algorithm 1, Step 4): also stop after the first iteration t >= 2
    whose every message changed by at most msg_tol."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    n = S.shape[0]
    R = np.zeros((n, n)) if R0 is None else np.array(R0, dtype=np.float64, order="C", copy=True)
    A = np.zeros((n, n)) if A0 is None else np.array(A0, dtype=np.float64, order="C", copy=True)
    dec = np.empty(n, dtype=np.int32)
    it, cv = _i32(0), _i32(0)
    trace = np.zeros(max_iter, dtype=np.int32)
    tol = -1.0 if msg_tol is None else float(msg_tol)
    rc = lib().apo_ap_tol(n, S, lam, max_iter, conv_iter, tol, R, A, dec, ctypes.byref(it),
                          ctypes.byref(cv), trace.ctypes.data)
    if rc != 0:
        raise ValueError(f"apo_ap failed with code {rc}")
    res = APResult(R, A, dec, int(it.value), bool(cv.value), trace[: it.value].copy())
    if finalize_labels:
        fin = finalize(S, dec)
        res.idx, res.n_exemplars = fin["idx"], fin["n_exemplars"]
        res.dpsim, res.expref, res.netsim = fin["dpsim"], fin["expref"], fin["netsim"]
    return res


def resp_rows(S, A, R, lam, rows) -> np.ndarray:
    """Eq. (2) with damping for the listed rows: R_next[rows] from (S, A, R)."""
    n = S.shape[0]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.size, n))
    lib().apo_resp_rows(n, np.ascontiguousarray(S, dtype=np.float64), np.ascontiguousarray(A, dtype=np.float64),
                        np.ascontiguousarray(R, dtype=np.float64), lam, rows, rows.size, out)
    return out


def column_sums(R) -> np.ndarray:
    """c_k = sum_{i != k} max(0, r(i,k))."""
    n = R.shape[0]
    c = np.empty(n)
    lib().apo_column_sums(n, np.ascontiguousarray(R, dtype=np.float64), c)
    return c


def avail_rows(Rnew, A, lam, rows) -> np.ndarray:
    """Eqs. (3), (4) with damping for the listed rows: A_next[rows] from (R_new, A)."""
    n = Rnew.shape[0]
    Rnew = np.ascontiguousarray(Rnew, dtype=np.float64)
    c = column_sums(Rnew)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.size, n))
    lib().apo_avail_rows(n, Rnew, c, np.ascontiguousarray(A, dtype=np.float64), lam, rows, rows.size, out)
    return out


def decisions(A: np.ndarray, R: np.ndarray) -> np.ndarray:
    n = A.shape[0]
    dec = np.empty(n, dtype=np.int32)
    lib().apo_decisions(n, np.ascontiguousarray(A, dtype=np.float64),
                        np.ascontiguousarray(R, dtype=np.float64), dec)
    return dec


def finalize(S: np.ndarray, dec: np.ndarray) -> dict:
    """Algorithm 1 outputs idx, dpsim, expref, netsim from raw decisions."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    n = S.shape[0]
    dec = np.ascontiguousarray(dec, dtype=np.int32)
    idx = np.empty(n, dtype=np.int32)
    dp, ep, ns = _dbl(), _dbl(), _dbl()
    nex = lib().apo_finalize(n, S, dec, idx, ctypes.byref(dp), ctypes.byref(ep), ctypes.byref(ns))
    return dict(idx=idx, n_exemplars=int(nex), dpsim=dp.value, expref=ep.value, netsim=ns.value)


def netsim_of_labels(S: np.ndarray, idx: np.ndarray) -> float:
    """-E(c) of Section 2 for a labelling: sum_i s(i, c_i)."""
    return float(S[np.arange(S.shape[0]), idx].sum())


# --------------------------------------------------------------------------
# Algorithm 2: partition AP
# --------------------------------------------------------------------------
def even_offsets(n: int, k: int) -> np.ndarray:
    """Algorithm 2, Step 1: k-1 parts of m = floor(n/k) and a last part of
    n - m(k-1)."""
    m = n // k
    off = [j * m for j in range(k)] + [n]
    return np.asarray(off, dtype=np.int64)


@dataclass
class PAPResult:
    full: APResult
    subs: list
    A_prime: np.ndarray


def pap(S: np.ndarray, k: int, perm: np.ndarray | None = None, offsets: np.ndarray | None = None,
        lam: float = 0.5, max_iter: int = 200, conv_iter: int = 15) -> PAPResult:
    """Algorithm 2.  Part j holds the points perm[offsets[j]:offsets[j+1]];
    AP runs on each diagonal block S_jj (which keeps the global preferences),
    the availabilities are placed block-diagonally in A' with zeros elsewhere,
    and AP runs on the whole S from A' (with R_0 = 0)."""
    n = S.shape[0]
    perm = np.arange(n, dtype=np.int64) if perm is None else np.asarray(perm, dtype=np.int64)
    offsets = even_offsets(n, k) if offsets is None else np.asarray(offsets, dtype=np.int64)
    assert offsets.size == k + 1 and offsets[0] == 0 and offsets[-1] == n
    A_prime = np.zeros((n, n))
    subs = []
    for j in range(k):
        members = perm[offsets[j]:offsets[j + 1]]
        Sjj = np.ascontiguousarray(S[np.ix_(members, members)])
        rj = ap(Sjj, lam, max_iter, conv_iter)
        subs.append(rj)
        A_prime[np.ix_(members, members)] = rj.A
    full = ap(S, lam, max_iter, conv_iter, A0=A_prime, R0=None)
    return PAPResult(full, subs, A_prime)


# --------------------------------------------------------------------------
# Algorithm 3 (Steps 1-2): landmark AP with nearest-exemplar assignment
# --------------------------------------------------------------------------
@dataclass
class LAPResult:
    landmark: APResult
    exemplars: np.ndarray   # global indices, ascending
    idx: np.ndarray         # (n,) labels
    dpsim: float
    expref: float
    netsim: float
    pref: float


def lap(X: np.ndarray, landmarks: np.ndarray, seed: int = 0, lam: float = 0.9,
        max_iter: int = 2000, conv_iter: int = 15, noise_rel: float = 1e-12,
        pref="median") -> LAPResult:
    """AP on the landmark points (preference: the median of the landmark
    similarities, or one given value; tie noise), then every point goes to
    its nearest exemplar by FP64 squared distance.  The landmark matrix lists
    the landmarks in ascending point index."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    M = np.sort(np.asarray(landmarks, dtype=np.int64))
    XM = np.ascontiguousarray(X[M])
    prep = prepare(similarity(XM), pref, seed, noise_rel)
    res = ap(prep.S, lam, max_iter, conv_iter)
    ex_local = res.exemplars
    ex = np.sort(M[ex_local]).astype(np.int64)
    n, d = X.shape
    idx = np.empty(n, dtype=np.int32)
    dp = _dbl()
    if ex.size == 0:
        idx[:] = -1
        return LAPResult(res, ex, idx, float("nan"), float("nan"), float("nan"), prep.pref)
    lib().apo_assign_nearest(n, d, X, d, ex.size, ex, idx, ctypes.byref(dp))
    expref = float(prep.pref) * ex.size
    return LAPResult(res, ex, idx, dp.value, expref, dp.value + expref, prep.pref)


def nearest_of(X: np.ndarray, query: np.ndarray, cand: np.ndarray):
    """For every query point (global indices), the nearest candidate point
    (ascending global indices) by FP64 squared distance, lowest index on
    ties: (labels int32, distances float64)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    q = np.ascontiguousarray(query, dtype=np.int64)
    c = np.ascontiguousarray(cand, dtype=np.int64)
    idx = np.empty(q.size, dtype=np.int32)
    dist = np.empty(q.size, dtype=np.float64)
    lib().apo_nearest_of(X.shape[1], X, X.shape[1], q.size, q, c.size, c, idx, dist)
    return idx, dist


def pair_dist(X: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """FP64 squared distances between points a[i] and b[i] (global indices)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    a = np.ascontiguousarray(a, dtype=np.int64)
    b = np.ascontiguousarray(b, dtype=np.int64)
    out = np.empty(a.size)
    lib().apo_pair_dist(X.shape[1], X, X.shape[1], a.size, a, b, out)
    return out


def medoid(X: np.ndarray, members: np.ndarray) -> int:
    """The member of least summed FP64 squared distance to all members
    (members ascending global indices; lowest index on ties)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    mem = np.ascontiguousarray(members, dtype=np.int64)
    return int(lib().apo_medoid(X.shape[1], X, X.shape[1], mem.size, mem))


def sqdist(x: np.ndarray, y: np.ndarray) -> float:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    return float(lib().apo_sqdist(x.size, x, y))
