"""Algorithm 3 (landmark affinity propagation), Steps 1-4, for the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Composed from the
oracle's Algorithm 1 (``oracle.ap``), similarity, preference/noise and FP64
nearest-candidate routines, in the paper's step order (Section 4):

Step 1  AP on the landmark set M gives the centres C1 and the landmarks'
        classes.
Step 2  max_distance(c) is the largest distance of a landmark of class c to
        its centre; every other point goes to its nearest centre c if its
        distance is below max_distance(c), and otherwise stays unassigned.
Step 3  The m unassigned points: AP on them when m <= m0, the whole method
        on them when m > m0; their centres join C1.
Step 4  Every point goes to its nearest merged centre, and each class's
        centre becomes the class member of least summed distance to the
        class (its medoid); every point then goes to the nearest refined
        centre.

Readings where the paper leaves a choice (the GPU library takes the same):
* "distance" is the squared Euclidean distance, -s(i,k); ties go to the
  lowest index; "below" is strict, so a class of one landmark takes nothing.
* The preference p of the top level's landmark AP (the median of the
  landmark similarities, or a given value) is used by every later AP.
* Step 4 ("refine the final set of centers and classes ... obtain the best
  final results") is one round of: classes by nearest merged centre, each
  class's medoid as its centre (for fixed classes the member that maximises
  the class's similarity sum, the energy of Section 2), and the labels by
  nearest refined centre.  (AP on the bare centres, another reading, ignores
  how many points each centre stands for; with the same preference it
  merged 26 centres of a 10-component 2-D set into 5 and lowered the net
  similarity from -5163 to -36295, where the medoid round raised it to
  -4234.)  Exemplars label themselves.  A recursive call is the whole
  method, Step 4 included, and returns its refined centres.
* Below the top, the m > m0 case draws min(L, m0) landmarks uniformly
  without replacement from the unassigned points: a partial Fisher-Yates
  shuffle of their positions driven by the SplitMix64 stream (Steele, Lea,
  Flood 2014) seeded with the level's seed.  The top level uses the given
  landmarks, or the same draw over all points with `seed`.
* Tie noise of each AP (Section 2 reading of the preference/noise): at
  recursion level l, Step 1 uses seed + 3l, Step 3's AP seed + 3l + 1 and
  Step 4's AP seed + 3l + 2.
* m = 1 (or one merged centre) needs no message passing: the point is its
  own exemplar.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import ap, medoid, nearest_of, pair_dist, prepare, similarity

_MASK = (1 << 64) - 1


def splitmix64_stream(seed: int):
    """The SplitMix64 generator: state += golden gamma, then the output
    function on the state."""
    state = seed & _MASK
    while True:
        state = (state + 0x9E3779B97F4A7C15) & _MASK
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        yield z ^ (z >> 31)


def sample_positions(m: int, count: int, seed: int) -> np.ndarray:
    """`count` distinct positions of 0..m-1 (ascending): the first `count`
    slots of a Fisher-Yates shuffle driven by the SplitMix64 stream."""
    pool = list(range(m))
    g = splitmix64_stream(seed)
    for i in range(count):
        j = i + next(g) % (m - i)
        pool[i], pool[j] = pool[j], pool[i]
    return np.sort(np.asarray(pool[:count], dtype=np.int64))


def _ap_centres(X, pts, pref, seed, lam, max_iter, conv_iter, noise_rel):
    """AP on the points `pts` (ascending global indices): (centres, the AP
    result, the preference used)."""
    if pts.size == 1:
        return pts.copy(), None, pref
    prep = prepare(similarity(X[pts]), pref, seed, noise_rel)
    r = ap(prep.S, lam, max_iter, conv_iter)
    return pts[r.exemplars], r, prep.pref


@dataclass
class LevelStats:
    level: int
    points: int
    landmarks: int
    step1_centres: int
    step1_iterations: int
    assigned: int
    unassigned: int
    step3: str              # "none", "ap", "lap"
    merged: int
    refined: int


@dataclass
class LAPFullResult:
    exemplars: np.ndarray
    idx: np.ndarray
    dpsim: float
    expref: float
    netsim: float
    pref: float
    levels: list = field(default_factory=list)


def step2(X, Q, M, C1, cls):
    """Algorithm 3, Step 2: max_distance(c) over the landmarks M of class c
    (cls[i]: landmark i's centre), then each point of Q goes to its nearest
    centre of C1 if strictly closer than that centre's max_distance.
    Returns (assigned flags over Q, the unassigned points U)."""
    if C1.size == 0 or Q.size == 0:
        return np.zeros(Q.size, dtype=bool), Q
    maxd = {int(c): 0.0 for c in C1}
    for c, dd in zip(cls, pair_dist(X, M, cls)):
        maxd[int(c)] = max(maxd[int(c)], float(dd))
    lab, dist = nearest_of(X, Q, C1)
    limit = np.array([maxd[int(c)] for c in lab])
    assigned = dist < limit
    return assigned, Q[~assigned]


def classes(X, P, C):
    """Nearest centre of every point of P (centres label themselves)."""
    lab, _ = nearest_of(X, P, C)
    isc = np.isin(P, C)
    lab[isc] = P[isc]
    return lab


def refine(X, P, C):
    """Step 4: classes of P by nearest centre of C, each class's medoid."""
    lab = classes(X, P, C)
    E = [medoid(X, P[lab == c]) for c in C if np.any(lab == c)]   # members ascending
    return np.unique(np.asarray(E, dtype=np.int64))


def _level(X, P, M, level, seed, lam, max_iter, conv_iter, m0, L, pref, noise_rel, stats):
    # Step 1: AP on the landmarks
    C1, r1, p = _ap_centres(X, M, pref, seed + 3 * level, lam, max_iter, conv_iter, noise_rel)
    # Step 2: per-class largest landmark distance, then the other points
    Q = np.setdiff1d(P, M, assume_unique=True)
    cls = (M[r1.idx] if r1 is not None else M) if C1.size > 0 else None
    assigned, U = step2(X, Q, M, C1, cls)
    # Step 3
    if U.size == 0:
        C3, how = np.zeros(0, dtype=np.int64), "none"
    elif U.size <= m0:
        C3, _, _ = _ap_centres(X, U, p, seed + 3 * level + 1, lam, max_iter, conv_iter, noise_rel)
        how = "ap"
    else:
        Lr = min(L, m0)
        Mr = U[sample_positions(U.size, Lr, seed + 3 * (level + 1))]
        C3 = _level(X, U, Mr, level + 1, seed, lam, max_iter, conv_iter, m0, L, p, noise_rel, stats)
        how = "lap"
    C = np.union1d(C1, C3).astype(np.int64)
    # Step 4: classes by nearest merged centre, then each class's medoid
    E = refine(X, P, C) if C.size > 0 else C
    stats.append(LevelStats(level, int(P.size), int(M.size), int(C1.size),
                            r1.iterations if r1 is not None else 0, int(assigned.sum()), int(U.size), how,
                            int(C.size), int(E.size)))
    if level == 0:
        stats.sort(key=lambda s: s.level)
    return (E, p) if level == 0 else E


def lap_full(X: np.ndarray, landmarks: np.ndarray | None, L: int, seed: int = 0, lam: float = 0.9,
             max_iter: int = 2000, conv_iter: int = 15, m0: int = 20000, pref="median",
             noise_rel: float = 1e-12) -> LAPFullResult:
    """Algorithm 3, Steps 1-4, on points X (n x d FP32)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n = X.shape[0]
    M = (np.sort(np.asarray(landmarks, dtype=np.int64)) if landmarks is not None
         else sample_positions(n, L, seed))
    stats: list = []
    E, p = _level(X, np.arange(n, dtype=np.int64), M, 0, seed, lam, max_iter, conv_iter, m0, L, pref,
                  noise_rel, stats)
    if E.size == 0:
        return LAPFullResult(E, np.full(n, -1, dtype=np.int32), float("nan"), float("nan"), float("nan"),
                             p, stats)
    idx, dist = nearest_of(X, np.arange(n, dtype=np.int64), E)
    idx[E] = E
    dist[E] = 0.0
    dpsim = -float(np.sum(dist[np.setdiff1d(np.arange(n), E)]))
    expref = float(p) * E.size
    return LAPFullResult(E, idx, dpsim, expref, dpsim + expref, float(p), stats)
