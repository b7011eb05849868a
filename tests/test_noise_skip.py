"""The tie noise may be skipped where it cannot change an FP32 entry.

The similarity kernels add fl32((double)v + scale * u), u in [0, 1), to every
off-diagonal entry, and skip the counter generator when scale <= |v| 2^-27:
the claim is that the rounded sum is then v itself.  Checked here in the
kernels' arithmetic (FP64 sum, one rounding to FP32) at the bound, for
random entries, powers of two of both signs (where the spacing below |v|
halves), the largest and the subnormal floats, and u just below 1.
"""
import numpy as np


def _noisy(v, scale, u):
    return (v.astype(np.float64) + scale * u).astype(np.float32)


def test_skip_bound_keeps_every_entry():
    rng = np.random.default_rng(7)
    v = np.concatenate([
        rng.standard_normal(200000).astype(np.float32) * np.float32(1e3),
        (rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000)).astype(np.float32),
        np.ldexp(1.0, np.arange(-126, 128)).astype(np.float32),
        -np.ldexp(1.0, np.arange(-126, 128)).astype(np.float32),
        np.array([np.finfo(np.float32).max, -np.finfo(np.float32).max,
                  np.finfo(np.float32).tiny, -np.finfo(np.float32).tiny,
                  np.float32(1e-45), np.float32(-1e-45)], dtype=np.float32),
    ])
    v = v[np.isfinite(v) & (v != 0)]
    scale = np.abs(v.astype(np.float64)) * 2.0 ** -27          # the largest skipped scale
    for u in (0.0, 0.5, 1.0 - 2.0 ** -53):
        assert np.array_equal(_noisy(v, scale, u), v)


def test_bound_is_not_vacuous():
    # a scale far above the bound does move entries: the bound is what
    # decides, not the size of the noise alone
    v = np.float32([1.0, -1.0, 3.0, -1000.0])
    scale = np.abs(v.astype(np.float64)) * 2.0 ** -20
    assert not np.array_equal(_noisy(v, scale, 1.0 - 2.0 ** -53), v)
