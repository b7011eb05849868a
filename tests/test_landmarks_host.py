"""Host-side pieces that need no GPU: the landmark set of apx_lap_landmarks
(kept points plus a SplitMix64-driven uniform sample of the others), checked
against the oracle's independent implementation of the same published
generator, and the pair metrics of the evaluation on a hand-worked case."""
import os

import numpy as np
import pytest

from oracle import lap_full as LF

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_0910_1650_amd", "libapx.so")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libapx.so not built")
def test_landmarks_keep_and_sample_like_the_oracle():
    import paper_0910_1650_amd as apx
    n, L = 5000, 300
    keep = np.array([3, 17, 4000, 4999, 250], dtype=np.int64)
    M = apx.apx_lap_landmarks(n, L, keep, seed=77)
    assert M.size == L and np.all(np.diff(M) > 0) and np.all(np.isin(keep, M))
    rest = np.setdiff1d(np.arange(n), keep)
    ref = np.sort(np.concatenate([keep, rest[LF.sample_positions(rest.size, L - keep.size, 77)]]))
    assert np.array_equal(M, ref)
    # no kept points: the same draw the top level of the landmark method uses
    assert np.array_equal(apx.apx_lap_landmarks(n, L, None, seed=5), LF.sample_positions(n, L, 5))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libapx.so not built")
def test_landmarks_reject_bad_arguments():
    import paper_0910_1650_amd as apx
    with pytest.raises(apx.ApxError):
        apx.apx_lap_landmarks(10, 3, np.array([1, 1]), 0)
    with pytest.raises(apx.ApxError):
        apx.apx_lap_landmarks(10, 2, np.array([1, 2, 3]), 0)
    with pytest.raises(apx.ApxError):
        apx.apx_lap_landmarks(10, 11, None, 0)


def test_association_rates_hand_example():
    from paper_0910_1650_amd.experiments import association_rates
    truth = [0, 0, 0, 1, 1, 2]
    labels = [5, 5, 7, 7, 7, 9]
    # same-class pairs: 3 + 1 = 4, of which together: (0,1) and (3,4) -> 2
    # different-class pairs: 15 - 4 = 11, of which together: (2,3), (2,4) -> 2
    tar, far = association_rates(truth, labels)
    assert tar == 2 / 4 and far == 2 / 11
