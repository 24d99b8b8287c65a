"""Host logic of the learned warm start: the fallback rule on residual histories
(forced from the host; no GPU work)."""
import numpy as np

from paper_1701_04685_amd.warmstart import residual_grew


def test_fallback_rule():
    dec = np.geomspace(1e-1, 1e-3, 10)
    assert not residual_grew(dec, 10)
    assert residual_grew(dec[::-1], 10)
    # a bump that settles below the first residual is kept
    assert not residual_grew(np.array([1e-2, 3e-2, 2e-2, 5e-3]), 4)
    # growth, infinities and an empty history fall back
    assert residual_grew(np.array([1e-2, 5e-3, 2e-2]), 3)
    assert residual_grew(np.array([1e-2, np.inf]), 2)
    assert residual_grew(np.array([np.nan, np.nan]), 2)
    # entries after the solve stopped (NaN) are ignored
    assert not residual_grew(np.array([1e-2, 1e-7, np.nan, np.nan]), 4)
    # only the first `check` entries count
    assert not residual_grew(np.concatenate([dec, [1.0]]), 10)
