"""Validation of integration snapshots before anything reaches the device:
a snapshot of another element type, shape or an out-of-range sample count
is refused with ValueError (CPU only; no GPU call is made)."""

import numpy as np
import pytest

from paper_1503_06189_amd import xengine as xe


class _Shaped:
    """Stands in for an accumulator tensor: the checks read only .shape."""

    def __init__(self, shape):
        self.shape = shape


def _state(vis_dtype=np.int32, count_dtype=np.int64, samples=0, F=1, P=3):
    return {"vis": np.zeros((F, P, 2), vis_dtype), "count": np.zeros(F, count_dtype),
            "samples": samples}


@pytest.mark.parametrize("state,what", [
    (_state(vis_dtype=np.float32), "types"),
    (_state(count_dtype=np.int32), "types"),
    (_state(samples=-1), "samples"),
    (_state(samples=xe.XE_MAX_SAMPLES + 1), "samples"),
    (_state(F=2), "shape"),
])
def test_restore_refuses_bad_snapshots(state, what):
    with pytest.raises(ValueError, match=what):
        xe.restore(state, _Shaped((1, 3, 2)), _Shaped((1,)))
