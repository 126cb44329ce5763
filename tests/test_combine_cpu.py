"""Combining the aligned integrations of several streams (host logic, no
GPU): windows are joined only when every stream has delivered them, in
stream-id order along the channel axis, whatever order results arrive in."""

import numpy as np
import pytest

from paper_1503_06189_amd.serve import Combiner, IntegrationResult


def _res(sid, window, F, P=3, frames=2, fill=None):
    v = np.full((F, P, 2), sid * 100 + window if fill is None else fill, dtype=np.int32)
    return IntegrationResult(sid, window, frames, v, np.full(F, 10 * sid, dtype=np.int64),
                             v.astype(np.float32) / 2, 0.0, 2 * window, 2 * window + 1, window)


def test_join_in_stream_id_order_whatever_the_arrival_order():
    c = Combiner([9, 3, 4])
    assert c.add(_res(9, 0, F=1)) is None
    assert c.add(_res(4, 1, F=2)) is None
    assert c.add(_res(3, 0, F=3)) is None
    assert c.incomplete() == {0: [4], 1: [3, 9]}
    out = c.add(_res(4, 0, F=2))
    assert out is not None and out.window == 0
    assert out.stream_ids == [3, 4, 9] and out.channel_offsets == [0, 3, 5]
    assert out.vis.shape == (6, 3, 2)
    assert [int(x) for x in out.vis[:, 0, 0]] == [300, 300, 300, 400, 400, 900]
    assert [int(x) for x in out.count] == [30, 30, 30, 40, 40, 90]
    assert (out.seq_first, out.seq_last) == (0, 1)
    assert c.incomplete() == {1: [3, 9]}


def test_errors():
    c = Combiner([1, 2])
    with pytest.raises(KeyError):
        c.add(_res(5, 0, F=1))
    c.add(_res(1, 0, F=1))
    with pytest.raises(ValueError):
        c.add(_res(1, 0, F=1))            # the same window twice
    r = _res(2, 0, F=1)
    r.window = -1                          # not aligned
    with pytest.raises(ValueError):
        c.add(r)
    with pytest.raises(ValueError):
        c.add(_res(2, 0, F=1, P=6))        # another input count
    with pytest.raises(ValueError):
        Combiner([1, 1])
