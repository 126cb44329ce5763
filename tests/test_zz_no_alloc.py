"""The allocation-free accumulate (xe_accumulate_noalloc) against the
accumulate that uses the handle's workspace (GPU).

Two calls in a row on the same static scratch array, the second with a
smaller frame, each into sums that already hold an integration: the sums
and counts must equal those of xe_accumulate bit for bit, and the oracle's.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_1503_06189_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def xe():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_06189_amd import xengine
    xengine.lib()
    return xengine


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# (N, F, T, B): both chunked in time, so both use the scratch array; the
# second is smaller and leaves the first call's partials behind it
CASES = [(256, 16, 8192, 256), (96, 3, 5000, 64)]


def test_noalloc_matches_workspace_accumulate(xe):
    orc = oracle.load()
    for k, (N, F, T, B) in enumerate(CASES):
        plan = xe.plan_query(N, F, T, B)
        assert plan.splits > 1, "the case must go through the scratch array"
        _say(f"noalloc call {k}: N={N} F={F} T={T} B={B} chunks={plan.splits}")
        fr = synth.random_bytes_frame(500 + k, N, F, T, B, p_loss=0.1, fill="garbage")
        prior = synth.random_bytes_frame(600 + k, N, F, 300, B, p_loss=0.0)
        packed, mask = _dev(fr.packed), _dev(fr.mask)
        start_v, start_n = xe.correlate_frame(_dev(prior.packed), None, B)
        v1, n1 = start_v.clone(), start_n.clone()
        v2, n2 = start_v.clone(), start_n.clone()
        xe.reset_integration(v1)
        xe.reset_integration(v2)
        xe.accumulate(packed, mask, B, v1, n1)
        xe.accumulate_noalloc(packed, mask, B, v2, n2)
        torch.cuda.synchronize()
        assert torch.equal(n1, n2), f"call {k}: counts differ"
        assert torch.equal(v1, v2), f"call {k}: sums differ"
        ev, en = orc.correlate(fr.packed, fr.mask, B)
        pv, pn = orc.correlate(prior.packed, None, B)
        assert np.array_equal(v2.cpu().numpy(), ev + pv), f"call {k}: sums vs oracle"
        assert np.array_equal(n2.cpu().numpy(), en + pn), f"call {k}: counts vs oracle"


def test_noalloc_unchunked_and_repeated(xe):
    """A frame with enough channels needs no chunks (nothing in scratch);
    repeated calls keep adding."""
    orc = oracle.load()
    N, F, T, B = 64, 300, 700, 100
    assert xe.plan_query(N, F, T, B).splits == 1
    fr = synth.random_bytes_frame(700, N, F, T, B, p_loss=0.2)
    packed, mask = _dev(fr.packed), _dev(fr.mask)
    vis, cnt = xe.new_accumulators(N, F, packed.device)
    for _ in range(3):
        xe.accumulate_noalloc(packed, mask, B, vis, cnt)
    torch.cuda.synchronize()
    ev, en = orc.correlate(fr.packed, fr.mask, B)
    assert np.array_equal(vis.cpu().numpy(), 3 * ev)
    assert np.array_equal(cnt.cpu().numpy(), 3 * en)
