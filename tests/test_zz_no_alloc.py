"""The allocation-free batched run (sf_batch_run_noalloc, for callers that
cannot allocate device memory) against
sf_batch_run on the same inputs (needs an MI355X): two calls in a row, the
second on fewer and smaller frames, each compared bit for bit (tableau, phase
vectors, amplitudes, outcomes), and the first also against the oracle.  The
allocator hook counts requests: the allocation-free calls make none."""
import numpy as np
import pytest

from oracle.frame import OracleFrame
from paper_1712_03554_amd import workloads as wl
from tests.oracle_helpers import assert_frames_equal, sigma_ints

pytestmark = pytest.mark.gpu


def _results(states):
    return [(st.read_frame(), st.outcomes()) for st in states]


def _same(a, b, what):
    (ta, sa, aa), oa = a
    (tb, sb, ab), ob = b
    assert np.array_equal(ta, tb) and np.array_equal(sa, sb), what
    assert np.array_equal(aa.view(np.uint64), ab.view(np.uint64)), what
    assert oa == ob, what


def test_noalloc_batch_matches_batch_run():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1712_03554_amd as sf
    requests = []
    eng = sf.Engine(0, refuse=lambda nbytes: requests.append(nbytes) and False)
    big = [wl.config2(0), wl.config1(1)] + [wl.config3(t) for t in range(40)] + \
          [wl.config4(j) for j in (3, 17, 250)] + [wl.random_clifford_t(200, 300, 3, 9100)]
    small = [wl.config1(4), wl.config3(41), wl.config4(5)]
    for calls, circs in enumerate((big, small)):
        seeds = [9000 + 31 * calls + i for i in range(len(circs))]
        loaded = [eng.load(c.n, c) for c in circs]
        ref_states = [lc.state(c.init_bits, s) for lc, c, s in zip(loaded, circs, seeds)]
        eng.batch_run(ref_states)
        want = _results(ref_states)
        states = [lc.state(c.init_bits, s) for lc, c, s in zip(loaded, circs, seeds)]
        print(f"case noalloc call {calls}: {len(circs)} frames", flush=True)
        before = len(requests)
        eng.batch_run_noalloc(states)
        assert len(requests) == before, "the allocation-free run asked the allocator for memory"
        got = _results(states)
        for c, a, b in zip(circs, got, want):
            _same(a, b, c.name)
        if calls == 0:
            for c, s, ((tab, sig, amp), out) in zip(circs, seeds, got):
                ref = OracleFrame(c.n, c.init_bits, s)
                ref.run(c.array())
                rtab, rsig, ramp = ref.read()
                assert np.array_equal(tab, rtab), c.name
                assert_frames_equal(sigma_ints(sig), amp, sigma_ints(rsig), ramp, what=c.name)
                assert out == ref.outcomes(), c.name
        for st in ref_states + states:
            st.close()
    eng.close()
