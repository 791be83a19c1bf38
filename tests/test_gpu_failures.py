"""Failure paths of the C ABI forced from the host (needs an MI355X): a
device allocator that refuses requests (SF_E_OOM) and a frame read into a
buffer that is too small (SF_E_BUFSIZE).  Every kernel still runs to its
normal end; the failures come from the host side only."""
import ctypes

import numpy as np
import pytest

from oracle.frame import OracleFrame
from paper_1712_03554_amd import workloads as wl
from tests.oracle_helpers import assert_frames_equal, sigma_ints

pytestmark = pytest.mark.gpu


def _engine(**kw):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1712_03554_amd as sf
    return sf.Engine(0, **kw)


def _superposed_t(n, k):
    """H then T on qubits 0..k-1: a frame of 2^k elements."""
    c = wl.Circuit(n, name=f"ht{k}-n{n}")
    for q in range(k):
        c.h(q)
    for q in range(k):
        c.t(q)
    c.cnot(0, n - 1)
    return c


def test_read_frame_reports_size_when_buffer_too_small():
    import paper_1712_03554_amd as sf
    eng = _engine()
    c = wl.random_clifford_t(20, 120, 4, 8101)
    st = eng.load(c.n, c).state(c.init_bits, 3)
    st.run()
    K = st.frame_size()
    assert K > 1
    W = 1
    tab = np.full((c.n, 2 * W), 0xAB, dtype=np.uint64)
    sig = np.full((K, W), 0xCD, dtype=np.uint64)
    amp = np.full(2 * K, 7.0)
    Kout = ctypes.c_size_t(0)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = eng._L.sf_read_frame(st._h, p(tab), p(sig), p(amp), K - 1, ctypes.byref(Kout))
    assert rc == sf.SF_E_BUFSIZE and Kout.value == K
    # nothing written
    assert np.all(tab == 0xAB) and np.all(sig == 0xCD) and np.all(amp == 7.0)
    # with room for K elements the read succeeds and matches the oracle
    rc = eng._L.sf_read_frame(st._h, p(tab), p(sig), p(amp), K, ctypes.byref(Kout))
    assert rc == sf.SF_OK and Kout.value == K
    ref = OracleFrame(c.n, c.init_bits, 3)
    ref.run(c.array())
    rtab, rsig, ramp = ref.read()
    assert np.array_equal(tab, rtab)
    assert_frames_equal(sigma_ints(sig), amp[0::2] + 1j * amp[1::2], sigma_ints(rsig), ramp, what="bufsize")
    st.close()
    eng.close()


def test_state_init_fails_with_oom_from_the_allocator():
    import paper_1712_03554_amd as sf
    eng = _engine(refuse=lambda nbytes: nbytes > (1 << 20))
    c = _superposed_t(30, 18)   # a frame bound of 2^18: 4 MiB per amplitude buffer
    lc = eng.load(c.n, c)
    assert lc.info()[0] == 18
    with pytest.raises(sf.SFrameError) as e:
        lc.state(c.init_bits, 1)
    assert e.value.status == sf.SF_E_OOM
    # the context still works for a state that fits
    small = wl.config1(0)
    st = eng.load(small.n, small).state(small.init_bits, 5)
    st.run()
    ref = OracleFrame(small.n, small.init_bits, 5)
    ref.run(small.array())
    assert st.outcomes() == ref.outcomes()
    st.close()
    eng.close()


def test_served_jobs_finish_when_one_cannot_allocate():
    """One job's device buffers cannot be had: with a large amplitude buffer
    it waits while others are resident and then fails; a wide frame whose
    per-gate record buffer is refused fails in the round that first needs it.
    Every other job finishes with the result it has alone, and later small
    jobs are admitted past the blocked one."""
    import paper_1712_03554_amd as sf
    limit = 8 << 20
    eng = _engine(refuse=lambda nbytes: nbytes > limit)
    ref_eng = _engine()
    big = _superposed_t(40, 22)                                            # 2^22 x 16 B amplitudes
    wide = wl.random_clifford_t(200, 1500, 3, 8104, name="wide-records")  # 1025 records of 13.5 KiB
    small = [wl.config1(0), wl.config3(1), wl.qft(6, [1, 0, 1, 1, 0, 1], max_k=6), wl.config1(3),
             wl.cuccaro_adder(2)]
    order = [small[0], big, small[1], wide, small[2], small[3], small[4]]
    seeds = [700 + i for i in range(len(order))]
    alone = {}
    for i, (c, s) in enumerate(zip(order, seeds)):
        if c in (big, wide):
            continue
        st = ref_eng.load(c.n, c).state(c.init_bits, s)
        st.run()
        alone[i] = (st.read_frame(), st.outcomes())
        st.close()
    loaded = [eng.load(c.n, c) for c in order]
    srv = sf.Server(eng, budget_bytes=0, max_resident=3)
    ids = [srv.submit(lc, c.init_bits, s) for lc, c, s in zip(loaded, order, seeds)]
    status = {}
    for _ in range(500):
        srv.tick()
        for i, jid in enumerate(ids):
            stt, st = srv.poll(jid)
            if stt in (sf.Server.DONE, sf.Server.FAILED) and i not in status:
                status[i] = (stt, (st.read_frame(), st.outcomes()) if st is not None else None)
        if len(status) == len(ids):
            break
    assert len(status) == len(ids)
    for i, c in enumerate(order):
        stt, res = status[i]
        if c in (big, wide):
            assert stt == sf.Server.FAILED, c.name
            continue
        assert stt == sf.Server.DONE, c.name
        (tab, sig, amp), out = res
        (ta, sa, aa), oa = alone[i]
        assert np.array_equal(tab, ta) and np.array_equal(sig, sa), c.name
        assert np.array_equal(amp.view(np.uint64), aa.view(np.uint64)), c.name
        assert out == oa, c.name
    for jid in ids:
        srv.release(jid)
    assert srv.stats()["used_bytes"] == 0
    srv.close()
    eng.close()
    ref_eng.close()
