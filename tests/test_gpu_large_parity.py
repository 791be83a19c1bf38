"""Parity with the oracle on frames of millions of elements (needs an
MI355X): a hull of dimension 23 (the element kernels at their largest grid,
where the measurement reduction and the segment and filter loops stride), the
approximate QFT of the served mix at its largest size (n = 20, AQFT k <= 6)
and the exact QFT on |1...1> at n = 20, whose frame has 2^(n-1) elements
(section 6) of equal modulus (Eq. 4 is a product state of equal-weight
factors).  Frames are compared element by element: phase vectors bit-exact,
amplitudes within |a - a_ref| <= 1e-10 |a_ref| + 1e-13, outcomes bit-exact."""
import numpy as np
import pytest

from oracle.frame import OracleFrame
from paper_1712_03554_amd import workloads as wl
from tests.oracle_helpers import assert_frame_arrays_equal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1712_03554_amd as sf
    return sf.Engine(0)


def _oracle(c, seed):
    f = OracleFrame(c.n, c.init_bits, seed)
    sizes = f.run(c.array())
    return f, sizes


def _check(st, ref, what):
    tab, sig, amp = st.read_frame()
    rtab, rsig, ramp = ref.read()
    assert np.array_equal(tab, rtab), f"{what}: tableau differs"
    assert_frame_arrays_equal(sig, amp, rsig, ramp, what=what)
    assert st.outcomes() == ref.outcomes(), f"{what}: outcomes differ"
    assert not ref.fragile and not st.info()[1], what
    return amp


def hull23_circuit():
    """24 qubits: H and T on qubits 0..21 (2^22 elements), H.T on qubit 22
    (the hull grows to 2^23), H.T on it again (partner pairs merge in
    place over all 2^23 slots), mixing Cliffords, a deterministic T, then
    three measurements."""
    c = wl.Circuit(24, name="hull23")
    for q in range(22):
        c.h(q)
    for q in range(22):
        c.t(q)
    c.h(22); c.t(22)
    c.h(22); c.t(22)
    c.cnot(0, 23); c.h(23); c.cnot(5, 17); c.s(3); c.h(7); c.cnot(21, 1); c.t(3); c.h(2)
    c.measure(4); c.measure(22); c.measure(11)
    return c


@pytest.mark.timeout(300)
def test_hull_of_dimension_23_plain_and_batched(eng):
    c = hull23_circuit()
    seed = 2301
    print(f"case {c.name} plain and batched", flush=True)
    ref, sizes = _oracle(c, seed)
    assert int(sizes.max()) == 1 << 23
    lc = eng.load(c.n, c)
    assert lc.info()[0] == 23
    st = lc.state(c.init_bits, seed)
    st.run()
    _check(st, ref, "hull23 plain")
    # batched beside a small frame: the batched segment and measurement kernels
    small = wl.config1(2)
    s2 = eng.load(small.n, small).state(small.init_bits, 17)
    st.reset(c.init_bits, seed)
    eng.batch_run([st, s2])
    _check(st, ref, "hull23 batched")
    ref2, _ = _oracle(small, 17)
    _check(s2, ref2, "small beside hull23")
    st.close()
    s2.close()


@pytest.mark.parametrize("direct", [False, True])
def test_aqft_n20_matches_oracle(eng, direct):
    """Config 5(a) at its largest size: approximate QFT (k <= 6) on 20 qubits
    from a random basis state, controlled rotations as three phase gates or
    in direct form, then every qubit measured."""
    rng = np.random.default_rng(2020)
    x = rng.integers(0, 2, size=20).tolist()
    c = wl.qft(20, x, max_k=6, name=f"aqft20-{'direct' if direct else 'decomposed'}", direct=direct)
    pre = wl.Circuit(20, c.init_bits, c.name)
    pre.gates = list(c.gates)
    print(f"case {c.name}", flush=True)
    lc = eng.load(pre.n, pre)
    st = lc.state(pre.init_bits, 41)
    st.run()
    ref, _ = _oracle(pre, 41)
    amp = _check(st, ref, c.name)
    assert len(amp) == 1 << 19
    # measured afterwards: same outcomes, one element left
    for q in range(20):
        c.measure(q)
    lm = eng.load(c.n, c)
    sm = lm.state(c.init_bits, 43)
    sm.run()
    refm, _ = _oracle(c, 43)
    _check(sm, refm, c.name + " measured")
    assert sm.frame_size() == 1
    st.close()
    sm.close()


@pytest.mark.parametrize("direct", [True, False])
def test_qft_on_all_ones_n20_has_half_size_frame(eng, direct):
    """Exact QFT on |1...1> at n = 20: 2^19 elements, all of modulus
    2^(-19/2), and the oracle's frame element by element."""
    n = 20
    c = wl.qft(n, [1] * n, name=f"qft20-ones-{'direct' if direct else 'decomposed'}", direct=direct)
    print(f"case {c.name}", flush=True)
    st = eng.load(c.n, c).state(c.init_bits, 5)
    st.run()
    assert st.frame_size() == 1 << (n - 1)
    ref, _ = _oracle(c, 5)
    amp = _check(st, ref, c.name)
    assert np.allclose(np.abs(amp), 2.0 ** (-(n - 1) / 2), rtol=1e-12, atol=0)
    st.close()
