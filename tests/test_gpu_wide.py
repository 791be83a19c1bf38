"""Wide frames (257..2048 qubits) on the device against the oracle (needs an
MI355X): stabilizer circuits only (section 6, random stabilizer circuits:
ceil(beta n log2 n) gates uniform over H, S, CNOT, then every qubit
measured), whose frames keep one element.  Tableau and phase vector
bit-exact, outcomes bit-exact, the amplitude within
|a - a_ref| <= 1e-10 |a_ref| + 1e-13."""
import numpy as np
import pytest

from oracle.frame import OracleFrame
from paper_1712_03554_amd import workloads as wl
from tests.oracle_helpers import assert_frame_arrays_equal, oracle_pool, oracle_stabilizer

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
    f.run(c.array())
    return f


def _check(st, ref, what):
    (rtab, rsig, ramp), routs, rfrag = ref
    tab, sig, amp = st.read_frame()
    assert np.array_equal(tab, rtab), f"{what}: tableau differs"
    assert_frame_arrays_equal(sig, amp, rsig, ramp, what=what)
    assert st.outcomes() == routs, f"{what}: outcomes differ"
    assert not rfrag and not st.info()[1], what
    assert st.frame_size() == 1


def _ref(c, seed):
    f = _oracle(c, seed)
    return f.read(), f.outcomes(), f.fragile


def random_clifford_mix(n, gates, n_meas, seed, measure_all=False):
    """Every Clifford gate kind (phase gates at multiples of pi/2 included)
    and measurements at random points, from a random basis state."""
    rng = np.random.default_rng(seed)
    c = wl.Circuit(n, rng.integers(0, 2, size=n).tolist(), name=f"mix-n{n}-{seed}")
    kinds = [wl.H, wl.S, wl.SDG, wl.X, wl.Y, wl.Z, wl.CNOT, wl.CZ, wl.PHASE]
    meas_at = set(rng.choice(gates, size=min(n_meas, gates), replace=False).tolist())
    for g in range(gates):
        if g in meas_at:
            c.measure(int(rng.integers(n)))
            continue
        op = kinds[int(rng.integers(len(kinds)))]
        a = int(rng.integers(n))
        if op in (wl.CNOT, wl.CZ):
            c.add(op, a, int((a + 1 + rng.integers(n - 1)) % n))
        elif op == wl.PHASE:
            c.phase(a, int(rng.choice([1, 2, 3, -1, 4])), 2)
        else:
            c.add(op, a)
    if measure_all:
        for q in range(n):
            c.measure(q)
    return c


@pytest.mark.parametrize("n", [257, 320, 511, 700])
def test_wide_mix_matches_oracle(eng, n):
    c = random_clifford_mix(n, 3 * n, n // 8, 7000 + n, measure_all=(n % 2 == 1))
    seed = 71 + n
    print(f"case {c.name} gates={len(c)}", flush=True)
    st = eng.load(c.n, c).state(c.init_bits, seed)
    assert st.circ.info()[0] == 0
    st.run()
    _check(st, _ref(c, seed), c.name)
    st.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n,beta", [(512, 1.0), (1024, 1.0), (2048, 0.08)])
def test_stabilizer_experiment_matches_oracle(eng, n, beta):
    """The section 6 workload at n = 512 and 1024 with beta = 1 (4608 and
    10240 gates, then n measurements), and a shorter one at n = 2048."""
    c = wl.stabilizer_circuit(n, 8100 + n, beta)
    seeds = [5 + n, 6 + n]
    print(f"case {c.name} gates={len(c)}", flush=True)
    with oracle_pool(2) as pool:
        futs = [pool.submit(oracle_stabilizer, n, 8100 + n, beta, s) for s in seeds]
        lc = eng.load(c.n, c)
        sts = [lc.state(c.init_bits, s) for s in seeds]
        eng.batch_run(sts)
        for st, fut, s in zip(sts, futs, seeds):
            _check(st, fut.result(), f"{c.name} seed {s}")
            st.close()


def test_gate_by_gate_wide(eng):
    """n = 300: the frame after each of the first 150 gates (single steps)."""
    c = random_clifford_mix(300, 150, 12, 7300)
    seed = 9
    f = OracleFrame(c.n, c.init_bits, seed)
    st = eng.load(c.n, c).state(c.init_bits, seed)
    for gi, g in enumerate(c.gates):
        f.apply(*g)
        assert st.step(1) == 1
        _check(st, (f.read(), f.outcomes(), f.fragile), f"gate {gi} {g}")
    st.close()


def test_wide_frames_in_a_batch_with_narrow_ones(eng):
    """Wide and narrow frames in one batched run give what each gives alone."""
    circs = [random_clifford_mix(257, 500, 20, 7401), wl.config1(3), random_clifford_mix(640, 900, 30, 7402),
             wl.config2(5), random_clifford_mix(1030, 700, 40, 7403, measure_all=True)]
    seeds = [11, 12, 13, 14, 15]
    alone = []
    for c, s in zip(circs, seeds):
        st = eng.load(c.n, c).state(c.init_bits, s)
        st.run()
        alone.append((st.read_frame(), st.outcomes()))
        st.close()
    sts = [eng.load(c.n, c).state(c.init_bits, s) for c, s in zip(circs, seeds)]
    eng.batch_run(sts)
    for st, (ref, outs), c in zip(sts, alone, circs):
        tab, sig, amp = st.read_frame()
        assert np.array_equal(tab, ref[0]) and np.array_equal(sig, ref[1]), c.name
        assert np.array_equal(amp.view(np.uint64), ref[2].view(np.uint64)), c.name
        assert st.outcomes() == outs, c.name
    for c, s, (ref, outs) in zip(circs, seeds, alone):
        if c.n > 256:
            _check_arrays(ref, outs, _ref(c, s), c.name)
    for st in sts:
        st.close()


def _check_arrays(got, outs, ref, what):
    (rtab, rsig, ramp), routs, rfrag = ref
    tab, sig, amp = got
    assert np.array_equal(tab, rtab), f"{what}: tableau differs"
    assert_frame_arrays_equal(sig, amp, rsig, ramp, what=what)
    assert outs == routs and not rfrag, what


def _steps(st, count):
    """Apply the next count circuit gates (a step ends after a measurement)."""
    done = 0
    while done < count:
        k = st.step(count - done)
        assert k > 0
        done += k
    assert st.info()[0] == count


def test_wide_adhoc_measure_and_reset(eng):
    """sf_measure between gates equals a measurement gate at that point, and a
    reset state runs again to the same frame."""
    c = random_clifford_mix(400, 600, 10, 7500)
    seed = 21
    lc = eng.load(c.n, c)
    st = lc.state(c.init_bits, seed)
    _steps(st, 250)
    o1 = st.measure(399)
    o2 = st.measure(0)
    st.run()
    ref_c = wl.Circuit(c.n, c.init_bits, "adhoc")
    ref_c.gates = c.gates[:250] + [(wl.MEASURE, 399, 0, 0, 0, 1), (wl.MEASURE, 0, 0, 0, 0, 1)] + c.gates[250:]
    ref = _ref(ref_c, seed)
    _check(st, ref, "adhoc")
    m0 = sum(1 for g in c.gates[:250] if g[0] == wl.MEASURE)
    assert [o1, o2] == ref[1][m0:m0 + 2]
    first = st.read_frame()
    bits = np.random.default_rng(3).integers(0, 2, size=c.n).tolist()
    st.reset(bits, 99)
    st.run()
    c2 = wl.Circuit(c.n, bits, "reset")
    c2.gates = list(c.gates)
    _check(st, _ref(c2, 99), "after reset")
    st.reset(c.init_bits, seed)
    _steps(st, 250)
    st.measure(399)
    st.measure(0)
    st.run()
    again = st.read_frame()
    assert np.array_equal(first[0], again[0]) and np.array_equal(first[1], again[1])
    assert np.array_equal(first[2].view(np.uint64), again[2].view(np.uint64))
    st.close()


EMBED = [(700, [0, 255, 256, 511, 512, 513, 640, 699]), (1100, [63, 64, 511, 512, 1023, 1024, 1025, 1099]),
         (2048, [0, 1, 1023, 1024, 1983, 1984, 2046, 2047])]


@pytest.mark.parametrize("case", range(len(EMBED)))
def test_narrow_stabilizer_circuit_spread_over_a_wide_register(eng, case):
    """A stabilizer circuit on 8 qubits placed across word boundaries of a
    wide register gives the narrow circuit's outcomes and amplitude."""
    N, pos = EMBED[case]
    small = random_clifford_mix(8, 160, 10, 7600 + case, measure_all=True)
    wide = wl.Circuit(N, name=f"spread-{N}")
    for q, p in enumerate(pos):
        wide.init_bits[p] = small.init_bits[q]
    for op, q0, q1, q2, num, den in small.gates:
        wide.add(op, pos[q0], pos[q1] if op in (wl.CNOT, wl.CZ) else 0, 0, num, den)
    seed = 31 + case
    st = eng.load(N, wide).state(wide.init_bits, seed)
    st.run()
    fs = _oracle(small, seed)
    assert st.outcomes() == fs.outcomes()
    _, _, amp = st.read_frame()
    _, _, ramp = fs.read()
    assert abs(amp[0] - ramp[0]) <= 1e-10 * abs(ramp[0]) + 1e-13
    _check(st, _ref(wide, seed), wide.name)
    st.close()


def test_wide_limits_and_refusals(eng):
    import paper_1712_03554_amd as sf
    # non-Clifford gates on more than 256 qubits
    c = wl.Circuit(300)
    c.h(0); c.t(0)
    with pytest.raises(sf.SFrameError) as e:
        eng.load(300, c)
    assert e.value.status == sf.SF_E_INVALID
    with pytest.raises(sf.SFrameError) as e:
        eng.load(2049, wl.Circuit(2049))
    assert e.value.status == sf.SF_E_INVALID
    # the batched forms that take narrow frames only
    w = random_clifford_mix(300, 50, 2, 7700)
    st = eng.load(w.n, w).state(w.init_bits, 1)
    for call in (lambda: eng.batch_reset([st], [w.init_bits], [1]), lambda: eng.batch_run_noalloc([st]),
                 lambda: eng.batch_graph([st])):
        with pytest.raises(sf.SFrameError) as e:
            call()
        assert e.value.status == sf.SF_E_INVALID
    srv = sf.Server(eng)
    with pytest.raises(sf.SFrameError) as e:
        srv.submit(st.circ, w.init_bits, 1)
    assert e.value.status == sf.SF_E_INVALID
    srv.close()
    # a full read into a buffer without room
    import ctypes
    st.run()
    K = ctypes.c_size_t(0)
    tab = np.zeros((w.n, 2 * st.W), dtype=np.uint64)
    rc = eng._L.sf_read_frame(st._h, tab.ctypes.data_as(ctypes.c_void_p), None, None, 0, ctypes.byref(K))
    assert rc == sf.SF_E_BUFSIZE and K.value == 1
    # the identity circuit: one element, amplitude 1, the basis bits
    idc = wl.Circuit(1500, [1, 0, 1] * 500)
    ist = eng.load(1500, idc).state(idc.init_bits, 0)
    ist.run()
    tab, sig, amp = ist.read_frame()
    ref = _ref(idc, 0)
    assert np.array_equal(tab, ref[0][0]) and np.array_equal(sig, ref[0][1]) and amp[0] == 1.0
    ist.close()
    st.close()
