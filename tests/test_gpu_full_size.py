"""The benchmark workloads at full size, in the launch configuration the
benchmark times (one batched reset and one batched run of every frame, and
the graph form), checked against the oracle (needs an MI355X).

* 3 random Clifford+T circuits, n = 128, 2000 Cliffords + 16 T, 16
  measurements: every frame against the oracle; and 1024 of them in one
  batch (the headline step as the benchmark times it): 16 against the
  oracle, all against size-independent properties.
* 4096 Steane fault-injection trials: every trial against the oracle.
* 1024 uneven random Clifford+T circuits (n in 16..256, up to 12 T): every
  frame against the oracle (run in a process pool while the GPU works), and
  every frame's norm and size bound.
* The large frame (Cuccaro adder, m = 12, on an equal superposition: 2^26
  elements): every qubit measured afterwards gives a consistent addition.

Eager and graph results agree bit for bit on every frame.
"""
import numpy as np
import pytest

from oracle.frame import OracleFrame
from paper_1712_03554_amd import workloads as wl
from tests.oracle_helpers import (assert_frame_arrays_equal, assert_frames_equal, oracle_config2, oracle_config4,
                                  oracle_pool, sigma_ints)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1712_03554_amd as sf
    return sf.Engine(0)


def _full_batch(eng, circs, seeds):
    """Batched reset + run of all frames, then the graph form with the same
    inputs (checked equal bit for bit); returns the eager results per frame:
    ((tableau, sigma, amplitudes), outcomes, fragile flag)."""
    import paper_1712_03554_amd as sf
    loaded = [eng.load(c.n, c) for c in circs]
    states = [l.state(c.init_bits, s) for l, c, s in zip(loaded, circs, seeds)]
    batch = sf.StateBatch(states)
    nmax = max(c.n for c in circs)
    bases = np.zeros((len(circs), nmax), dtype=np.uint8)
    for i, c in enumerate(circs):
        bases[i, :c.n] = np.asarray(c.init_bits, dtype=np.uint8)
    seed_arr = np.asarray(seeds, dtype=np.uint64)
    # run once from other inputs so that the reset has state to clear
    eng.batch_run(batch)
    eng.batch_reset(batch, bases, seed_arr)
    eng.batch_run(batch)
    eager = [(st.read_frame(), st.outcomes(), st.info()[1]) for st in states]
    g = eng.batch_graph(states, [c.init_bits for c in circs], seeds)
    g.launch()
    for i, (c, st) in enumerate(zip(circs, states)):
        (ta, sa, aa), oa, _ = eager[i]
        tb, sb, ab = st.read_frame()
        assert np.array_equal(ta, tb) and np.array_equal(sa, sb), c.name
        assert np.array_equal(aa.view(np.uint64), ab.view(np.uint64)), c.name
        assert st.outcomes() == oa, c.name
    g.close()
    for st in states:
        st.close()
    return eager


def _check_oracle(c, seed, res):
    (tab, sig, amp), outs, frag = res
    assert not frag, c.name
    ref = OracleFrame(c.n, c.init_bits, seed)
    ref.run(c.array())
    rtab, rsig, ramp = ref.read()
    assert not ref.fragile, c.name
    assert np.array_equal(tab, rtab), c.name
    assert_frames_equal(sigma_ints(sig), amp, sigma_ints(rsig), ramp, what=c.name)
    assert outs == ref.outcomes(), c.name


def test_random_clifford_t_n128_full_batch(eng):
    circs = [wl.config2(j) for j in range(3)]
    seeds = [wl.derive_seed(2, j) for j in range(3)]
    print("case 3 x n=128 Clifford+T circuits, batched and graph", flush=True)
    eager = _full_batch(eng, circs, seeds)
    for c, s, res in zip(circs, seeds, eager):
        assert len(res[1]) == 16, c.name
        _check_oracle(c, s, res)


@pytest.mark.timeout(600)
def test_random_clifford_t_n128_device_filling_batch(eng):
    """The headline step as the benchmark times it: 1024 circuits in one
    batched run (and its graph form, equal bit for bit); 16 of them against
    the oracle (in a process pool while the GPU works), every one against the
    properties that hold at any size: 16 outcomes, norm 1, at most 2^16
    elements, no fragile outcome."""
    circs = [wl.config2(j) for j in range(1024)]
    seeds = [wl.derive_seed(2, j) for j in range(1024)]
    sample = list(range(0, 1024, 64))
    print("case 1024 x n=128 Clifford+T circuits, batched and graph", flush=True)
    with oracle_pool() as pool:
        futs = {j: pool.submit(oracle_config2, j) for j in sample}
        eager = _full_batch(eng, circs, seeds)
        for j, (c, res) in enumerate(zip(circs, eager)):
            (tab, sig, amp), outs, frag = res
            assert len(outs) == 16 and not frag, c.name
            assert 1 <= len(amp) <= 1 << 16, c.name
            assert abs(float(np.sum(amp.real ** 2 + amp.imag ** 2)) - 1.0) <= 1e-12, c.name
        for j in sample:
            (tab, sig, amp), outs, frag = eager[j]
            rtab, rsig, ramp, routs, rfrag = futs[j].result()
            assert not rfrag, circs[j].name
            assert np.array_equal(tab, rtab), circs[j].name
            assert_frame_arrays_equal(sig, amp, rsig, ramp, what=circs[j].name)
            assert outs == routs, circs[j].name


def test_steane_trials_full_batch(eng):
    circs = [wl.config3(t) for t in range(4096)]
    seeds = [wl.derive_seed(3, t) for t in range(4096)]
    print("case 4096 Steane trials, batched and graph", flush=True)
    eager = _full_batch(eng, circs, seeds)
    for c, s, res in zip(circs, seeds, eager):
        amp = res[0][2]
        assert 1 <= len(amp) <= 2, c.name
        assert len(res[1]) == 6, c.name
        _check_oracle(c, s, res)


@pytest.mark.timeout(600)
def test_uneven_batch_full_size(eng):
    circs = [wl.config4(j) for j in range(1024)]
    seeds = [wl.derive_seed(4, j) for j in range(1024)]
    print("case 1024 uneven circuits, batched and graph; oracle in a process pool", flush=True)
    with oracle_pool() as pool:
        futs = [pool.submit(oracle_config4, j) for j in range(1024)]
        eager = _full_batch(eng, circs, seeds)
        for j, (c, res, fut) in enumerate(zip(circs, eager, futs)):
            (tab, sig, amp), outs, frag = res
            n_t = sum(1 for g in c.gates if g[0] in (wl.T, wl.TDG))
            assert 1 <= len(amp) <= 2 ** n_t, c.name
            assert abs(float(np.sum(amp.real ** 2 + amp.imag ** 2)) - 1.0) <= 1e-12, c.name
            assert not frag, c.name
            rtab, rsig, ramp, routs, rfrag = fut.result()
            assert not rfrag, c.name
            assert np.array_equal(tab, rtab), c.name
            assert_frame_arrays_equal(sig, amp, rsig, ramp, what=c.name)
            assert outs == routs, c.name


@pytest.mark.parametrize("seed", [11, 12])
def test_cuccaro_adder_m12_superposed_measured(eng, seed):
    """The large-frame workload at its full size (Cuccaro adder of two 12-bit
    registers on an equal superposition: a frame of 2^26 elements), checked by
    a property that holds at any size: measured afterwards, every outcome is
    a consistent addition (sum register s = a + b mod 2^m, carry = [s < a],
    ancilla 0), and one element of modulus 1 remains."""
    m = 12
    c = wl.cuccaro_adder(m, superpose=True, name=f"cuccaro{m}-measured")
    for q in range(c.n):
        c.add(wl.MEASURE, q)
    print(f"case {c.name} seed={seed}", flush=True)
    lc = eng.load(c.n, c)
    assert lc.info()[0] >= 2 * m
    st = lc.state(c.init_bits, seed)
    st.run()
    outs = st.outcomes()
    assert len(outs) == c.n
    a = sum(outs[2 + 2 * i] << i for i in range(m))
    s = sum(outs[1 + 2 * i] << i for i in range(m))
    assert outs[0] == 0
    assert outs[2 * m + 1] == (1 if s < a else 0)
    _, _, amp = st.read_frame()
    assert len(amp) == 1 and abs(abs(amp[0]) - 1.0) <= 1e-10
    assert not st.info()[1]
    st.close()
