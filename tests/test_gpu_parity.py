"""Parity of the HIP library with the CPU oracle (needs an MI355X).

Tableau and canonically ordered phase vectors bit-exact, seeded outcomes
bit-exact, complex128 amplitudes within |a - a_ref| <= 1e-10 |a_ref| + 1e-13.
"""
import numpy as np
import pytest

from oracle.frame import OracleFrame
from paper_1712_03554_amd import workloads as wl
from tests.oracle_helpers import assert_frames_equal, sigma_ints

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1712_03554_amd as sf
    return sf.Engine(0)


def _compare(st, ref, what):
    tab, sig, amp = st.read_frame()
    rtab, rsig, ramp = ref.read()
    assert np.array_equal(tab, rtab), f"{what}: tableau differs"
    assert_frames_equal(sigma_ints(sig), amp, sigma_ints(rsig), ramp, what=what)


def run_pair(eng, circ, seed, boundaries=()):
    """Run the circuit on the GPU and the oracle; compare at the listed gate
    counts (in the circuit's own gate units) and at the end."""
    print(f"case {circ.name} n={circ.n} gates={len(circ)} seed={seed}", flush=True)
    c = eng.load(circ.n, circ)
    st = c.state(circ.init_bits, seed)
    ref = OracleFrame(circ.n, circ.init_bits, seed)
    done = 0
    for b in sorted(set(boundaries)) + [len(circ)]:
        while done < b:
            k = st.step(b - done)
            assert k > 0
            for g in circ.gates[done:done + k]:
                ref.apply(*g)
            done += k
        _compare(st, ref, f"{circ.name} after {done} gates")
    assert st.outcomes() == ref.outcomes(), f"{circ.name}: outcomes differ"
    assert not ref.fragile
    _, frag = st.info()
    assert not frag
    return st, ref


def _mixed_circuit(seed, n, n_cliff=60, n_t=5, meas=True):
    rng = np.random.default_rng(seed)
    c = wl.random_clifford_t(n, n_cliff, n_t, 7000 + seed,
                             measure_qubits=rng.permutation(n)[: int(rng.integers(0, n + 1))] if meas else ())
    extra = [(wl.SDG, 0, 0, 0, 0, 1), (wl.X, n - 1, 0, 0, 0, 1), (wl.Y, 0, 0, 0, 0, 1), (wl.Z, 1, 0, 0, 0, 1),
             (wl.CZ, 0, 1, 0, 0, 1), (wl.TDG, 0, 0, 0, 0, 1), (wl.PHASE, 1, 0, 0, 1, 8),
             (wl.PHASE, 0, 0, 0, 3, 2), (wl.PHASE, 1, 0, 0, -5, 12), (wl.H, 1, 0, 0, 0, 1)]
    if meas:
        extra.append((wl.MEASURE, 1, 0, 0, 0, 1))
    for g in extra:
        c.gates.insert(int(rng.integers(0, len(c.gates))), g)
    c.name = f"mixed{seed}-n{n}"
    return c


@pytest.mark.parametrize("seed", range(16))
def test_random_small_circuits(eng, seed):
    n = 2 + seed % 9
    run_pair(eng, _mixed_circuit(seed, n), seed, boundaries=(5, 20, 41))


def test_gate_by_gate(eng):
    circ = _mixed_circuit(99, 5, n_cliff=40, n_t=4)
    run_pair(eng, circ, 3, boundaries=range(1, len(circ)))


@pytest.mark.parametrize("job", range(10))
def test_config1_all_seeds(eng, job):
    circ = wl.config1(job)
    run_pair(eng, circ, wl.derive_seed(1, job), boundaries=(100, 204))


def test_config1_matches_dense_vector(eng):
    from oracle import dense
    circ = wl.config1(0)
    seed = wl.derive_seed(1, 0)
    c = eng.load(circ.n, circ)
    st = c.state(circ.init_bits, seed)
    st.step(204)
    tab, sig, amp = st.read_frame()
    psi, M, _ = dense.simulate(8, circ.gates[:204])
    from tests.oracle_helpers import tableau_bits
    assert np.array_equal(tableau_bits(tab, 8), M)
    exp = dense.frame_expansion_fast(M, psi, 8)
    assert_frames_equal(sigma_ints(sig), amp, [s for s, _ in exp], [a for _, a in exp], what="cfg1 vs dense")


@pytest.mark.parametrize("trial", range(12))
def test_config3_steane_trials(eng, trial):
    run_pair(eng, wl.config3(trial), trial)


@pytest.mark.parametrize("n", [3, 6, 9])
def test_qft(eng, n):
    rng = np.random.default_rng(n)
    x = rng.integers(0, 2, size=n).tolist()
    run_pair(eng, wl.qft(n, x, max_k=6), 0)


def test_cuccaro_small(eng):
    run_pair(eng, wl.cuccaro_adder(2), 0)


def test_library_expands_tof_and_cphase(eng):
    base = wl.random_clifford_t(5, 20, 2, 11)
    base.add(wl.TOF, 0, 2, 4)
    base.add(wl.CPHASE, 1, 3, 0, 1, 4)
    base.add(wl.CPHASE, 4, 0, 0, -3, 8)
    base.add(wl.CPHASE, 2, 1, 0, 1, 1)
    base.name = "tof-cphase"
    run_pair(eng, base, 5)


@pytest.mark.parametrize("n", [63, 64, 65, 128, 150, 192, 200, 256])
def test_word_boundaries_and_max_qubits(eng, n):
    circ = wl.random_clifford_t(n, 4 * n, 6, 500 + n, measure_qubits=(0, n - 1, n // 2))
    cz_c = 63 % n if 63 % n != n - 1 else 0
    circ.add(wl.CNOT, n - 1, 0).add(wl.H, n - 1).add(wl.T, n - 1).add(wl.CZ, cz_c, n - 1)
    circ.name = f"wide{n}"
    run_pair(eng, circ, n)


@pytest.mark.parametrize("job", [0, 3, 5, 39, 42, 76])
def test_config4_circuits(eng, job):
    """Uneven-batch circuits at full size (up to 12 T gates, up to 232 qubits)."""
    run_pair(eng, wl.config4(job), job)


def test_config2_full_size(eng):
    circ = wl.config2(0)
    run_pair(eng, circ, wl.derive_seed(2, 0), boundaries=(1000,))


def test_edge_cases(eng):
    # no gates, n = 1
    c1 = wl.Circuit(1, name="empty")
    run_pair(eng, c1, 0)
    # only measurements on a basis state
    c2 = wl.Circuit(3, init_bits=[1, 0, 1], name="measure-only")
    for q in range(3):
        c2.measure(q)
    st, _ = run_pair(eng, c2, 0)
    assert st.outcomes() == [1, 0, 1]
    # Clifford angles of the phase gate and identity phases
    c3 = wl.Circuit(2, name="clifford-phases")
    c3.h(0).h(1).phase(0, 1, 2).phase(1, 2, 2).phase(0, -1, 2).phase(1, 4, 1).phase(0, 3, 2).t(1)
    run_pair(eng, c3, 0)
    # repeated measurement of the same qubit is deterministic
    c4 = wl.random_clifford_t(4, 20, 3, 77)
    c4.measure(2).measure(2).measure(2)
    c4.name = "remeasure"
    st, _ = run_pair(eng, c4, 9)
    o = st.outcomes()
    assert o[0] == o[1] == o[2]


def test_invalid_circuits_rejected(eng):
    import paper_1712_03554_amd as sf
    bad = [
        [(wl.H, 5, 0, 0, 0, 1)],
        [(wl.CNOT, 1, 1, 0, 0, 1)],
        [(wl.PHASE, 0, 0, 0, 1, 0)],
        [(99, 0, 0, 0, 0, 1)],
        [(wl.TOF, 0, 1, 1, 0, 1)],
    ]
    for gates in bad:
        c = wl.Circuit(3)
        c.gates = gates
        with pytest.raises(sf.SFrameError) as ei:
            eng.load(3, c)
        assert ei.value.status == sf.SF_E_INVALID
    with pytest.raises(sf.SFrameError):
        eng.load(0, wl.Circuit(1))
    with pytest.raises(sf.SFrameError):
        eng.load(2049, wl.Circuit(1))
    # more than 256 qubits: stabilizer circuits only
    c = wl.Circuit(257)
    c.t(3)
    with pytest.raises(sf.SFrameError) as ei:
        eng.load(257, c)
    assert ei.value.status == sf.SF_E_INVALID


def test_too_large_frame_rejected(eng):
    import paper_1712_03554_amd as sf
    c = wl.Circuit(40)
    for q in range(40):
        c.h(q)
    for q in range(32):
        c.t(q)
    with pytest.raises(sf.SFrameError) as ei:
        eng.load(40, c)
    assert ei.value.status == sf.SF_E_TOO_LARGE


def test_budget_rejects_state(eng):
    import paper_1712_03554_amd as sf
    small = sf.Engine(0, budget_bytes=1 << 16)
    c = wl.Circuit(20)
    for q in range(20):
        c.h(q)
    for q in range(14):
        c.t(q)
    circ = small.load(20, c)
    bound, need = circ.info()
    assert bound == 14 and need > (1 << 16)
    with pytest.raises(sf.SFrameError) as ei:
        circ.state()
    assert ei.value.status == sf.SF_E_TOO_LARGE


def test_frame_size_and_determinism(eng):
    circ = _mixed_circuit(5, 7, n_cliff=80, n_t=6)
    a, ref = run_pair(eng, circ, 42)
    assert a.frame_size() == ref.size
    c = eng.load(circ.n, circ)
    b = c.state(circ.init_bits, 42)
    b.run()
    ta, sa, aa = a.read_frame()
    tb, sb, ab = b.read_frame()
    assert np.array_equal(sa, sb) and np.array_equal(aa.view(np.uint64), ab.view(np.uint64))


def test_batch_matches_alone(eng):
    """Each frame's result in a batched run equals its result run alone (bit
    for bit: same kernels, same reduction shapes), and matches the oracle."""
    circs = [wl.config1(j) for j in range(4)] + [wl.config3(t) for t in range(6)] + \
            [_mixed_circuit(s, 3 + s) for s in range(4)] + [wl.config4(1)]
    seeds = list(range(100, 100 + len(circs)))
    alone = []
    for c, s in zip(circs, seeds):
        st = eng.load(c.n, c).state(c.init_bits, s)
        st.run()
        alone.append((st.read_frame(), st.outcomes()))
    loaded = [eng.load(c.n, c) for c in circs]
    states = [l.state(c.init_bits, s) for l, c, s in zip(loaded, circs, seeds)]
    eng.batch_run(states)
    for c, s, st, (fa, oa) in zip(circs, seeds, states, alone):
        tab, sig, amp = st.read_frame()
        assert np.array_equal(tab, fa[0]) and np.array_equal(sig, fa[1]), c.name
        assert np.array_equal(amp.view(np.uint64), fa[2].view(np.uint64)), c.name
        assert st.outcomes() == oa, c.name
        ref = OracleFrame(c.n, c.init_bits, s)
        ref.run(c.array())
        rtab, rsig, ramp = ref.read()
        assert np.array_equal(tab, rtab), c.name
        assert_frames_equal(sigma_ints(sig), amp, sigma_ints(rsig), ramp, what=c.name)
        assert st.outcomes() == ref.outcomes(), c.name


def _run_alone(eng, circ, seed):
    st = eng.load(circ.n, circ).state(circ.init_bits, seed)
    st.run()
    return st.read_frame(), st.outcomes()


@pytest.mark.parametrize("tick_segments", [0, 1, 3])
def test_serve_mix_matches_alone(eng, tick_segments):
    """Jobs that arrive while others run join the batch; each result equals
    the job run alone (bit for bit) and the oracle, whatever the tick slice."""
    import paper_1712_03554_amd as sf
    circs = [wl.config1(j) for j in range(3)] + [wl.config3(t) for t in range(3)] + \
            [_mixed_circuit(s, 4 + s) for s in range(3)] + [wl.qft(5, [1, 0, 1, 1, 0], max_k=6)] + \
            [wl.cuccaro_adder(3), wl.config5_job(4)]
    seeds = list(range(300, 300 + len(circs)))
    alone = [_run_alone(eng, c, s) for c, s in zip(circs, seeds)]
    loaded = [eng.load(c.n, c) for c in circs]
    srv = sf.Server(eng, budget_bytes=0, max_resident=4, tick_segments=tick_segments)
    ids, pending = {}, list(range(len(circs)))
    done = {}
    ticks = 0
    while len(done) < len(circs):
        for _ in range(2):  # two arrivals per tick
            if pending:
                i = pending.pop(0)
                ids[srv.submit(loaded[i], circs[i].init_bits, seeds[i])] = i
        srv.tick()
        ticks += 1
        for jid, i in list(ids.items()):
            stt, st = srv.poll(jid)
            if stt == sf.Server.DONE and i not in done:
                done[i] = (st.read_frame(), st.outcomes())
                srv.release(jid)
                del ids[jid]
        assert ticks < 2000
    for i, (c, s) in enumerate(zip(circs, seeds)):
        (tab, sig, amp), out = done[i]
        (ta, sa, aa), oa = alone[i]
        assert np.array_equal(tab, ta) and np.array_equal(sig, sa), c.name
        assert np.array_equal(amp.view(np.uint64), aa.view(np.uint64)), c.name
        assert out == oa, c.name
        ref = OracleFrame(c.n, c.init_bits, s)
        ref.run(c.array())
        rtab, rsig, ramp = ref.read()
        assert_frames_equal(sigma_ints(sig), amp, sigma_ints(rsig), ramp, what=c.name)
    st = srv.stats()
    assert st["admitted"] == len(circs) and st["used_bytes"] == 0


def test_serve_budget_cancel_and_rejection(eng):
    import paper_1712_03554_amd as sf
    c = wl.config1(0)
    lc = eng.load(c.n, c)
    need = lc.info()[1]
    srv = sf.Server(eng, budget_bytes=int(need * 1.5), max_resident=8)
    j1 = srv.submit(lc, c.init_bits, 1)
    j2 = srv.submit(lc, c.init_bits, 2)
    j3 = srv.submit(lc, c.init_bits, 3)
    r, q = srv.tick()
    assert (r, q) in ((1, 2), (0, 2))            # only one fits the budget
    srv.cancel(j2)                                # cancel a queued job
    assert srv.poll(j2)[0] == sf.Server.CANCELLED
    for _ in range(200):
        if srv.poll(j1)[0] == sf.Server.DONE:
            break
        srv.tick()
    assert srv.poll(j1)[0] == sf.Server.DONE
    assert srv.poll(j3)[0] == sf.Server.QUEUED    # still waiting: j1 holds the budget
    srv.release(j1)
    for _ in range(200):
        if srv.poll(j3)[0] == sf.Server.DONE:
            break
        srv.tick()
    assert srv.poll(j3)[0] == sf.Server.DONE
    (tab, sig, amp), out = _run_alone(eng, c, 3)
    stt, st = srv.poll(j3)
    assert np.array_equal(st.read_frame()[1], sig) and st.outcomes() == out
    srv.release(j3)
    # a job larger than the whole budget is refused at submission
    big = wl.Circuit(20)
    for q_ in range(20):
        big.h(q_)
    for q_ in range(20):
        big.t(q_)                                 # frame bound 2^20: 32 MiB of amplitudes
    lb = eng.load(20, big)
    small = sf.Server(eng, budget_bytes=1 << 20, max_resident=2)
    with pytest.raises(sf.SFrameError) as ei:
        small.submit(lb)
    assert ei.value.status == sf.SF_E_TOO_LARGE
    assert small.stats()["rejected"] == 1


@pytest.mark.parametrize("case", range(6))
def test_adhoc_measurement(eng, case):
    """sf_measure between gates equals a MEASURE gate inserted at that point
    (same outcome index, same frame) in the oracle."""
    import paper_1712_03554_amd as sf
    circ = [wl.config1(case), _mixed_circuit(40 + case, 5 + case), wl.config3(case),
            wl.qft(6, [1, 1, 0, 1, 0, 1], max_k=6), wl.config1(7), _mixed_circuit(50, 9)][case]
    rng = np.random.default_rng(900 + case)
    seed = 77 + case
    print(f"case adhoc {circ.name} n={circ.n} seed={seed}", flush=True)
    c = eng.load(circ.n, circ)
    st = c.state(circ.init_bits, seed)
    ref = OracleFrame(circ.n, circ.init_bits, seed)
    cuts = sorted(set(int(x) for x in rng.integers(0, len(circ) + 1, size=3)))
    done = 0
    for cut in cuts + [len(circ)]:
        while done < cut:
            k = st.step(cut - done)
            for g in circ.gates[done:done + k]:
                ref.apply(*g)
            done += k
        if cut < len(circ) or case % 2:
            for q in rng.permutation(circ.n)[:2]:
                o = st.measure(int(q))
                ref.apply(wl.MEASURE, int(q), 0, 0, 0, 1)
                assert o == ref.outcomes()[-1]
            _compare(st, ref, f"{circ.name} after ad-hoc measurements at {done}")
    assert st.outcomes() == ref.outcomes()
    _compare(st, ref, f"{circ.name} end")
    with pytest.raises(sf.SFrameError) as ei:
        st.measure(circ.n)
    assert ei.value.status == sf.SF_E_INVALID


def test_graph_replays_match_eager(eng):
    """A recorded batched run, replayed with new basis states and seeds, gives
    each frame the result of an eager run alone with the same inputs (bit for
    bit), replay after replay, with eager work between the replays."""
    import paper_1712_03554_amd as sf
    circs = [wl.config1(j) for j in range(3)] + [wl.config3(t) for t in range(3)] + \
            [_mixed_circuit(s, 4 + s) for s in range(3)] + [wl.config4(1), wl.qft(5, [0] * 5, max_k=6)]
    loaded = [eng.load(c.n, c) for c in circs]
    states = [l.state(c.init_bits, 0) for l, c in zip(loaded, circs)]
    g = eng.batch_graph(states, [c.init_bits for c in circs], [5] * len(circs))
    assert eng._L.sf_state_destroy(states[0]._h) == sf.SF_E_STATE
    rng = np.random.default_rng(4242)
    for rep in range(3):
        print(f"case graph replay {rep}", flush=True)
        bases = [c.init_bits if rep == 0 else rng.integers(0, 2, size=c.n).tolist() for c in circs]
        seeds = [int(rng.integers(0, 1 << 62)) for _ in circs]
        for i in range(len(circs)):
            g.set_input(i, bases[i], seeds[i])
        g.launch()
        for i, (c, st) in enumerate(zip(circs, states)):
            alone = loaded[i].state(bases[i], seeds[i])
            alone.run()
            ta, sa, aa = alone.read_frame()
            tb, sb, ab = st.read_frame()
            assert np.array_equal(ta, tb) and np.array_equal(sa, sb), (rep, c.name)
            assert np.array_equal(aa.view(np.uint64), ab.view(np.uint64)), (rep, c.name)
            assert alone.outcomes() == st.outcomes(), (rep, c.name)
            alone.close()
        ref = OracleFrame(circs[0].n, bases[0], seeds[0])
        ref.run(circs[0].array())
        _compare(states[0], ref, f"graph replay {rep}")
        assert states[0].outcomes() == ref.outcomes()
    g.close()
    for st in states:
        st.close()


def test_autotune_keeps_results(eng):
    """Launch shapes picked by the autotuner change no result bit."""
    circs = [wl.config1(2), _mixed_circuit(60, 8), wl.config2(0, n_t=10), wl.qft(9, [1, 0] * 4 + [1], max_k=6)]
    before = [_run_alone(eng, c, 31) for c in circs]
    choice = eng.autotune(0, 14)
    assert set(choice) == set(range(15))
    for d, (b, g, ms) in choice.items():
        assert b in (64, 128, 256) and 1 <= g <= 65535 and ms > 0
    after = [_run_alone(eng, c, 31) for c in circs]
    for c, ((ta, sa, aa), oa), ((tb, sb, ab), ob) in zip(circs, before, after):
        assert np.array_equal(ta, tb) and np.array_equal(sa, sb), c.name
        assert np.array_equal(aa.view(np.uint64), ab.view(np.uint64)), c.name
        assert oa == ob, c.name
    loaded = [eng.load(c.n, c) for c in circs]
    states = [l.state(c.init_bits, 31) for l, c in zip(loaded, circs)]
    eng.batch_run(states)
    for c, st, ((ta, sa, aa), oa) in zip(circs, states, before):
        tb, sb, ab = st.read_frame()
        assert np.array_equal(sa, sb) and np.array_equal(aa.view(np.uint64), ab.view(np.uint64)), c.name


def _direct_circuit(seed, n, n_cliff=40, n_t=2):
    rng = np.random.default_rng(seed)
    c = wl.random_clifford_t(n, n_cliff, n_t, 7700 + seed,
                             measure_qubits=rng.permutation(n)[: int(rng.integers(0, 3))])
    extra = []
    for _ in range(4):
        a, b, t = (int(v) for v in rng.permutation(n)[:3])
        extra.append((wl.TOF_D, a, b, t, 0, 1))
        num, den = [(1, 2), (1, 4), (-3, 8), (1, 1), (2, 1), (5, 6), (1, 32)][int(rng.integers(7))]
        extra.append((wl.CPHASE_D, a, t, 0, num, den))
    for g in extra:
        c.gates.insert(int(rng.integers(0, len(c.gates) + 1)), g)
    c.name = f"direct{seed}-n{n}"
    return c


@pytest.mark.parametrize("seed", range(12))
def test_direct_controlled_gates(eng, seed):
    """Direct controlled phase and Toffoli (double cofactor) against the oracle,
    compared after every gate for the first circuits."""
    circ = _direct_circuit(seed, 3 + seed % 6)
    run_pair(eng, circ, seed, boundaries=range(1, len(circ)) if seed < 4 else ())


@pytest.mark.parametrize("n", [6, 9])
def test_qft_direct(eng, n):
    x = [(i * 5 + 1) % 2 for i in range(n)]
    run_pair(eng, wl.qft(n, x, max_k=6, direct=True), n)


@pytest.mark.parametrize("m", [2, 3])
def test_cuccaro_direct(eng, m):
    run_pair(eng, wl.cuccaro_adder(m, direct=True), m)


@pytest.mark.parametrize("n", [70, 150, 200])
def test_direct_gates_wide(eng, n):
    circ = wl.random_clifford_t(n, 3 * n, 3, 880 + n, measure_qubits=(0, n - 1))
    circ.gates.insert(n, (wl.TOF_D, 0, n - 1, n // 2, 0, 1))
    circ.gates.insert(2 * n, (wl.CPHASE_D, n // 3, 63 % n, 0, 1, 4))
    circ.name = f"directwide{n}"
    run_pair(eng, circ, n)


def test_direct_in_batch_and_graph(eng):
    circs = [_direct_circuit(s, 5 + s % 3) for s in range(20, 26)] + [wl.cuccaro_adder(2, direct=True)]
    seeds = list(range(500, 500 + len(circs)))
    alone = [_run_alone(eng, c, s) for c, s in zip(circs, seeds)]
    loaded = [eng.load(c.n, c) for c in circs]
    states = [l.state(c.init_bits, s) for l, c, s in zip(loaded, circs, seeds)]
    eng.batch_run(states)
    for c, st, ((ta, sa, aa), oa) in zip(circs, states, alone):
        tb, sb, ab = st.read_frame()
        assert np.array_equal(sa, sb) and np.array_equal(aa.view(np.uint64), ab.view(np.uint64)), c.name
        assert st.outcomes() == oa, c.name
    g = eng.batch_graph(states, [c.init_bits for c in circs], seeds)
    g.launch()
    for c, st, ((ta, sa, aa), oa) in zip(circs, states, alone):
        tb, sb, ab = st.read_frame()
        assert np.array_equal(sa, sb) and np.array_equal(aa.view(np.uint64), ab.view(np.uint64)), c.name
    g.close()


def test_batch_reset_matches_single_resets(eng):
    """One-launch re-initialisation equals per-state resets (bit for bit)."""
    circs = [wl.config1(j) for j in range(3)] + [wl.config3(t) for t in range(3)] + [wl.config4(1)]
    rng = np.random.default_rng(77)
    bases = [rng.integers(0, 2, size=c.n).tolist() for c in circs]
    seeds = [int(rng.integers(0, 1 << 62)) for _ in circs]
    loaded = [eng.load(c.n, c) for c in circs]
    states = [l.state(c.init_bits, 0) for l, c in zip(loaded, circs)]
    eng.batch_run(states)                      # dirty the states first
    eng.batch_reset(states, bases, seeds)
    eng.batch_run(states)
    for l, c, st, b, s in zip(loaded, circs, states, bases, seeds):
        alone = l.state(b, s)
        alone.run()
        ta, sa, aa = alone.read_frame()
        tb, sb, ab = st.read_frame()
        assert np.array_equal(ta, tb) and np.array_equal(sa, sb), c.name
        assert np.array_equal(aa.view(np.uint64), ab.view(np.uint64)), c.name
        assert alone.outcomes() == st.outcomes(), c.name


def test_api_error_paths(eng):
    """Invalid calls of the newer entry points fail cleanly and leave the
    states usable."""
    import ctypes
    import paper_1712_03554_amd as sf
    L = eng._L
    c = wl.config1(0)
    lc = eng.load(c.n, c)
    st = lc.state(c.init_bits, 9)
    # autotune: bad ranges
    for lo, hi in ((-1, 3), (5, 4), (0, 30)):
        assert L.sf_autotune(eng._h, lo, hi, None, None, None) == sf.SF_E_INVALID
    # graph: input index out of range; a state in a graph cannot be destroyed
    g = eng.batch_graph([st], [c.init_bits], [9])
    assert L.sf_graph_set_input(g._h, 1, None, ctypes.c_uint64(0)) != sf.SF_OK
    assert L.sf_state_destroy(st._h) == sf.SF_E_STATE
    g.launch()
    g.close()
    # the same state twice in one graph is refused
    arr = (ctypes.c_void_p * 2)(st._h.value, st._h.value)
    out = ctypes.c_void_p()
    assert L.sf_batch_graph(eng._h, ctypes.cast(arr, ctypes.c_void_p), 2, None, None, ctypes.byref(out)) \
        == sf.SF_E_INVALID
    # a state of another context is refused by the batched calls
    eng2 = sf.Engine(0)
    arr1 = (ctypes.c_void_p * 1)(st._h.value)
    assert L.sf_batch_run(eng2._h, ctypes.cast(arr1, ctypes.c_void_p), 1) == sf.SF_E_INVALID
    assert L.sf_batch_reset(eng2._h, ctypes.cast(arr1, ctypes.c_void_p), 1, None, None) == sf.SF_E_INVALID
    eng2.close()
    # the state still runs to the oracle's result
    st.reset(c.init_bits, 9)
    st.run()
    ref = OracleFrame(c.n, c.init_bits, 9)
    ref.run(c.array())
    _compare(st, ref, "after error paths")


@pytest.mark.parametrize("n", [40, 100])
def test_long_ranges_same_segments_on_every_path(eng, n):
    """Circuits longer than two device ranges (frames of up to 128 qubits are
    tracked in ranges of at most 1024 gates): the plain, batched and graph
    paths form the same segments, so their frames agree bit for bit; a run in
    small steps (more range ends) agrees within the amplitude bound; all
    match the oracle.  A measurement sits just after the first range end."""
    circ = wl.random_clifford_t(n, 2600, 12, 8800 + n, measure_qubits=(3, 10, n - 1))
    circ.gates.insert(1030, (wl.MEASURE, 7, 0, 0, 0, 1))
    circ.name = f"long-n{n}"
    seed = 77 + n
    print(f"case {circ.name} gates={len(circ)}", flush=True)
    lc = eng.load(circ.n, circ)
    plain = lc.state(circ.init_bits, seed)
    plain.run()
    tp, sp, ap = plain.read_frame()
    batched = lc.state(circ.init_bits, seed)
    eng.batch_run([batched])
    tb, sb, ab = batched.read_frame()
    assert np.array_equal(tp, tb) and np.array_equal(sp, sb)
    assert np.array_equal(ap.view(np.uint64), ab.view(np.uint64))
    assert plain.outcomes() == batched.outcomes()
    gs = lc.state(circ.init_bits, 0)
    g = eng.batch_graph([gs], [circ.init_bits], [seed])
    g.launch()
    tg, sg, ag = gs.read_frame()
    assert np.array_equal(tp, tg) and np.array_equal(sp, sg)
    assert np.array_equal(ap.view(np.uint64), ag.view(np.uint64))
    assert plain.outcomes() == gs.outcomes()
    g.close()
    stepped = lc.state(circ.init_bits, seed)
    while stepped.step(37):
        pass
    ref = OracleFrame(circ.n, circ.init_bits, seed)
    ref.run(circ.array())
    _compare(plain, ref, f"{circ.name} plain")
    _compare(stepped, ref, f"{circ.name} stepped")
    assert plain.outcomes() == ref.outcomes() == stepped.outcomes()
    for st in (plain, batched, gs, stepped):
        st.close()


@pytest.mark.parametrize("n", [100, 200])
def test_stabilizer_circuits_keep_one_element(eng, n):
    """The paper's Clifford-only workload (n log2 n random H/S/CNOT, then every
    qubit measured): the frame keeps one element throughout, and tableau,
    amplitude and outcomes match the oracle."""
    circ = wl.stabilizer_circuit(n, 9100 + n)
    seed = 13 + n
    print(f"case {circ.name} gates={len(circ)}", flush=True)
    st = eng.load(circ.n, circ).state(circ.init_bits, seed)
    done = 0
    while True:
        k = st.step(max(1, len(circ) // 7))
        if not k:
            break
        done += k
        assert st.frame_size() == 1, done
    ref = OracleFrame(circ.n, circ.init_bits, seed)
    ref.run(circ.array())
    _compare(st, ref, circ.name)
    assert st.outcomes() == ref.outcomes()
    st.close()


def _wide_frames(count):
    """count frames of 129..256 qubits, alternately three and four words."""
    circs = []
    for j in range(count):
        n = 129 + (j * 37) % 64 + (64 if j % 2 else 0)
        c = wl.random_clifford_t(n, n, 1 + j % 4, 9100 + j,
                                 measure_qubits=(j % n, n - 1) if j % 3 == 0 else ())
        c.name = f"batchwide{j}-n{n}"
        circs.append(c)
    return circs


def test_many_wide_frames_in_one_batch(eng):
    """More wide frames (n > 128) in one batched launch than take the split
    track: they evaluate the phase factors inside the track kernel.  Each
    result equals the same frame run alone (split track) bit for bit and
    matches the oracle."""
    circs = _wide_frames(136)
    seeds = [300 + j for j in range(len(circs))]
    print(f"case batch of {len(circs)} wide frames", flush=True)
    loaded = [eng.load(c.n, c) for c in circs]
    states = [l.state(c.init_bits, s) for l, c, s in zip(loaded, circs, seeds)]
    eng.batch_run(states)
    for j, (c, s, st) in enumerate(zip(circs, seeds, states)):
        tab, sig, amp = st.read_frame()
        if j % 16 < 2:
            (ta, sa, aa), oa = _run_alone(eng, c, s)
            assert np.array_equal(tab, ta) and np.array_equal(sig, sa), c.name
            assert np.array_equal(amp.view(np.uint64), aa.view(np.uint64)), c.name
            assert st.outcomes() == oa, c.name
        ref = OracleFrame(c.n, c.init_bits, s)
        ref.run(c.array())
        rtab, rsig, ramp = ref.read()
        assert np.array_equal(tab, rtab), c.name
        assert_frames_equal(sigma_ints(sig), amp, sigma_ints(rsig), ramp, what=c.name)
        assert st.outcomes() == ref.outcomes(), c.name


@pytest.mark.parametrize("count", [6, 136])
def test_graph_with_wide_frames(eng, count):
    """The graph form of a batch of wide frames (split track for a few of
    them, in-kernel phase evaluation for more than 64 of one word count)
    gives the eager batched results bit for bit, on two replays with new
    inputs."""
    import paper_1712_03554_amd as sf
    circs = _wide_frames(count) + [wl.config3(1), _mixed_circuit(3, 6)]
    loaded = [eng.load(c.n, c) for c in circs]
    states = [l.state(c.init_bits, 0) for l, c in zip(loaded, circs)]
    g = eng.batch_graph(states, [c.init_bits for c in circs], [7] * len(circs))
    rng = np.random.default_rng(77 + count)
    for rep in range(2):
        print(f"case graph of {count} wide frames, replay {rep}", flush=True)
        bases = [rng.integers(0, 2, size=c.n).tolist() for c in circs]
        seeds = [int(rng.integers(0, 1 << 62)) for _ in circs]
        for i in range(len(circs)):
            g.set_input(i, bases[i], seeds[i])
        g.launch()
        eager = [l.state(b, s) for l, b, s in zip(loaded, bases, seeds)]
        eng.batch_run(eager)
        for c, st, e in zip(circs, states, eager):
            ta, sa, aa = e.read_frame()
            tb, sb, ab = st.read_frame()
            assert np.array_equal(ta, tb) and np.array_equal(sa, sb), (rep, c.name)
            assert np.array_equal(aa.view(np.uint64), ab.view(np.uint64)), (rep, c.name)
            assert e.outcomes() == st.outcomes(), (rep, c.name)
            e.close()
        i = rep * 3
        ref = OracleFrame(circs[i].n, bases[i], seeds[i])
        ref.run(circs[i].array())
        _compare(states[i], ref, f"graph of wide frames, replay {rep}")
        assert states[i].outcomes() == ref.outcomes()
    g.close()
    for st in states:
        st.close()


def test_small_frames_same_alone_and_in_mixed_rounds(eng):
    """Frames whose hull stays within 256 slots run their element stage in one
    block when alone (or batched only with such frames) and through the
    separate segment and measurement launches when batched with a larger
    frame; both give the same bits (one reduction block either way)."""
    small = [wl.config1(j) for j in range(3)] + [wl.config3(t) for t in range(3)] + \
            [_mixed_circuit(s, 4 + s) for s in range(2)]
    big = wl.random_clifford_t(20, 200, 14, 4242, measure_qubits=(0, 5, 19))  # frame reaches 512
    big.name = "big20"
    assert eng.load(big.n, big).info()[0] > 8
    for c in small:
        assert eng.load(c.n, c).info()[0] <= 8, c.name
    seeds = list(range(700, 700 + len(small) + 1))
    alone = [_run_alone(eng, c, s) for c, s in zip(small, seeds)]
    for with_big in (False, True):
        circs = small + ([big] if with_big else [])
        loaded = [eng.load(c.n, c) for c in circs]
        states = [l.state(c.init_bits, s) for l, c, s in zip(loaded, circs, seeds)]
        print(f"case small frames batched, with a larger frame: {with_big}", flush=True)
        eng.batch_run(states)
        for c, st, ((ta, sa, aa), oa) in zip(small, states, alone):
            tb, sb, ab = st.read_frame()
            assert np.array_equal(ta, tb) and np.array_equal(sa, sb), (with_big, c.name)
            assert np.array_equal(aa.view(np.uint64), ab.view(np.uint64)), (with_big, c.name)
            assert st.outcomes() == oa, (with_big, c.name)
        for st in states:
            st.close()


def test_tuning_roundtrip_and_results_independent_of_it(eng, tmp_path):
    """The launch tuning can be read, changed, saved and loaded; invalid
    values are refused without change; batched results are bit-identical
    under very different tunings (one gate per phase wavefront, small and
    large element-kernel grids)."""
    import paper_1712_03554_amd as sf
    t0 = eng.tuning()
    assert len(t0["blocks"]) == 31 and t0["phase_waves"] >= 1
    circs = [wl.config2(j) for j in range(3)] + [wl.config3(t) for t in range(5)]
    seeds = [wl.derive_seed(2, j) for j in range(3)] + [wl.derive_seed(3, t) for t in range(5)]
    results = []
    for tun in (t0, {"blocks": [64] * 31, "grids": [1] * 31, "phase_waves": 1},
                {"blocks": [256] * 31, "grids": [4096] * 31, "phase_waves": 1 << 20}):
        eng.set_tuning(tun)
        assert eng.tuning()["phase_waves"] == tun["phase_waves"]
        sts = [eng.load(c.n, c).state(c.init_bits, s) for c, s in zip(circs, seeds)]
        eng.batch_run(sts)
        results.append([(st.read_frame(), st.outcomes()) for st in sts])
        for st in sts:
            st.close()
    for other in results[1:]:
        for (a, oa), (b, ob) in zip(results[0], other):
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
            assert np.array_equal(a[2].view(np.uint64), b[2].view(np.uint64)) and oa == ob
    # refused without change
    eng.set_tuning(t0)
    for bad in ({"blocks": [96] * 31, "grids": [1] * 31, "phase_waves": 8},
                {"blocks": [64] * 31, "grids": [0] * 31, "phase_waves": 8}, {"phase_waves": 0}):
        with pytest.raises(sf.SFrameError) as e:
            eng.set_tuning(bad)
        assert e.value.status == sf.SF_E_INVALID
        assert eng.tuning() == t0
    # saved and loaded (a file from another kind of device is ignored)
    path = str(tmp_path / "tuning.json")
    eng.set_tuning({"blocks": [128] * 31, "grids": [7] * 31, "phase_waves": 123})
    eng.save_tuning(path)
    eng.set_tuning(t0)
    assert eng.load_tuning(path) and eng.tuning()["phase_waves"] == 123 and eng.tuning()["grids"] == [7] * 31
    import json
    rec = json.load(open(path))
    rec["device"] = "another device"
    json.dump(rec, open(path, "w"))
    eng.set_tuning(t0)
    assert not eng.load_tuning(path) and eng.tuning() == t0


def test_batch_mixes_large_and_small_hulls(eng):
    """Frames whose hulls differ by many orders of magnitude in one batch (a
    superposed Cuccaro adder growing to 2^16 slots beside 13-qubit trials and
    8-qubit circuits): each frame's blocks in the flattened element launches
    and each measurement's reduction shape are its own, so the eager batched
    run and the graph replay give every frame's result alone, bit for bit."""
    circs = [wl.cuccaro_adder(7, name="cuccaro-m7"), wl.config1(0), wl.config3(3), wl.config3(11),
             _mixed_circuit(41, 12), wl.qft(11, [1, 0] * 5 + [1], name="qft-11"), wl.config1(5)]
    seeds = list(range(900, 900 + len(circs)))
    alone = [_run_alone(eng, c, s) for c, s in zip(circs, seeds)]
    loaded = [eng.load(c.n, c) for c in circs]
    assert max(l.info()[0] for l in loaded) >= 14
    states = [l.state(c.init_bits, s) for l, c, s in zip(loaded, circs, seeds)]
    eng.batch_run(states)
    for c, st, ((ta, sa, aa), oa) in zip(circs, states, alone):
        tb, sb, ab = st.read_frame()
        assert np.array_equal(ta, tb) and np.array_equal(sa, sb), c.name
        assert np.array_equal(aa.view(np.uint64), ab.view(np.uint64)), c.name
        assert st.outcomes() == oa, c.name
    g = eng.batch_graph(states, [c.init_bits for c in circs], seeds)
    for _ in range(2):
        g.launch()
        for c, st, ((ta, sa, aa), oa) in zip(circs, states, alone):
            tb, sb, ab = st.read_frame()
            assert np.array_equal(sa, sb) and np.array_equal(aa.view(np.uint64), ab.view(np.uint64)), c.name
            assert st.outcomes() == oa, c.name
    g.close()
    # the reference values of the small frames are the oracle's
    for c, s, ((ta, sa, aa), oa) in list(zip(circs, seeds, alone))[1:5]:
        ref = OracleFrame(c.n, c.init_bits, s)
        ref.run(c.array())
        rtab, rsig, ramp = ref.read()
        assert np.array_equal(ta, rtab), c.name
        assert_frames_equal(sigma_ints(sa), aa, sigma_ints(rsig), ramp, what=c.name)
        assert oa == ref.outcomes(), c.name
