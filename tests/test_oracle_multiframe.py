"""Pins of the multiframe oracle (section 4: COALESCE, merging frames with
equal matrices, Invariant 2 and orthogonalization) against the dense
definition and the paper's worked example:

* after every gate of random circuits (Clifford, T, phase gates, direct and
  decomposed Toffoli and controlled phase, measurements) the sum over all
  frames of a_j psi(M_i, sigma_j) equals the dense state vector, and the
  seeded outcomes equal the dense checker's;
* Example 4: a computational-basis frame with pairs differing on qubit 2 and
  on qubits 2, 3 coalesces into two one-element frames, one with H on
  column 2 and one with H on column 2 then CNOT on columns 2, 3, whose
  matrices share the row ZII (the intersection example);
* the orthogonality check agrees with dense inner products on random pairs
  of frames, and orthogonalization leaves one frame with the same vector;
* Cuccaro adders on superposed inputs (section 6): the multiframe ends with
  a number of states linear in the register width, far below the single
  frame, and measured afterwards every outcome is a consistent addition.
"""
import numpy as np
import pytest

from oracle import dense
from oracle.frame import OracleFrame, OracleMultiframe
from paper_1712_03554_amd import workloads as wl
from tests.oracle_helpers import sigma_ints, tableau_bits


def _vector(mf):
    n = mf.n
    psi = np.zeros(1 << n, dtype=complex)
    for tab, sig, amp in mf.frames():
        M = tableau_bits(tab, n)
        for s, a in zip(sigma_ints(sig), amp):
            psi += a * dense.canonical_state(M, [(s >> i) & 1 for i in range(n)], n)
    return psi


def _check_structure(mf):
    mats = []
    for tab, sig, amp in mf.frames():
        s = sigma_ints(sig)
        assert len(s) > 0 and s == sorted(s) and len(set(s)) == len(s)
        M = tableau_bits(tab, mf.n)
        assert np.array_equal(M, dense.rref(M)), "frame matrix not canonical"
        mats.append(tab.tobytes())
    assert len(set(mats)) == len(mats), "two frames share a matrix"


def _random_mix(seed, n, n_gates=28):
    rng = np.random.default_rng(seed)
    c = wl.Circuit(n, rng.integers(0, 2, size=n).tolist(), name=f"mf{seed}")
    for _ in range(n_gates):
        k = int(rng.integers(12))
        a, b, t = (int(v) for v in rng.permutation(n)[:3])
        if k < 3:
            c.add((wl.H, wl.S, wl.SDG)[k], a)
        elif k < 5:
            c.cnot(a, b)
        elif k == 5:
            c.t(a)
        elif k == 6:
            c.phase(a, int(rng.choice([1, -3, 5])), int(rng.choice([4, 8])))
        elif k == 7:
            c.add(wl.CPHASE_D, a, b, 0, 1, int(rng.choice([2, 4, 8])))
        elif k == 8:
            c.add(wl.TOF_D, a, b, t)
        elif k == 9:
            c.add(wl.TOF, a, b, t)
        elif k == 10:
            c.tdg(a)
        else:
            c.measure(a)
    return c


@pytest.mark.parametrize("general", [False, True])
@pytest.mark.parametrize("seed", range(10))
def test_multiframe_state_equals_dense_at_every_gate(seed, general):
    n = 3 + seed % 3
    c = _random_mix(seed, n)
    mf = OracleMultiframe(n, c.init_bits, seed)
    mf.set_general(general)
    vec = dense.basis_state(n, c.init_bits)
    nmeas = 0
    for gi, g in enumerate(c.gates):
        op, q0, q1, q2, num, den = g
        mf.apply(*g)
        if op == wl.MEASURE:
            p1 = dense.qubit_prob1(vec, n, q0)
            u = dense.measurement_u(seed, nmeas)
            nmeas += 1
            o = int(u < p1)
            assert mf.outcomes()[-1] == o, f"gate {gi}: outcome"
            vec = dense.project(vec, n, q0, o)
        else:
            vec = dense.apply_gate(vec, n, op, q0, q1, q2, num, den)
        _check_structure(mf)
        assert np.allclose(_vector(mf), vec, atol=1e-10), f"gate {gi} {g}"
    assert not mf.fragile


def _basis_frame_tab(n):
    tab = np.zeros((n, 2), dtype=np.uint64)
    for q in range(n):
        tab[q, 1] = np.uint64(1 << q)
    return tab


def test_example4_coalesces_into_two_frames():
    """Qubits 1, 2, 3 of the example are 0, 1, 2 here.  Pairs (000, 010) and
    (100, 111) have equal amplitudes within a pair and different moduli across
    pairs, so only the two intended pairs are candidates."""
    n = 3
    alpha, beta = 0.6 / np.sqrt(2), 0.8 / np.sqrt(2)
    states = {0b000: alpha, 0b010: alpha, 0b001: beta, 0b111: beta}   # bit q = qubit q
    sig = np.array([[s] for s in sorted(states)], dtype=np.uint64)
    amp = np.array([states[s] for s in sorted(states)], dtype=complex)
    mf = OracleMultiframe.load(n, _basis_frame_tab(n), sig, amp)
    want = _vector(mf)
    assert mf.coalesce() == 2
    assert mf.nframes == 2 and mf.size == 2
    assert np.allclose(_vector(mf), want, atol=1e-12)
    rows = []
    for tab, _, _ in mf.frames():
        M = tableau_bits(tab, n)
        rows.append({tuple(r) for r in M})
    zii = (0, 0, 0, 1, 0, 0)
    f1 = {zii, (0, 1, 0, 0, 0, 0), (0, 0, 0, 0, 0, 1)}            # ZII, IXI, IIZ
    f2 = {zii, (0, 1, 1, 0, 0, 0), (0, 0, 0, 0, 1, 1)}            # ZII, IXX, IZZ
    assert sorted(map(sorted, rows)) == sorted(map(sorted, [f1, f2]))
    # the intersection of the two matrices' rows is ZII
    assert rows[0] & rows[1] == {zii}
    assert mf.orthogonal()


def test_coalesce_with_phase_factor_uses_p():
    """A pair whose amplitudes differ by i coalesces through P H (d = 1):
    (|0> + i|1>)/sqrt2 on qubit 0 becomes one element with stabilizer Y."""
    n = 2
    sig = np.array([[0b00], [0b01]], dtype=np.uint64)
    amp = np.array([1 / np.sqrt(2), 1j / np.sqrt(2)])
    mf = OracleMultiframe.load(n, _basis_frame_tab(n), sig, amp)
    want = _vector(mf)
    assert mf.coalesce() == 1 and mf.nframes == 1 and mf.size == 1
    tab, s, a = mf.frames()[0]
    M = tableau_bits(tab, n)
    assert {tuple(r) for r in M} == {(1, 0, 1, 0), (0, 0, 0, 1)}   # Y on qubit 0, Z on qubit 1
    assert np.allclose(_vector(mf), want, atol=1e-12)


def _random_frame(rng, n, k):
    tr = dense.TableauTrack(n)
    for _ in range(5 * n):
        op = int(rng.integers(3))
        a = int(rng.integers(n))
        if op == 2 and n > 1:
            tr.conjugate(wl.CNOT, a, int((a + 1 + rng.integers(n - 1)) % n))
        else:
            tr.conjugate((wl.H, wl.S, wl.H)[op], a)
    M = tr.canonical()
    tab = np.zeros((n, 2), dtype=np.uint64)
    for i in range(n):
        tab[i, 0] = np.uint64(sum(int(M[i, q]) << q for q in range(n)))
        tab[i, 1] = np.uint64(sum(int(M[i, n + q]) << q for q in range(n)))
    sig = np.array(sorted({int(v) for v in rng.integers(0, 1 << n, size=k)}), dtype=np.uint64).reshape(-1, 1)
    amp = rng.standard_normal(len(sig)) + 1j * rng.standard_normal(len(sig))
    return M, tab, sig, amp


@pytest.mark.parametrize("seed", range(30))
def test_orthogonality_check_matches_inner_products(seed):
    rng = np.random.default_rng(seed)
    n = 2 + seed % 3
    Ma, ta, sa, aa = _random_frame(rng, n, 2)
    Mb, tb, sb, ab = _random_frame(rng, n, 2)
    mf = OracleMultiframe.load(n, ta, sa, aa)
    mf.add_frame(tb, sb, ab)
    if mf.nframes == 1:
        return  # equal matrices merged: nothing to check
    ortho = True
    for s in sigma_ints(sa):
        va = dense.canonical_state(Ma, [(s >> i) & 1 for i in range(n)], n)
        for t in sigma_ints(sb):
            vb = dense.canonical_state(Mb, [(t >> i) & 1 for i in range(n)], n)
            if abs(np.vdot(va, vb)) > 1e-9:
                ortho = False
    assert mf.orthogonal() == ortho
    want = _vector(mf)
    assert mf.orthogonalize() == (not ortho)
    assert mf.nframes == (1 if not ortho else 2)
    assert np.allclose(_vector(mf), want, atol=1e-10)


@pytest.mark.parametrize("direct", [False, True])
def test_cuccaro_multiframe_stays_small(direct):
    """Section 6: with multiframes the number of states of superposed Cuccaro
    adders (7-T Toffolis) at the end of the circuit grows linearly in the
    width while the single frame grows exponentially; with direct Toffolis
    the multiframe still stays below the single frame."""
    finals = []
    for m in range(1, 7):
        c = wl.cuccaro_adder(m, direct=direct)
        mf = OracleMultiframe(c.n, c.init_bits, 1)
        mf.run(c.array())
        sf = OracleFrame(c.n, c.init_bits, 1)
        sf.run(c.array())
        finals.append(mf.size)
        assert not mf.fragile
        if m >= 3:
            assert mf.size < sf.size
        if m <= 3:
            assert np.allclose(_vector(mf), _dense(c), atol=1e-10)
    if not direct:
        steps = np.diff(finals)
        assert np.all(steps == steps[0]) and steps[0] > 0, finals
    else:
        assert finals[-1] <= 2 ** 6


def _dense(c):
    vec = dense.basis_state(c.n, c.init_bits)
    for op, q0, q1, q2, num, den in c.gates:
        vec = dense.apply_gate(vec, c.n, op, q0, q1, q2, num, den)
    return vec


@pytest.mark.parametrize("m", [3, 5])
def test_cuccaro_multiframe_measured_adds(m):
    c = wl.cuccaro_adder(m, superpose=True)
    for q in range(c.n):
        c.measure(q)
    for seed in range(4):
        mf = OracleMultiframe(c.n, c.init_bits, seed)
        mf.run(c.array())
        outs = mf.outcomes()
        a = sum(outs[2 + 2 * i] << i for i in range(m))
        s = sum(outs[1 + 2 * i] << i for i in range(m))
        assert outs[0] == 0 and outs[2 * m + 1] == (1 if s < a else 0)
        assert mf.nframes == 1 and mf.size == 1
        sf = OracleFrame(c.n, c.init_bits, seed)
        sf.run(c.array())
        assert sf.outcomes() == outs


def test_cuccaro_general_coalescing_keeps_the_peak_polynomial():
    """With COALESCE extended through the basis circuit, the largest number
    of states during a superposed 7-T Cuccaro adder stays far below the
    basic form's (which doubles with every bit) and grows at most
    quadratically in the width; the final state equals the dense vector."""
    peaks = []
    for m in range(1, 7):
        c = wl.cuccaro_adder(m)
        mf = OracleMultiframe(c.n, c.init_bits, 1)
        mf.set_general(True)
        sizes, _ = mf.run(c.array())
        peaks.append(int(max(int(sizes.max()), mf.size)))
        if m <= 3:
            assert np.allclose(_vector(mf), _dense(c), atol=1e-10)
    assert all(p <= 3 * (m + 1) ** 2 for m, p in zip(range(1, 7), peaks)), peaks
