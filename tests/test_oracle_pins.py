"""Pins of the CPU oracles against what the paper and the mathematics fix.

The frame oracle (oracle/frame.c) is checked against the worked examples and
tables of Garcia & Markov, against the dense state-vector definition
(oracle/dense.py: the exact state expanded in the canonical stabilizer basis),
closed forms and invariants.  The dense checker itself is pinned by gate
identities, Table 2 via explicit matrix conjugation and the QFT closed form.
"""
import ctypes
import itertools
import os

import numpy as np
import pytest

from oracle import dense
from oracle import frame as ofr
from oracle.frame import OracleFrame
from paper_1712_03554_amd import workloads as wl
from tests.oracle_helpers import (assert_frames_equal, oracle_vs_dense, sigma_ints,
                                  tableau_bits)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LIT = {"I": (0, 0), "Z": (0, 1), "X": (1, 0), "Y": (1, 1)}
PH = {"+1": 0, "+i": 1, "-1": 2, "-i": 3}


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [l.split() for l in fh if l.strip() and not l.startswith("#")]


def _pauli_matrix(s):
    m = np.array([[1.0 + 0j]])
    for ch in s:
        m = np.kron(m, dense.PAULI[ch])
    return m


# ---------------------------------------------------------------------------
# Table 1 and Table 2
# ---------------------------------------------------------------------------

def test_table1_pauli_products_oracle_and_matrices():
    L = ofr._load()
    rows = _lines("table1_pauli_products.txt")
    assert len(rows) == 16
    for a, b, ph, r in rows:
        e = L.ofr_pauli_g(*LIT[a], *LIT[b]) % 4
        assert e == PH[ph], (a, b)
        # the fixture itself agrees with 2x2 matrix products
        prod = dense.PAULI[a] @ dense.PAULI[b]
        assert np.allclose(prod, (1j ** PH[ph]) * dense.PAULI[r])


def _row_bits(s):
    x = z = 0
    for q, ch in enumerate(s):
        xb, zb = LIT[ch]
        x |= xb << q
        z |= zb << q
    return x, z


def _bits_str(x, z, n):
    inv = {v: k for k, v in LIT.items()}
    return "".join(inv[((x >> q) & 1, (z >> q) & 1)] for q in range(n))


def test_table2_clifford_conjugation():
    L = ofr._load()
    opmap = {"H": wl.H, "P": wl.S, "CNOT": wl.CNOT}
    for gate, inp, sign, out in _lines("table2_clifford_conjugation.txt"):
        n = len(inp)
        x, z = _row_bits(inp)
        cx, cz = ctypes.c_uint64(x), ctypes.c_uint64(z)
        flip = L.ofr_conjugate_row(n, opmap[gate], 0, 1, ctypes.byref(cx), ctypes.byref(cz))
        assert _bits_str(cx.value, cz.value, n) == out, (gate, inp)
        assert flip == (sign == "-"), (gate, inp)


@pytest.mark.parametrize("op", [wl.H, wl.S, wl.SDG, wl.X, wl.Y, wl.Z, wl.CNOT, wl.CZ])
def test_conjugation_rules_match_matrices(op):
    """U P U^dagger for every Pauli on two qubits, by explicit matrices."""
    L = ofr._load()
    two = op in (wl.CNOT, wl.CZ)
    psi_ops = {wl.CNOT: (wl.CNOT, 0, 1), wl.CZ: (wl.CZ, 0, 1)}
    U = np.eye(4, dtype=complex)
    for k in range(4):
        v = np.zeros(4, dtype=complex); v[k] = 1
        if two:
            U[:, k] = dense.apply_gate(v, 2, op, 0, 1)
        else:
            U[:, k] = dense.apply_gate(v, 2, op, 0)
    for s in itertools.product("IXYZ", repeat=2):
        s = "".join(s)
        x, z = _row_bits(s)
        cx, cz = ctypes.c_uint64(x), ctypes.c_uint64(z)
        flip = L.ofr_conjugate_row(2, op, 0, 1, ctypes.byref(cx), ctypes.byref(cz))
        want = U @ _pauli_matrix(s) @ U.conj().T
        got = (-1) ** flip * _pauli_matrix(_bits_str(cx.value, cz.value, 2))
        assert np.allclose(want, got), (op, s)


# ---------------------------------------------------------------------------
# Worked examples
# ---------------------------------------------------------------------------

def _parse_signed(rows):
    xs, zs, sig = [], [], 0
    for i, r in enumerate(rows):
        x, z = _row_bits(r[1:])
        xs.append(x); zs.append(z)
        if r[0] == "-":
            sig |= 1 << i
    return xs, zs, sig


def test_example1_equivalent_matrices_share_canonical_form():
    L = ofr._load()
    ex = {r[1]: r[2:] for r in _lines("examples.txt") if r[0] == "ex1"}
    want = _parse_signed(ex["canonical"])
    for name in ("M1", "M2", "M3"):
        xs, zs, sig = _parse_signed(ex[name])
        X = (ctypes.c_uint64 * 2)(*xs); Z = (ctypes.c_uint64 * 2)(*zs)
        S = (ctypes.c_uint64 * 1)(sig)
        L.ofr_canonicalize_signed(2, X, Z, S)
        assert (list(X), list(Z), S[0]) == (want[0], want[1], want[2]), name


def test_example2_cnot_on_bell():
    ex = {r[1]: r[2:] for r in _lines("examples.txt") if r[0] == "ex2"}
    f = OracleFrame(2)
    f.apply(wl.H, 0); f.apply(wl.CNOT, 0, 1)
    tab, sig, amp = f.read()
    bx, bz, bs = _parse_signed(ex["before"])
    assert [int(t[0]) for t in tab] == bx and [int(t[1]) for t in tab] == bz and sigma_ints(sig) == [bs]
    f.apply(wl.CNOT, 0, 1)
    tab, sig, amp = f.read()
    ax, az, as_ = _parse_signed(ex["after"])
    assert [int(t[0]) for t in tab] == ax and [int(t[1]) for t in tab] == az and sigma_ints(sig) == [as_]
    assert np.allclose(amp, [1.0])


def test_global_phase_example_P_on_one():
    f = OracleFrame(1, [1])
    f.apply(wl.S, 0)
    tab, sig, amp = f.read()
    assert sigma_ints(sig) == [1] and int(tab[0][1]) == 1
    assert abs(amp[0] - 1j) < 1e-15


def test_hadamard_global_phase_two_amplitudes():
    """H on (|0>+i|1>)/sqrt2 gives exp(i pi/4)(|0>-i|1>)/sqrt2: the sum of one
    real and one imaginary basis amplitude (global-phase steps, section 3)."""
    f = OracleFrame(1)
    f.apply(wl.H, 0); f.apply(wl.S, 0)
    tab, sig, amp = f.read()
    assert sigma_ints(sig) == [0] and abs(amp[0] - 1) < 1e-15
    f.apply(wl.H, 0)
    tab, sig, amp = f.read()
    assert (int(tab[0][0]), int(tab[0][1])) == (1, 1)   # Y row, sign -
    assert sigma_ints(sig) == [1]
    assert abs(amp[0] - np.exp(1j * np.pi / 4)) < 1e-15


def test_example3_two_element_frame():
    """a1(|00>+|01>) + a2(|10>+|11>) uses two phase vectors over {IX, ZI}."""
    f = OracleFrame(2)
    f.apply(wl.H, 0); f.apply(wl.T, 0); f.apply(wl.H, 1)
    tab, sig, amp = f.read()
    assert tableau_bits(tab, 2).tolist() == [[0, 1, 0, 0], [0, 0, 1, 0]]
    assert sigma_ints(sig) == [0, 2]
    assert np.allclose(amp, [2 ** -0.5, np.exp(1j * np.pi / 4) * 2 ** -0.5], atol=1e-15)


def test_example5_cofactor_two_qubits_gives_four_states():
    """|000>+|010>+|100>+|110> cofactored over its first two qubits: 4 states.
    COFACTOR is reached through T then T-dagger on each qubit (the phases
    cancel, the split remains)."""
    f = OracleFrame(3)
    f.apply(wl.H, 0); f.apply(wl.H, 1)
    assert f.size == 1
    f.apply(wl.T, 0)
    assert f.size == 2
    f.apply(wl.TDG, 0)
    f.apply(wl.T, 1)
    assert f.size == 4
    f.apply(wl.TDG, 1)
    tab, sig, amp = f.read()
    assert f.size == 4
    assert tableau_bits(tab, 3).tolist() == [[0, 0, 0, 1, 0, 0], [0, 0, 0, 0, 1, 0], [0, 0, 0, 0, 0, 1]]
    assert np.allclose(amp, [0.5] * 4, atol=1e-15)


def test_cofactor_size_law_same_or_double():
    rng = np.random.default_rng(7)
    for trial in range(20):
        c = wl.random_clifford_t(6, 30, 0, 100 + trial)
        f = OracleFrame(6)
        f.run(c.array())
        k_before = f.size
        q = int(rng.integers(6))
        x = f.xblock
        f.apply(wl.T, q)
        assert f.size in (k_before, 2 * k_before)


# ---------------------------------------------------------------------------
# The frame oracle against the dense definition
# ---------------------------------------------------------------------------

def test_single_gates_exhaustive_small():
    """Every gate on every qubit (pair) after each 2-qubit prefix of depth 2."""
    g1 = [wl.H, wl.S, wl.SDG, wl.X, wl.Y, wl.Z, wl.T, wl.TDG]
    layer = [(op, q) for op in g1 for q in range(2)] + [(wl.CNOT, 0, 1), (wl.CNOT, 1, 0), (wl.CZ, 0, 1)]
    count = 0
    for seq in itertools.product(layer, repeat=3):
        c = wl.Circuit(2)
        for g in seq:
            c.add(*g)
        oracle_vs_dense(c, every_gate=False)
        count += 1
    assert count == len(layer) ** 3


@pytest.mark.parametrize("seed", range(12))
def test_random_clifford_t_vs_dense(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 7))
    c = wl.random_clifford_t(n, 40, int(rng.integers(1, 6)), 1000 + seed,
                             measure_qubits=rng.permutation(n)[: int(rng.integers(0, n + 1))])
    # mix in every gate kind
    extra = [(wl.SDG, 0), (wl.X, n - 1), (wl.Y, 0), (wl.Z, 1 % n), (wl.CZ, 0, 1), (wl.TDG, 0),
             (wl.PHASE, 1 % n, 0, 0, 1, 8), (wl.PHASE, 0, 0, 0, 3, 2), (wl.PHASE, 0, 0, 0, -5, 12)]
    for i, g in enumerate(extra):
        c.gates.insert(int(rng.integers(0, len(c.gates))), tuple(list(g) + [0] * (6 - len(g)))
                       if len(g) < 6 else g)
    oracle_vs_dense(c, seed=seed)


def test_config1_against_256_amplitude_dense():
    for job in range(3):
        c = wl.config1(job)
        oracle_vs_dense(c, seed=wl.derive_seed(1, job), every_gate=False)


def test_circuit_identities():
    """T T = S and T^8 = I on a random state, as frames and as vectors."""
    base = wl.random_clifford_t(3, 25, 2, 55)
    for reps, replacement in ((2, [(wl.S, 1)]), (8, [])):
        a = wl.Circuit(3); a.gates = list(base.gates) + [(wl.T, 1, 0, 0, 0, 1)] * reps
        b = wl.Circuit(3); b.gates = list(base.gates) + [(op, q, 0, 0, 0, 1) for op, q in replacement]
        fa = OracleFrame(3); fa.run(a.array())
        fb = OracleFrame(3); fb.run(b.array())
        psi_a = _state_from_frame(fa)
        psi_b = _state_from_frame(fb)
        assert np.allclose(psi_a, psi_b, atol=1e-12)


def _state_from_frame(f):
    tab, sig, amp = f.read()
    n = f.n
    M = tableau_bits(tab, n)
    psi = np.zeros(1 << n, dtype=complex)
    for s, a in zip(sigma_ints(sig), amp):
        psi += a * dense.canonical_state(M, [(s >> i) & 1 for i in range(n)], n)
    return psi


# ---------------------------------------------------------------------------
# Closed forms and invariants
# ---------------------------------------------------------------------------

def qft_closed_form(x_bits):
    """Eq. 4 of the QFT section: the product state with factor l (l = 1..n)
    (|0> + exp(2 pi i 0.x_{n-l+1}...x_n)|1>)/sqrt2; the swap-free circuit
    produces the factors in reverse qubit order."""
    n = len(x_bits)
    factors = []
    for l in range(1, n + 1):
        frac = sum(x_bits[j - 1] * 2.0 ** -(j - (n - l)) for j in range(n - l + 1, n + 1))
        factors.append(np.array([1, np.exp(2j * np.pi * frac)]) / np.sqrt(2))
    factors = factors[::-1]
    v = np.array([1.0 + 0j])
    for fct in factors:
        v = np.kron(v, fct)
    return v


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_qft_dense_and_frame_match_closed_form(n):
    rng = np.random.default_rng(n)
    for _ in range(3):
        x = rng.integers(0, 2, size=n).tolist()
        c = wl.qft(n, x)
        psi, M, _ = dense.simulate(n, c.gates, c.init_bits)
        want = qft_closed_form(x)
        assert np.allclose(psi, want, atol=1e-12)
        f = OracleFrame(n, x)
        f.run(c.array())
        assert np.allclose(_state_from_frame(f), want, atol=1e-11)


def test_toffoli_network_is_toffoli():
    U = np.zeros((8, 8), dtype=complex)
    c = wl.Circuit(3).toffoli_7t(0, 1, 2)
    for k in range(8):
        v = np.zeros(8, dtype=complex); v[k] = 1
        for g in c.gates:
            v = dense.apply_gate(v, 3, g[0], g[1], g[2])
        U[:, k] = v
    want = np.eye(8); want[[6, 7]] = want[[7, 6]]
    assert np.allclose(U, want, atol=1e-12)
    assert c.count([wl.T, wl.TDG]) == 7 and c.count([wl.CNOT]) == 6 and c.count([wl.H]) == 2


def test_oracle_toffoli_and_cphase_ops_match_dense():
    rng = np.random.default_rng(3)
    for trial in range(6):
        base = wl.random_clifford_t(4, 12, 1, 300 + trial)
        for op in (wl.TOF, wl.CPHASE):
            f = OracleFrame(4)
            f.run(base.array())
            psi, _, _ = dense.simulate(4, base.gates)
            if op == wl.TOF:
                f.apply(op, 2, 0, 3)
                psi = dense.apply_gate(psi, 4, op, 2, 0, 3)
            else:
                f.apply(op, 1, 3, 0, 1, 4)
                psi = dense.apply_gate(psi, 4, op, 1, 3, num=1, den=4)
            assert np.allclose(_state_from_frame(f), psi, atol=1e-11)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_cuccaro_adds_basis_inputs(m):
    rng = np.random.default_rng(m)
    for _ in range(3):
        a = rng.integers(0, 2, size=m).tolist()
        b = rng.integers(0, 2, size=m).tolist()
        c = wl.cuccaro_adder(m, a, b, superpose=False)
        f = OracleFrame(c.n, c.init_bits)
        f.run(c.array())
        psi = _state_from_frame(f)
        idx = int(np.argmax(np.abs(psi)))
        assert abs(abs(psi[idx]) - 1) < 1e-12
        bits = [(idx >> (c.n - 1 - q)) & 1 for q in range(c.n)]
        A = sum(a[i] << i for i in range(m)); B = sum(b[i] << i for i in range(m))
        S = sum(bits[1 + 2 * i] << i for i in range(m))
        assert S == (A + B) % (1 << m)
        assert bits[2 * m + 1] == (A + B) >> m
        assert [bits[2 + 2 * i] for i in range(m)] == a and bits[0] == 0


def test_invariants_along_random_circuits():
    """Rows commute and are independent; norm 1; distinct phase vectors;
    Clifford-only circuits keep one element (Theorem 1, Definition 1, section 3)."""
    for seed in range(6):
        n = 5
        c = wl.random_clifford_t(n, 60, 4 if seed % 2 else 0, 500 + seed)
        f = OracleFrame(n)
        for g in c.gates:
            f.apply(*g)
            tab, sig, amp = f.read()
            M = tableau_bits(tab, n)
            for i in range(n):
                for j in range(n):
                    assert dense.symplectic(M[i], M[j], n) == 0
            assert dense.gf2_rank(M) == n
            assert abs(np.sum(np.abs(amp) ** 2) - 1) < 1e-12
            s = sigma_ints(sig)
            assert len(set(s)) == len(s) and s == sorted(s)
            if seed % 2 == 0:
                assert f.size == 1


def test_stabilizer_measurement_probabilities():
    """Clifford-only states measure with p in {0, 1/2, 1} (section 2.2)."""
    for seed in range(10):
        c = wl.random_clifford_t(5, 30, 0, 900 + seed)
        psi, _, _ = dense.simulate(5, c.gates)
        for q in range(5):
            p = dense.qubit_prob1(psi, 5, q)
            assert min(abs(p), abs(p - 0.5), abs(p - 1)) < 1e-12


def test_steane_syndromes():
    """Without T and faults every syndrome is a deterministic 0; one X (Z) on
    data qubit j flips the Z-checks (X-checks) whose support holds j; with T on
    data qubit 0 the Z-checks stay deterministic."""
    base = wl.steane_base()
    no_t = [g for g in base.gates if g[0] != wl.T]
    for fault in [None] + [(wl.X, j) for j in range(7)] + [(wl.Z, j) for j in range(7)]:
        c = wl.Circuit(13)
        c.gates = list(no_t[:13]) + ([(fault[0], fault[1], 0, 0, 0, 1)] if fault else []) + list(no_t[13:])
        for a in range(7, 13):
            c.measure(a)
        for seed in (1, 2):
            f = OracleFrame(13, None, seed)
            f.run(c.array())
            outs = f.outcomes()
            want = [0] * 6
            if fault:
                kind, j = fault
                for k, sup in enumerate(wl.HAMMING_CHECKS):
                    if j in sup:
                        want[(3 + k) if kind == wl.X else k] = 1
            assert outs == want, (fault, outs)
            assert f.size == 1
    # with T: Z-check outcomes deterministic 0, frame has at most 2 elements
    c = wl.steane_base()
    for a in range(7, 13):
        c.measure(a)
    for seed in range(8):
        f = OracleFrame(13, None, seed)
        sizes = f.run(c.array())
        assert max(sizes) <= 2
        assert f.outcomes()[3:] == [0, 0, 0]


def test_measurement_outcomes_follow_seeded_coin():
    c = wl.random_clifford_t(6, 50, 3, 77, measure_qubits=range(6))
    for seed in range(5):
        oracle_vs_dense(c, seed=seed, every_gate=False)


# ---------------------------------------------------------------------------
# Direct controlled phase and Toffoli (double cofactor, Eqs. 2 and 3)
# ---------------------------------------------------------------------------
def _direct_mix(seed, n, n_gates=14):
    """Random Clifford/T circuit on n qubits with direct CPHASE and Toffoli
    gates and a measurement sprinkled in."""
    rng = np.random.default_rng(seed)
    c = wl.random_clifford_t(n, n_gates, 1, 900 + seed)
    extra = []
    for _ in range(3):
        a, b, t = (int(v) for v in rng.permutation(n)[:3])
        extra.append((wl.TOF_D, a, b, t, 0, 1))
        num, den = [(1, 2), (1, 4), (-3, 8), (1, 1), (2, 1), (5, 6)][int(rng.integers(6))]
        extra.append((wl.CPHASE_D, a, t, 0, num, den))
    extra.append((wl.MEASURE, int(rng.integers(n)), 0, 0, 0, 1))
    for g in extra:
        c.gates.insert(int(rng.integers(0, len(c.gates) + 1)), g)
    c.name = f"direct{seed}"
    return c


@pytest.mark.parametrize("seed", range(10))
def test_direct_gates_vs_dense(seed):
    """The direct forms give the expansion of the exact state in the basis of
    the matrix the double cofactor leaves, gate by gate."""
    oracle_vs_dense(_direct_mix(seed, 3 + seed % 4), seed=seed)


def test_direct_and_decomposed_forms_give_the_same_state():
    for trial in range(6):
        base = wl.random_clifford_t(5, 16, 2, 400 + trial)
        for direct, dec in (((wl.TOF_D, 1, 4, 2, 0, 1), (wl.TOF, 1, 4, 2, 0, 1)),
                            ((wl.CPHASE_D, 3, 0, 0, 1, 4), (wl.CPHASE, 3, 0, 0, 1, 4))):
            f1, f2 = OracleFrame(5), OracleFrame(5)
            f1.run(base.array()); f2.run(base.array())
            f1.apply(*direct); f2.apply(*dec)
            assert np.allclose(_state_from_frame(f1), _state_from_frame(f2), atol=1e-11)


def test_direct_toffoli_grows_a_frame_at_most_fourfold():
    """Two cofactors and a controlled Pauli: at most 4x growth per Toffoli
    (against up to 2^7 for the 7-T network)."""
    c = wl.cuccaro_adder(3, direct=True)
    f = OracleFrame(c.n, c.init_bits)
    for g in c.gates:
        before = f.size
        f.apply(*g)
        if g[0] == wl.TOF_D:
            assert f.size <= 4 * before


@pytest.mark.parametrize("m", [1, 2, 3])
def test_cuccaro_direct_adds_basis_inputs(m):
    rng = np.random.default_rng(50 + m)
    for _ in range(3):
        a = rng.integers(0, 2, size=m).tolist()
        b = rng.integers(0, 2, size=m).tolist()
        c = wl.cuccaro_adder(m, a, b, superpose=False, direct=True)
        f = OracleFrame(c.n, c.init_bits)
        f.run(c.array())
        assert f.size == 1                       # controls on basis inputs are deterministic
        psi = _state_from_frame(f)
        idx = int(np.argmax(np.abs(psi)))
        bits = [(idx >> (c.n - 1 - q)) & 1 for q in range(c.n)]
        A = sum(a[i] << i for i in range(m)); B = sum(b[i] << i for i in range(m))
        assert sum(bits[1 + 2 * i] << i for i in range(m)) == (A + B) % (1 << m)
        assert bits[2 * m + 1] == (A + B) >> m


@pytest.mark.parametrize("n", [2, 3, 5])
def test_qft_direct_matches_closed_form(n):
    x = [1] * n
    c = wl.qft(n, x, direct=True)
    f = OracleFrame(n, x)
    f.run(c.array())
    psi = _state_from_frame(f)
    # Eq. 4 with the qubit order reversed (no final swaps): prod_j (|0> + e^{2 pi i 0.x_j..x_n}|1>)/sqrt2
    X = sum(b << (n - 1 - q) for q, b in enumerate(x))
    ref = np.zeros(1 << n, dtype=complex)
    for y in range(1 << n):
        yr = int(format(y, f"0{n}b")[::-1], 2)
        ref[y] = np.exp(2j * np.pi * X * yr / (1 << n)) / np.sqrt(1 << n)
    assert np.allclose(psi, ref, atol=1e-11)


def test_splitmix64_known_answers():
    """The measurement generator is SplitMix64 (Steele, Lea & Flood 2014):
    started from state 0, the reference implementation's first outputs are
    e220a8397b1dcdaf, 6e789e6aa1b965f4, 06c45d188009454f."""
    assert [wl.splitmix64(0, i) for i in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                      0x06C45D188009454F]
    assert wl.measurement_uniform(0, 0) == (0xE220A8397B1DCDAF >> 11) * 2.0 ** -53


def test_oracle_coin_is_u_below_p1():
    """Measurement outcome 1 exactly when u < p(1), u from the 53 high bits of
    output k of the state's generator (k counts its measurements): |+>
    measured again and again (p(1) = 1/2 each time), and H T H |0> measured
    once (p(1) = (1 - cos(pi/4)) / 2) for 64 seeds."""
    for seed in (0, 1, 7, 20171210, 2**63 + 5):
        f = OracleFrame(1, [0], seed)
        for _ in range(12):
            f.apply(wl.H, 0)
            f.apply(wl.MEASURE, 0)
        want = [int(wl.measurement_uniform(seed, k) < 0.5) for k in range(12)]
        assert f.outcomes() == want, seed
    p1 = (1.0 - np.cos(np.pi / 4)) / 2.0
    ones = 0
    for seed in range(64):
        u = wl.measurement_uniform(seed, 0)
        if abs(u - p1) < 1e-12:
            continue
        f = OracleFrame(1, [0], seed)
        for g in ((wl.H, 0), (wl.T, 0), (wl.H, 0), (wl.MEASURE, 0)):
            f.apply(*g)
        assert f.outcomes() == [int(u < p1)], seed
        ones += f.outcomes()[0]
    assert 0 < ones < 32
