"""Pins of the C frame oracle on registers of more than 64 qubits (two to four
packed words per row and per phase vector), where no dense state vector can
be formed.  Each check is fixed by the paper or by plain mathematics, not by
the oracle itself:

* the rows of the stabilizer matrix commute pairwise and are independent
  (Theorem 1), the matrix is the fully reduced echelon form with sorted
  pivots (the canonical form read from the Figure 2b caption), the amplitudes
  have norm 1 and the phase vectors are distinct and in canonical order
  (Definition 1), and Clifford-only circuits keep one element (section 3);
* the unsigned matrix equals the group recursion of the tableau track
  (conjugation by each Clifford gate; a random cofactor keeps the commutant
  of Z_q and adds Z_q), run here on plain 0/1 arrays;
* a circuit on a few qubits gives the same frame when its qubits are spread
  over a wide register across the 63/64, 127/128, 191/192, 511/512 and
  1023/1024 word boundaries (registers of up to 1100 qubits): the wide tableau restricted to those qubits equals the narrow
  one, the other rows are Z_q, the phase vectors agree on the matching rows,
  the outcomes and amplitudes agree, and the narrow frame read back out of
  the wide one expands to the narrow circuit's dense state vector;
* a circuit, T.T.S^dagger and T^8 on some qubits, then the inverse circuit
  is the identity: measuring every qubit gives the initial bits for every
  seed and leaves amplitude exactly 1 (circuit identities).

Also here: the branch-pruned frame expansion of the dense checker equals the
plain expansion it stands in for, and the frame-size law of the QFT on
|1...1> (section 6) with the Eq. 4 state at more qubits.
"""
import numpy as np
import pytest

from oracle import dense
from oracle.frame import OracleFrame
from paper_1712_03554_amd import workloads as wl
from tests.oracle_helpers import assert_frames_equal, sigma_ints, tableau_bits

WIDE = [65, 128, 200, 256]


# ---------------------------------------------------------------------------
# Checks on packed words
# ---------------------------------------------------------------------------

def _popcnt(a):
    return np.bitwise_count(a).astype(np.int64)


def _assert_commuting(tab, n):
    W = (n + 63) // 64
    X, Z = tab[:, :W], tab[:, W:]
    s = np.zeros((n, n), dtype=np.int64)
    for w in range(W):
        s += _popcnt(X[:, None, w] & Z[None, :, w]) + _popcnt(Z[:, None, w] & X[None, :, w])
    assert not np.any(s & 1), "two rows anticommute"


def _pivot(row_words, n):
    """First set column in the order x_0..x_{n-1}, z_0..z_{n-1}; -1 if none."""
    W = (n + 63) // 64
    for half in (0, 1):
        for w in range(W):
            v = int(row_words[half * W + w])
            if v:
                return half * n + 64 * w + ((v & -v).bit_length() - 1)
    return -1


def _colbit(tab, i, col, n):
    W = (n + 63) // 64
    half, q = divmod(col, n)
    return (int(tab[i, half * W + (q >> 6)]) >> (q & 63)) & 1


def _assert_canonical(tab, n):
    """Fully reduced echelon form, pivots strictly increasing, n of them
    (so the rank is n)."""
    piv = [_pivot(tab[i], n) for i in range(n)]
    assert all(p >= 0 for p in piv), "a zero row: rank below n"
    assert all(a < b for a, b in zip(piv, piv[1:])), "pivots not increasing"
    for i, p in enumerate(piv):
        for j in range(n):
            if j != i:
                assert _colbit(tab, j, p, n) == 0, f"pivot column {p} of row {i} not reduced"


def _assert_frame_invariants(f, n, clifford_only):
    tab, sig, amp = f.read()
    _assert_commuting(tab, n)
    _assert_canonical(tab, n)
    assert abs(float(np.sum(amp.real ** 2 + amp.imag ** 2)) - 1.0) <= 1e-12
    s = sigma_ints(sig)
    assert len(set(s)) == len(s) and s == sorted(s)
    if clifford_only:
        assert len(s) == 1
    return tab


def _with_measurements(c, seed, count):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        c.gates.insert(int(rng.integers(len(c.gates) + 1)), (wl.MEASURE, int(rng.integers(c.n)), 0, 0, 0, 1))
    return c


def _track(n, gates):
    """The tableau track as the group recursion on 0/1 arrays (dense.TableauTrack)."""
    tr = dense.TableauTrack(n)
    for op, q0, q1, q2, num, den in gates:
        if op in (wl.H, wl.S, wl.SDG, wl.X, wl.Y, wl.Z, wl.CNOT, wl.CZ):
            tr.conjugate(op, q0, q1)
        elif op in (wl.T, wl.TDG, wl.MEASURE):
            tr.cofactor(q0)
        else:
            raise ValueError(op)
    return tr.canonical()


# ---------------------------------------------------------------------------
# Invariants at every gate, and the tableau against the group recursion
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", WIDE)
@pytest.mark.parametrize("n_t", [0, 5])
def test_invariants_at_every_gate_wide(n, n_t):
    gates = 150 if n > 128 else 260
    c = _with_measurements(wl.random_clifford_t(n, gates, n_t, 61000 + n + n_t), 62000 + n, 6)
    f = OracleFrame(n, None, 5 + n)
    for g in c.gates:
        f.apply(*g)
        tab = _assert_frame_invariants(f, n, clifford_only=(n_t == 0))
    assert not f.fragile
    assert np.array_equal(tableau_bits(tab, n), _track(n, c.gates))


@pytest.mark.parametrize("n", [130, 256, 600])
def test_tableau_matches_group_recursion_long_circuit(n):
    """Many gates on a wide register: the unsigned matrix equals the group
    recursion, checked at several points of the run."""
    c = _with_measurements(wl.random_clifford_t(n, 4 * n, 8, 63000 + n), 64000 + n, 10)
    f = OracleFrame(n, None, 1)
    done = 0
    for stop in (len(c) // 3, 2 * len(c) // 3, len(c)):
        for g in c.gates[done:stop]:
            f.apply(*g)
        done = stop
        tab, _, _ = f.read()
        assert np.array_equal(tableau_bits(tab, n), _track(n, c.gates[:stop])), f"after {stop} gates"


# ---------------------------------------------------------------------------
# A narrow circuit spread over a wide register
# ---------------------------------------------------------------------------

EMBEDDINGS = [
    (130, [0, 62, 63, 64, 65, 127, 128, 129]),
    (200, [1, 63, 64, 126, 127, 128, 191, 192]),
    (256, [0, 63, 64, 127, 128, 191, 192, 255]),
    (256, [60, 61, 62, 63, 64, 65, 66, 67]),
    (700, [0, 255, 256, 511, 512, 513, 640, 699]),
    (1100, [63, 64, 511, 512, 1023, 1024, 1025, 1099]),
]


def _narrow_circuit(seed, k):
    rng = np.random.default_rng(seed)
    c = wl.random_clifford_t(k, 70, 4 + seed % 3, 65000 + seed)
    extra = [(wl.SDG, 0, 0, 0, 0, 1), (wl.X, k - 1, 0, 0, 0, 1), (wl.Y, 1, 0, 0, 0, 1), (wl.Z, 2, 0, 0, 0, 1),
             (wl.CZ, 0, k - 1, 0, 0, 1), (wl.TDG, 3, 0, 0, 0, 1), (wl.PHASE, 1, 0, 0, 1, 8),
             (wl.PHASE, 4, 0, 0, -5, 12)]
    for g in extra:
        c.gates.insert(int(rng.integers(len(c.gates) + 1)), g)
    c = _with_measurements(c, 66000 + seed, 3)
    c.init_bits = rng.integers(0, 2, size=k).tolist()
    return c


def _spread(c, N, pos):
    wide = wl.Circuit(N)
    for q, p in enumerate(pos):
        wide.init_bits[p] = c.init_bits[q]
    for op, q0, q1, q2, num, den in c.gates:
        wide.add(op, pos[q0], pos[q1] if op in (wl.CNOT, wl.CZ, wl.CPHASE_D, wl.TOF_D) else 0,
                 pos[q2] if op == wl.TOF_D else 0, num, den)
    return wide


@pytest.mark.parametrize("case", range(len(EMBEDDINGS)))
@pytest.mark.parametrize("seed", range(5))
def test_narrow_circuit_spread_over_word_boundaries(case, seed):
    N, pos = EMBEDDINGS[case]
    k = len(pos)
    c = _narrow_circuit(seed + 10 * case, k)
    rng = np.random.default_rng(seed)
    if seed % 2:
        # a permutation of the active qubits as well (pos stays increasing, so
        # the narrow reference is the permuted narrow circuit)
        perm = rng.permutation(k).tolist()
        c = _spread(c, k, perm)
    wide = _spread(c, N, pos)
    run_seed = 900 + seed
    fn = OracleFrame(k, c.init_bits, run_seed)
    fn.run(c.array())
    fw = OracleFrame(N, wide.init_bits, run_seed)
    fw.run(wide.array())
    assert fw.outcomes() == fn.outcomes()
    assert fw.size == fn.size and fw.xblock == fn.xblock
    assert not fw.fragile and not fn.fragile

    tn, sn, an = fn.read()
    tw, sw, aw = fw.read()
    Mn = tableau_bits(tn, k)
    Mw = tableau_bits(tw, N)
    cols = pos + [N + p for p in pos]
    idle = [q for q in range(N) if q not in set(pos)]
    # rows of the wide matrix: the narrow rows in order, plus Z_q for idle q
    active_rows, idle_rows = [], []
    for i in range(N):
        if Mw[i].sum() == 1 and Mw[i, N:][idle].sum() == 1:
            idle_rows.append(i)
        else:
            active_rows.append(i)
    assert len(active_rows) == k and len(idle_rows) == N - k
    assert sorted(int(np.argmax(Mw[i, N:])) for i in idle_rows) == idle
    assert np.array_equal(Mw[np.ix_(active_rows, cols)], Mn)
    other = [col for col in range(2 * N) if col not in set(cols)]
    assert not np.any(Mw[np.ix_(active_rows, other)])
    # phase vectors: equal on the matching rows, + on the idle Z_q rows
    sig_n = sigma_ints(sn)
    sig_w = sigma_ints(sw)
    for a, b in zip(sig_n, sig_w):
        assert all(((b >> i) & 1) == 0 for i in idle_rows)
        assert a == sum(((b >> i) & 1) << r for r, i in enumerate(active_rows))
    assert np.array_equal(aw, an)
    # the narrow frame read out of the wide one is the narrow dense state
    psi, _, outs = dense.simulate(k, c.gates, c.init_bits, seed=run_seed)
    assert outs == fw.outcomes()
    state = np.zeros(1 << k, dtype=complex)
    for s, a in zip(sig_w, aw):
        bits = [(s >> i) & 1 for i in active_rows]
        state += a * dense.canonical_state(Mw[np.ix_(active_rows, cols)], bits, k)
    assert np.allclose(state, psi, atol=1e-11)


# ---------------------------------------------------------------------------
# Circuit identities on wide registers
# ---------------------------------------------------------------------------

_INVERSE = {wl.H: wl.H, wl.S: wl.SDG, wl.SDG: wl.S, wl.X: wl.X, wl.Y: wl.Y, wl.Z: wl.Z,
            wl.CNOT: wl.CNOT, wl.CZ: wl.CZ, wl.T: wl.TDG, wl.TDG: wl.T, wl.PHASE: wl.PHASE}


def _inverse(c):
    inv = wl.Circuit(c.n, c.init_bits)
    for op, q0, q1, q2, num, den in reversed(c.gates):
        inv.add(_INVERSE[op], q0, q1, q2, -num if op == wl.PHASE else num, den)
    return inv


@pytest.mark.parametrize("n", WIDE)
def test_identity_circuits_return_the_basis_state(n):
    """C, then T.T.S^dagger and T^8 on qubits at the word edges, then
    C^dagger is the identity: measuring every qubit afterwards gives the
    initial bits for every seed (each outcome has probability 1) and leaves
    one element of amplitude exactly 1 (global phase included)."""
    rng = np.random.default_rng(n)
    c = wl.random_clifford_t(n, 3 * n, 7, 67000 + n)
    for g in [(wl.PHASE, int(rng.integers(n)), 0, 0, 1, 8), (wl.PHASE, int(rng.integers(n)), 0, 0, -3, 16),
              (wl.SDG, int(rng.integers(n)), 0, 0, 0, 1), (wl.Y, int(rng.integers(n)), 0, 0, 0, 1),
              (wl.CZ, 0, n - 1, 0, 0, 1), (wl.TDG, n - 1, 0, 0, 0, 1)]:
        c.gates.insert(int(rng.integers(len(c.gates) + 1)), g)
    bits = rng.integers(0, 2, size=n).tolist()
    full = wl.Circuit(n, bits)
    full.gates = list(c.gates)
    for q in sorted({0, 63 % n, 64 % n, n - 1}):
        full.t(q); full.t(q); full.sdg(q)
    for _ in range(8):
        full.t(n // 2)
    full.gates += _inverse(c).gates
    for q in range(n):
        full.measure(q)
    for seed in range(3):
        f = OracleFrame(n, bits, seed)
        sizes = f.run(full.array())
        assert int(sizes.max()) > 1
        assert f.outcomes() == bits
        tab, sig, amp = f.read()
        want = np.zeros((n, 2 * n), dtype=np.uint8)
        want[np.arange(n), n + np.arange(n)] = 1
        assert np.array_equal(tableau_bits(tab, n), want)
        assert sigma_ints(sig) == [sum(b << q for q, b in enumerate(bits))]
        assert abs(amp[0] - 1.0) <= 1e-12
        assert not f.fragile


# ---------------------------------------------------------------------------
# The dense checker's pruned expansion equals the plain one
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_frame_expansion_fast_equals_plain(seed):
    rng = np.random.default_rng(seed)
    n = 1 + seed % 5
    tr = dense.TableauTrack(n)
    for _ in range(6 * n):
        op = int(rng.integers(3))
        a = int(rng.integers(n))
        if op == 2 and n > 1:
            b = int((a + 1 + rng.integers(n - 1)) % n)
            tr.conjugate(wl.CNOT, a, b)
        else:
            tr.conjugate((wl.H, wl.S, wl.H)[op], a)
    M = tr.canonical()
    kind = seed % 3
    if kind == 0:      # generic vector: every basis state appears
        psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    elif kind == 1:    # a few basis states
        psi = np.zeros(1 << n, dtype=complex)
        psi[rng.choice(1 << n, size=min(3, 1 << n), replace=False)] = rng.standard_normal(min(3, 1 << n))
    else:              # a superposition of two states of the same basis
        s1 = rng.integers(0, 2, size=n)
        s2 = rng.integers(0, 2, size=n)
        psi = dense.canonical_state(M, s1, n) + 0.5j * dense.canonical_state(M, s2, n)
    psi = psi / np.linalg.norm(psi)
    plain = dense.frame_expansion(M, psi, n)
    fast = dense.frame_expansion_fast(M, psi, n)
    assert [s for s, _ in fast] == [s for s, _ in plain]
    assert np.allclose([a for _, a in fast], [a for _, a in plain], atol=1e-13)
    if kind == 2:
        assert len(plain) == (1 if np.array_equal(s1, s2) else 2)


# ---------------------------------------------------------------------------
# QFT on |1...1>: frame size 2^(n-1) (section 6) and the Eq. 4 state
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("direct", [True, False])
@pytest.mark.parametrize("n", [2, 5, 8, 10, 12])
def test_qft_on_all_ones_has_half_size_frame(n, direct):
    """Exact QFT on |1...1> (controlled rotations direct, or three phase
    gates each): the frame ends with 2^(n-1) elements."""
    c = wl.qft(n, [1] * n, direct=direct)
    f = OracleFrame(n, c.init_bits)
    sizes = f.run(c.array())
    assert f.size == 2 ** (n - 1)
    assert int(sizes.max()) <= 2 ** (n - 1)
    assert not f.fragile


@pytest.mark.parametrize("n", [8, 10])
def test_qft_frame_matches_closed_form_more_qubits(n):
    from tests.test_oracle_pins import qft_closed_form
    rng = np.random.default_rng(100 + n)
    for x in ([1] * n, rng.integers(0, 2, size=n).tolist()):
        c = wl.qft(n, x, direct=True)
        f = OracleFrame(n, x)
        f.run(c.array())
        tab, sig, amp = f.read()
        M = tableau_bits(tab, n)
        want = qft_closed_form(x)
        exp = dense.frame_expansion_fast(M, want, n)
        assert_frames_equal(sigma_ints(sig), amp, [s for s, _ in exp], [a for _, a in exp], what=f"qft{n}")
