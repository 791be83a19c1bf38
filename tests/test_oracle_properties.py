"""Property tests of the C frame oracle (hypothesis): random circuits over
every gate kind on up to 8 qubits, and after every gate the facts that the
paper fixes for any frame, whatever the circuit:

* the stabilizer rows commute pairwise and are independent (Theorem 1);
* the amplitudes have norm 1 and the phase vectors are distinct, in the
  canonical ascending order (Definition 1);
* a frame reached by Clifford gates and measurements only has one element
  (a stabilizer state is a one-element frame, section 3);
* COFACTOR keeps or doubles the frame (section 3) and a measurement never
  grows it (section 4), so |F| <= 2^k with k the number of non-Clifford
  phase gates applied so far, and the phase vectors lie in an affine space
  of dimension at most k;
* a measurement is a projection (section 2.2 for stabilizer states, section
  4 for frames): measuring the same qubit again at once repeats the outcome.
"""
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle.frame import OracleFrame
from paper_1712_03554_amd import workloads as wl
from tests.oracle_helpers import sigma_ints, tableau_bits

ONE_QUBIT = [wl.H, wl.S, wl.SDG, wl.X, wl.Y, wl.Z, wl.T, wl.TDG]
ANGLES = [(1, 2), (2, 2), (3, 2), (4, 2), (-1, 2), (1, 4), (3, 4), (-1, 4), (1, 8), (5, 8), (1, 3)]


def _non_clifford(g):
    op, num, den = g[0], g[4], g[5]
    if op in (wl.T, wl.TDG):
        return True
    return op == wl.PHASE and (2 * num) % den != 0


@st.composite
def circuits(draw):
    n = draw(st.integers(1, 8))
    bits = draw(st.lists(st.integers(0, 1), min_size=n, max_size=n))
    gates = []
    for _ in range(draw(st.integers(0, 40))):
        kind = draw(st.integers(0, 4))
        q = draw(st.integers(0, n - 1))
        if kind == 0 and n > 1:
            r = draw(st.integers(0, n - 2))
            gates.append((draw(st.sampled_from([wl.CNOT, wl.CZ])), q, r + (r >= q), 0, 0, 1))
        elif kind == 1:
            num, den = draw(st.sampled_from(ANGLES))
            gates.append((wl.PHASE, q, 0, 0, num, den))
        elif kind == 2:
            gates.append((wl.MEASURE, q, 0, 0, 0, 1))
        else:
            gates.append((draw(st.sampled_from(ONE_QUBIT)), q, 0, 0, 0, 1))
    seed = draw(st.integers(0, 2**63 - 1))
    return n, bits, gates, seed


def _gf2_rank(rows):
    """Rank over GF(2) of a list of Python-int bit rows."""
    basis = []
    for v in rows:
        for b in basis:
            v = min(v, v ^ b)
        if v:
            basis.append(v)
    return len(basis)


def _check_frame(f, n, k, clifford_only, what):
    tab, sig, amp = f.read()
    M = tableau_bits(tab, n).astype(np.int64)
    X, Z = M[:, :n], M[:, n:]
    sym = (X @ Z.T + Z @ X.T) & 1
    assert not sym.any(), f"{what}: two rows anticommute"
    rows = [int("".join(map(str, r)), 2) for r in M]
    assert _gf2_rank(rows) == n, f"{what}: rows not independent"
    s = sigma_ints(sig)
    K = len(s)
    assert K >= 1
    assert all(a < b for a, b in zip(s, s[1:])), f"{what}: phase vectors not distinct and ascending"
    norm = float(np.sum(np.abs(np.asarray(amp, dtype=complex)) ** 2))
    assert abs(norm - 1.0) <= 1e-12, f"{what}: norm {norm!r}"
    assert K == f.size
    assert K <= 2 ** k, f"{what}: |F| = {K} after {k} non-Clifford gates"
    assert _gf2_rank([v ^ s[0] for v in s[1:]]) <= k, f"{what}: phase vectors span too much"
    if clifford_only:
        assert K == 1, f"{what}: Clifford-only circuit with {K} elements"
    return K


@settings(max_examples=300, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(circuits())
def test_frame_invariants_after_every_gate(case):
    n, bits, gates, seed = case
    f = OracleFrame(n, bits, seed)
    k = 0
    _check_frame(f, n, k, True, "initial state")
    nmeas = 0
    for gi, g in enumerate(gates):
        before = f.size
        f.apply(*g)
        k += _non_clifford(g)
        K = _check_frame(f, n, k, k == 0, f"gate {gi} {g}")
        if g[0] == wl.MEASURE:
            nmeas += 1
            assert K <= before, f"gate {gi}: a measurement grew the frame"
            o = f.outcomes()[-1]
            f.apply(wl.MEASURE, g[1])
            nmeas += 1
            assert f.outcomes()[-1] == o, f"gate {gi}: repeated measurement changed its outcome"
            assert f.size == K
            _check_frame(f, n, k, k == 0, f"repeat of gate {gi}")
        elif _non_clifford(g):
            assert K <= 2 * before, f"gate {gi}: a cofactor more than doubled the frame"
        else:
            assert K == before, f"gate {gi}: a Clifford gate changed the frame size"
    assert len(f.outcomes()) == nmeas


@pytest.mark.parametrize("n", [3, 6])
def test_bound_is_reached_by_t_on_superpositions(n):
    """H then T on every qubit: each T cofactors a random qubit, so the frame
    doubles every time and meets the bound 2^k with equality."""
    f = OracleFrame(n, [0] * n, 1)
    for q in range(n):
        f.apply(wl.H, q)
    for q in range(n):
        f.apply(wl.T, q)
        assert f.size == 2 ** (q + 1)
    _check_frame(f, n, n, False, "H^n T^n")
    assert math.isclose(sum(abs(a) ** 2 for a in f.read()[2]), 1.0, abs_tol=1e-12)
