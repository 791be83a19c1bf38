"""Dense state-vector checker -- TEST INFRASTRUCTURE ONLY.

The plain definition of what single-frame simulation computes (Garcia &
Markov, sections 2.2-4): the exact state vector of the circuit, and its
expansion in the orthonormal basis of stabilizer states that the frame's
stabilizer matrix defines (Observation 2, Definition 1).  Written
independently of oracle/frame.c and of the HIP library; n <= 12.

Conventions: qubit 0 is the most significant bit of a basis index; a Pauli row
is (x, z) bit vectors with literal I/Z/X/Y for 00/01/10/11 (section 2.2); the
canonical basis state for signs sigma has a real positive amplitude at the
smallest basis index of its support; the stabilizer matrix is the fully reduced
row echelon form over columns x_0..x_{n-1}, z_0..z_{n-1}.
"""
from __future__ import annotations

import numpy as np

H, S, SDG, X, Y, Z, CNOT, CZ, T, TDG, PHASE, CPHASE, TOF, MEASURE, CPHASE_D, TOF_D = range(16)

PAULI = {
    "I": np.eye(2, dtype=complex),
    "X": np.array([[0, 1], [1, 0]], dtype=complex),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=complex),
    "Z": np.array([[1, 0], [0, -1]], dtype=complex),
}


def phase_matrix(theta: float) -> np.ndarray:
    return np.array([[1, 0], [0, np.exp(1j * theta)]], dtype=complex)


def one_qubit_matrix(op: int, num: int = 0, den: int = 1) -> np.ndarray:
    if op == H:
        return np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2.0)
    if op == S:
        return phase_matrix(np.pi / 2)
    if op == SDG:
        return phase_matrix(-np.pi / 2)
    if op == X:
        return PAULI["X"]
    if op == Y:
        return PAULI["Y"]
    if op == Z:
        return PAULI["Z"]
    if op == T:
        return phase_matrix(np.pi / 4)
    if op == TDG:
        return phase_matrix(-np.pi / 4)
    if op == PHASE:
        return phase_matrix(np.pi * num / den)
    raise ValueError(op)


def apply_1q(psi: np.ndarray, n: int, q: int, U: np.ndarray) -> np.ndarray:
    t = psi.reshape((2,) * n)
    t = np.tensordot(U, t, axes=([1], [q]))
    t = np.moveaxis(t, 0, q)
    return t.reshape(-1)


def apply_controlled(psi: np.ndarray, n: int, controls, t: int, U: np.ndarray) -> np.ndarray:
    """Apply U to qubit t on the basis states whose controls are all 1."""
    idx = np.arange(psi.size)
    sel = np.ones(psi.size, dtype=bool)
    for c in controls:
        sel &= ((idx >> (n - 1 - c)) & 1) == 1
    out = psi.copy()
    full = apply_1q(psi, n, t, U)
    out[sel] = full[sel]
    return out


def apply_gate(psi, n, op, q0, q1=0, q2=0, num=0, den=1):
    if op in (H, S, SDG, X, Y, Z, T, TDG, PHASE):
        return apply_1q(psi, n, q0, one_qubit_matrix(op, num, den))
    if op == CNOT:
        return apply_controlled(psi, n, [q0], q1, PAULI["X"])
    if op == CZ:
        return apply_controlled(psi, n, [q0], q1, PAULI["Z"])
    if op in (CPHASE, CPHASE_D):
        return apply_controlled(psi, n, [q0], q1, phase_matrix(np.pi * num / den))
    if op in (TOF, TOF_D):
        return apply_controlled(psi, n, [q0, q1], q2, PAULI["X"])
    raise ValueError(op)


def basis_state(n: int, bits) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=complex)
    idx = 0
    for q in range(n):
        idx |= (int(bits[q]) & 1) << (n - 1 - q)
    psi[idx] = 1.0
    return psi


def qubit_prob1(psi: np.ndarray, n: int, q: int) -> float:
    idx = np.arange(psi.size)
    m = ((idx >> (n - 1 - q)) & 1) == 1
    return float(np.sum(np.abs(psi[m]) ** 2))


def project(psi: np.ndarray, n: int, q: int, outcome: int) -> np.ndarray:
    idx = np.arange(psi.size)
    m = ((idx >> (n - 1 - q)) & 1) == outcome
    out = np.where(m, psi, 0)
    return out / np.linalg.norm(out)


# ---------------------------------------------------------------------------
# Pauli rows and the stabilizer group of the frame (the tableau track)
# ---------------------------------------------------------------------------

def pauli_apply(x: np.ndarray, z: np.ndarray, v: np.ndarray, n: int) -> np.ndarray:
    """Apply the unsigned Pauli with literal bits (x, z) to state vector v."""
    U = np.array([[1.0 + 0j]])
    for q in range(n):
        key = {(0, 0): "I", (0, 1): "Z", (1, 0): "X", (1, 1): "Y"}[(int(x[q]), int(z[q]))]
        U = np.kron(U, PAULI[key]) if n <= 6 else None
        if U is None:
            break
    if n <= 6:
        return U @ v
    out = v.copy()
    for q in range(n):
        key = {(0, 0): "I", (0, 1): "Z", (1, 0): "X", (1, 1): "Y"}[(int(x[q]), int(z[q]))]
        if key != "I":
            out = apply_1q(out, n, q, PAULI[key])
    return out


def rref(rows: np.ndarray) -> np.ndarray:
    """Fully reduced row echelon form over GF(2) of a (r, 2n) 0/1 matrix."""
    A = rows.copy() % 2
    r = 0
    R, C = A.shape
    for col in range(C):
        piv = [i for i in range(r, R) if A[i, col]]
        if not piv:
            continue
        p = piv[0]
        A[[r, p]] = A[[p, r]]
        for i in range(R):
            if i != r and A[i, col]:
                A[i] ^= A[r]
        r += 1
        if r == R:
            break
    return A


def gf2_rank(rows: np.ndarray) -> int:
    A = rref(rows)
    return int(np.sum(np.any(A, axis=1)))


def symplectic(a: np.ndarray, b: np.ndarray, n: int) -> int:
    return int((np.dot(a[:n], b[n:]) + np.dot(a[n:], b[:n])) % 2)


class TableauTrack:
    """Unsigned generators of the group G_t (section 3): conjugated by each
    Clifford gate, and on a random non-Clifford gate or measurement of q
    replaced by {g in G : g commutes with Z_q} together with Z_q (forced-outcome
    measurement, section 2.2).  Rows are n x 2n bits [x | z]."""

    def __init__(self, n: int):
        self.n = n
        self.rows = np.zeros((n, 2 * n), dtype=np.uint8)
        for q in range(n):
            self.rows[q, n + q] = 1

    def canonical(self) -> np.ndarray:
        return rref(self.rows)

    def conjugate(self, op, a, b=0):
        n, R = self.n, self.rows
        xa, za = R[:, a].copy(), R[:, n + a].copy()
        if op == H:
            R[:, a], R[:, n + a] = za, xa
        elif op in (S, SDG):
            R[:, n + a] = za ^ xa
        elif op in (X, Y, Z):
            pass
        elif op == CNOT:
            R[:, b] ^= xa
            R[:, n + a] ^= R[:, n + b]
        elif op == CZ:
            xb = R[:, b].copy()
            R[:, n + a] ^= xb
            R[:, n + b] ^= xa
        else:
            raise ValueError(op)

    def cofactor(self, q):
        n = self.n
        zq = np.zeros(2 * n, dtype=np.uint8)
        zq[n + q] = 1
        anti = [i for i in range(n) if symplectic(self.rows[i], zq, n)]
        if not anti:
            return False
        p = anti[0]
        for i in anti[1:]:
            self.rows[i] ^= self.rows[p]
        self.rows[p] = zq
        return True


# ---------------------------------------------------------------------------
# The canonical basis and the frame as a basis expansion
# ---------------------------------------------------------------------------

def canonical_state(M: np.ndarray, sigma, n: int) -> np.ndarray:
    """The stabilizer state with generators (-1)^{sigma_i} row_i, with a real
    positive amplitude at the smallest basis index of its support."""
    dim = 1 << n
    rng = np.random.default_rng(12345)
    v = rng.standard_normal(dim) + 1j * rng.standard_normal(dim)
    for i in range(n):
        g = pauli_apply(M[i, :n], M[i, n:], v, n)
        v = (v + (-1) ** int(sigma[i]) * g) / 2
    nrm = np.linalg.norm(v)
    if nrm < 1e-8:
        raise ValueError("generators do not define a state")
    v = v / nrm
    first = int(np.argmax(np.abs(v) > 1e-9))
    v = v * (abs(v[first]) / v[first])
    return v


def sigma_to_int(sigma) -> int:
    return sum(int(b) << i for i, b in enumerate(sigma))


def frame_expansion(M: np.ndarray, psi: np.ndarray, n: int, eps: float = 1e-12):
    """All (sigma, a) with a = <psi_can(M, sigma)|psi> and |a| > eps, in
    canonical order (ascending sum_i sigma_i 2^i)."""
    out = []
    for s in range(1 << n):
        sigma = [(s >> i) & 1 for i in range(n)]
        a = np.vdot(canonical_state(M, sigma, n), psi)
        if abs(a) > eps:
            out.append((s, complex(a)))
    return out


def frame_expansion_fast(M: np.ndarray, psi: np.ndarray, n: int, eps: float = 1e-12):
    """Same set as frame_expansion, found by projecting psi on the joint
    eigenspaces: amplitudes only need the canonical states whose projection is
    non-zero, found by splitting psi over the generators one at a time."""
    branches = [((), psi)]
    for i in range(n):
        g_i = lambda v, i=i: pauli_apply(M[i, :n], M[i, n:], v, n)
        nxt = []
        for signs, v in branches:
            gv = g_i(v)
            for s in (0, 1):
                w = (v + (-1) ** s * gv) / 2
                if np.linalg.norm(w) > eps * 1e-3:
                    nxt.append((signs + (s,), w))
        branches = nxt
    out = []
    for signs, w in branches:
        a = np.vdot(canonical_state(M, signs, n), psi)
        if abs(a) > eps:
            out.append((sigma_to_int(signs), complex(a)))
    out.sort()
    return out


def measurement_u(seed: int, index: int) -> float:
    """SplitMix64 output ``index`` of the stream started at ``seed`` (published
    definition: golden-ratio increment, two xor-shift-multiply rounds and a
    final xor-shift), top 53 bits scaled to [0, 1)."""
    M64 = (1 << 64) - 1
    z = (seed + (index + 1) * 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    z ^= z >> 31
    return (z >> 11) * 2.0 ** -53


def simulate(n: int, gates, init_bits=None, seed: int = 0, trace: bool = False):
    """Run the circuit on a dense vector and on the tableau track.

    Returns (psi, canonical M, outcomes); with ``trace`` also a list of
    (psi, M) after every gate.  A measurement's outcome is 1 exactly when the
    seeded uniform is below p(1)."""
    psi = basis_state(n, init_bits if init_bits is not None else [0] * n)
    track = TableauTrack(n)
    outcomes, hist = [], []
    nmeas = 0
    for g in gates:
        op, q0, q1, q2, num, den = (int(v) for v in g)
        if op in (H, S, SDG, X, Y, Z, CNOT, CZ):
            psi = apply_gate(psi, n, op, q0, q1)
            track.conjugate(op, q0, q1)
        elif op in (T, TDG, PHASE):
            if op == PHASE and (2 * num) % den == 0:
                m = ((2 * num) // den) % 4
                psi = apply_gate(psi, n, op, q0, num=num, den=den)
                if m in (1, 3):
                    track.conjugate(S, q0)
            else:
                psi = apply_gate(psi, n, op, q0, num=num, den=den)
                track.cofactor(q0)
        elif op == CPHASE:
            psi = apply_gate(psi, n, op, q0, q1, num=num, den=den)
            raise NotImplementedError("tableau track of CPHASE: expand it first")
        elif op == CPHASE_D:
            # the direct form (Eq. 3): cofactor on both qubits, unless theta is
            # a multiple of pi (identity or CZ)
            psi = apply_gate(psi, n, op, q0, q1, num=num, den=den)
            if den < 0:
                num, den = -num, -den
            if num % den == 0:
                if (num // den) % 2:
                    track.conjugate(CZ, q0, q1)
            else:
                track.cofactor(q0)
                track.cofactor(q1)
        elif op == TOF_D:
            # the direct form (Eq. 2): cofactor on both controls; the X on the
            # target leaves the unsigned matrix as it is
            psi = apply_gate(psi, n, op, q0, q1, q2)
            track.cofactor(q0)
            track.cofactor(q1)
        elif op == MEASURE:
            p1 = qubit_prob1(psi, n, q0)
            u = measurement_u(seed, nmeas)
            nmeas += 1
            o = int(u < p1)
            psi = project(psi, n, q0, o)
            outcomes.append(o)
            track.cofactor(q0)
        else:
            raise ValueError(op)
        if trace:
            hist.append((psi.copy(), track.canonical()))
    if trace:
        return psi, track.canonical(), outcomes, hist
    return psi, track.canonical(), outcomes
