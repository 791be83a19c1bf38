"""Seeded synthetic circuit generators (inputs only).

This module builds gate lists and draws random numbers; it contains none of
the stabilizer-frame arithmetic.  Both the HIP library and the CPU oracle
consume what it produces, so it is the only code the two sides share.

Gate records use the layout of ``sf_gate`` in ``include/sframe.h``:
``(op:u32, q0:u32, q1:u32, q2:u32, num:i64, den:i64)``; a phase gate applies
``diag(1, exp(i*pi*num/den))``.

Workload shapes follow the evaluation section of Garcia & Markov (random
stabilizer circuits of section 6 with H/P/CNOT drawn with probability 1/3
each; Cuccaro adders on an equal superposition; QFT on basis states) plus the
batched mixes (Steane-code fault-injection trials, uneven random circuits) and
the served mix (AQFT, Cuccaro adders, one uneven circuit).
"""
from __future__ import annotations

import numpy as np

# Operation codes: an interface shared with include/sframe.h (same numbers).
H, S, SDG, X, Y, Z, CNOT, CZ, T, TDG, PHASE, CPHASE, TOF, MEASURE, CPHASE_D, TOF_D = range(16)
OP_NAMES = ["H", "S", "SDG", "X", "Y", "Z", "CNOT", "CZ", "T", "TDG", "PHASE",
            "CPHASE", "TOF", "MEASURE", "CPHASE_D", "TOF_D"]

GATE_DTYPE = np.dtype([("op", "<u4"), ("q0", "<u4"), ("q1", "<u4"), ("q2", "<u4"),
                       ("num", "<i8"), ("den", "<i8")])
assert GATE_DTYPE.itemsize == 32

MASTER_SEED = 20171210
_GOLDEN = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def splitmix64(state: int, index: int = 0) -> int:
    """Output ``index`` (0-based) of a SplitMix64 stream started at ``state``.

    Published definition (Steele, Lea & Flood 2014; Vigna's splitmix64.c):
    the state advances by the golden-ratio increment and each output is the
    state passed through the two xor-shift-multiply rounds and a final
    xor-shift.
    """
    z = (state + (index + 1) * _GOLDEN) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def derive_seed(config_id: int, job_index: int) -> int:
    """Seed of one job of one workload, from the fixed master seed."""
    return splitmix64(MASTER_SEED ^ (config_id << 32) ^ job_index)


def measurement_uniform(seed: int, meas_index: int) -> float:
    """The uniform in [0,1) that decides measurement ``meas_index`` of a run.

    53 high bits of SplitMix64 output ``meas_index`` scaled by 2^-53; the
    outcome of a measurement is 1 exactly when this value is below p(1).
    Exposed here only so tests can state expected outcomes; both the oracle
    and the library implement the generator themselves.
    """
    return (splitmix64(seed, meas_index) >> 11) * (1.0 / 9007199254740992.0)


class Circuit:
    """A gate list on ``n`` qubits plus the initial basis state."""

    def __init__(self, n: int, init_bits=None, name: str = ""):
        self.n = int(n)
        self.gates: list[tuple] = []
        self.init_bits = [0] * self.n if init_bits is None else [int(b) & 1 for b in init_bits]
        self.name = name

    # builders -----------------------------------------------------------
    def add(self, op, q0=0, q1=0, q2=0, num=0, den=1):
        self.gates.append((int(op), int(q0), int(q1), int(q2), int(num), int(den)))
        return self

    def h(self, q): return self.add(H, q)
    def s(self, q): return self.add(S, q)
    def sdg(self, q): return self.add(SDG, q)
    def x(self, q): return self.add(X, q)
    def y(self, q): return self.add(Y, q)
    def z(self, q): return self.add(Z, q)
    def cnot(self, c, t): return self.add(CNOT, c, t)
    def cz(self, c, t): return self.add(CZ, c, t)
    def t(self, q): return self.add(T, q)
    def tdg(self, q): return self.add(TDG, q)
    def phase(self, q, num, den): return self.add(PHASE, q, 0, 0, num, den)
    def measure(self, q): return self.add(MEASURE, q)
    def cphase_direct(self, c, t, num, den): return self.add(CPHASE_D, c, t, 0, num, den)
    def toffoli_direct(self, c1, c2, t): return self.add(TOF_D, c1, c2, t)

    def cphase_decomposed(self, c, t, num, den):
        """Controlled phase diag(1,1,1,e^{i*pi*num/den}) as three phase gates and two CNOTs.

        Uses phi*c*t = phi/2*(c + t - (c xor t)): phase phi/2 on the target,
        CNOT, phase -phi/2 on the target (now holding c xor t), CNOT back,
        phase phi/2 on the control.
        """
        self.phase(t, num, 2 * den)
        self.cnot(c, t)
        self.phase(t, -num, 2 * den)
        self.cnot(c, t)
        self.phase(c, num, 2 * den)
        return self

    def toffoli_7t(self, c1, c2, t):
        """Toffoli as the textbook network of 2 H, 6 CNOT and 7 T/T-dagger gates."""
        self.h(t)
        self.cnot(c2, t); self.tdg(t)
        self.cnot(c1, t); self.t(t)
        self.cnot(c2, t); self.tdg(t)
        self.cnot(c1, t); self.t(c2); self.t(t)
        self.h(t)
        self.cnot(c1, c2); self.t(c1); self.tdg(c2)
        self.cnot(c1, c2)
        return self

    def array(self) -> np.ndarray:
        a = np.zeros(len(self.gates), dtype=GATE_DTYPE)
        for i, g in enumerate(self.gates):
            a[i] = g
        return a

    def __len__(self):
        return len(self.gates)

    def count(self, ops) -> int:
        ops = set(ops)
        return sum(1 for g in self.gates if g[0] in ops)


# ----------------------------------------------------------------------------
# Random Clifford + T circuits (configurations 1, 2, 4 and 2-L)
# ----------------------------------------------------------------------------

def random_clifford_t(n: int, n_cliff: int, n_t: int, seed: int, measure_qubits=(),
                      name: str = "") -> Circuit:
    """``n_cliff`` gates uniform over {H, S, CNOT} (CNOT on a uniform ordered
    pair of distinct qubits), with ``n_t`` T gates on uniform qubits placed at
    distinct uniform slots among the ``n_cliff + n_t`` positions, then
    Z-basis measurements of ``measure_qubits`` in order."""
    rng = np.random.default_rng(seed)
    total = n_cliff + n_t
    t_slots = set(rng.choice(total, size=n_t, replace=False).tolist()) if n_t else set()
    c = Circuit(n, name=name)
    for slot in range(total):
        if slot in t_slots:
            c.t(int(rng.integers(n)))
            continue
        kind = int(rng.integers(3))
        if kind == 0:
            c.h(int(rng.integers(n)))
        elif kind == 1:
            c.s(int(rng.integers(n)))
        else:
            a = int(rng.integers(n))
            b = int(rng.integers(n - 1))
            if b >= a:
                b += 1
            c.cnot(a, b)
    for q in measure_qubits:
        c.measure(int(q))
    return c


def stabilizer_circuit(n: int, seed: int, beta: float = 1.0) -> Circuit:
    """Random stabilizer circuit of the paper's Clifford-only experiments
    (section 6): ceil(beta n log2 n) gates uniform over {H, S, CNOT}, then a
    Z measurement of every qubit."""
    gates = int(np.ceil(beta * n * np.log2(n)))
    return random_clifford_t(n, gates, 0, seed, measure_qubits=range(n), name=f"stab-n{n}")


def config1(job: int) -> Circuit:
    """n=8 from |0^8>: 200 Cliffords, 4 T, then measure qubits 0..7."""
    return random_clifford_t(8, 200, 4, derive_seed(1, job), measure_qubits=range(8),
                             name=f"cfg1-{job}")


def config2(job: int, n_t: int = 16) -> Circuit:
    """n=128 from |0^128>: 2000 Cliffords, ``n_t`` T, then measure 16 distinct uniform qubits."""
    seed = derive_seed(2 if n_t == 16 else 22, job)
    rng = np.random.default_rng(seed ^ 0xA5A5)
    mq = rng.choice(128, size=16, replace=False).tolist()
    return random_clifford_t(128, 2000, n_t, seed, measure_qubits=mq,
                             name=f"cfg2-{job}" if n_t == 16 else f"cfg2L{n_t}-{job}")


def config4(job: int) -> Circuit:
    """n uniform in [16,256], 10n Cliffords, T count uniform in [0,12], no measurement."""
    seed = derive_seed(4, job)
    rng = np.random.default_rng(seed ^ 0x5A5A)
    n = int(rng.integers(16, 257))
    t = int(rng.integers(0, 13))
    return random_clifford_t(n, 10 * n, t, seed, name=f"cfg4-{job}")


# ----------------------------------------------------------------------------
# Steane-code fault injection (configuration 3)
# ----------------------------------------------------------------------------

# [7,4] Hamming parity checks on data qubits 0..6 (column j+1 written in binary).
HAMMING_CHECKS = ((0, 2, 4, 6), (1, 2, 5, 6), (3, 4, 5, 6))


def steane_base() -> Circuit:
    """Encoder of |+_L> on data qubits 0..6, T on data qubit 0, then three
    X-checks (ancillas 7..9) and three Z-checks (ancillas 10..12), without the
    final measurements.

    The encoder puts the information qubits 2,4,5,6 in |+> and copies them to
    the parity qubits 0,1,3 with CNOTs, which yields the uniform superposition
    of the 16 Hamming codewords.
    """
    c = Circuit(13, name="steane")
    for q in (2, 4, 5, 6):
        c.h(q)
    for info, parity in ((2, 0), (4, 0), (6, 0), (2, 1), (5, 1), (6, 1), (4, 3), (5, 3), (6, 3)):
        c.cnot(info, parity)
    c.t(0)
    for k, sup in enumerate(HAMMING_CHECKS):      # X-checks
        a = 7 + k
        c.h(a)
        for d in sup:
            c.cnot(a, d)
        c.h(a)
    for k, sup in enumerate(HAMMING_CHECKS):      # Z-checks
        a = 10 + k
        for d in sup:
            c.cnot(d, a)
    return c


def config3(trial: int) -> Circuit:
    """One fault-injection trial: a uniform Pauli on a uniform qubit after a
    uniform gate of the Steane circuit, then the six ancilla measurements."""
    base = steane_base()
    rng = np.random.default_rng(derive_seed(3, trial))
    g = int(rng.integers(len(base.gates)))
    q = int(rng.integers(13))
    p = (X, Y, Z)[int(rng.integers(3))]
    c = Circuit(13, name=f"cfg3-{trial}")
    for i, gate in enumerate(base.gates):
        c.gates.append(gate)
        if i == g:
            c.add(p, q)
    for a in range(7, 13):
        c.measure(a)
    c.fault = (g, q, p)
    return c


# ----------------------------------------------------------------------------
# QFT and Cuccaro adder (configuration 5)
# ----------------------------------------------------------------------------

def qft(n: int, x_bits, max_k=None, name: str = "qft", direct: bool = False) -> Circuit:
    """QFT circuit without the final swaps on the basis state |x_bits>.

    Qubit j gets H and then controlled rotations R_k = diag(1, e^{2 pi i/2^k})
    from qubits j+1.., with k = distance + 1; rotations with k > max_k are
    dropped (approximate QFT).  Each controlled rotation is written as three
    phase gates and two CNOTs, or with ``direct`` as one direct controlled
    phase (double cofactor).
    """
    c = Circuit(n, init_bits=x_bits, name=name)
    for j in range(n):
        c.h(j)
        for ctl in range(j + 1, n):
            k = ctl - j + 1
            if max_k is not None and k > max_k:
                continue
            # 2*pi/2^k = pi * 1/2^(k-1)
            if direct:
                c.cphase_direct(ctl, j, 1, 1 << (k - 1))
            else:
                c.cphase_decomposed(ctl, j, 1, 1 << (k - 1))
    return c


def cuccaro_adder(m: int, a_bits=None, b_bits=None, superpose=True, name="cuccaro",
                  direct: bool = False) -> Circuit:
    """Cuccaro ripple-carry adder of two m-bit registers (2m+2 qubits).

    Layout: qubit 0 is the ancilla c0, qubits 1+2i and 2+2i hold b_i and a_i,
    qubit 2m+1 is the carry z.  With ``superpose`` every input qubit first gets
    an H.  Toffolis are 7-T networks, or direct (double cofactor) with ``direct``.  On basis inputs the b register ends up
    holding a+b mod 2^m and z the carry out.
    """
    nq = 2 * m + 2
    init = [0] * nq
    if a_bits is not None:
        for i in range(m):
            init[2 + 2 * i] = int(a_bits[i])
            init[1 + 2 * i] = int(b_bits[i])
    c = Circuit(nq, init_bits=init, name=name)
    A = lambda i: 2 + 2 * i
    B = lambda i: 1 + 2 * i
    zq = 2 * m + 1
    if superpose:
        for i in range(m):
            c.h(A(i))
            c.h(B(i))

    tof = c.toffoli_direct if direct else c.toffoli_7t

    def maj(x, y, w):
        c.cnot(w, y); c.cnot(w, x); tof(x, y, w)

    def uma(x, y, w):
        tof(x, y, w); c.cnot(w, x); c.cnot(x, y)

    maj(0, B(0), A(0))
    for i in range(1, m):
        maj(A(i - 1), B(i), A(i))
    c.cnot(A(m - 1), zq)
    for i in range(m - 1, 0, -1):
        uma(A(i - 1), B(i), A(i))
    uma(0, B(0), A(0))
    return c


def config5_job(job: int, direct: bool = False) -> Circuit:
    """One served request: 40% AQFT, 40% Cuccaro adder, 20% config-4 shape.
    With ``direct`` the controlled rotations and Toffolis use the direct
    (double-cofactor) forms; the draws are the same."""
    seed = derive_seed(5, job)
    rng = np.random.default_rng(seed)
    u = rng.random()
    if u < 0.4:
        n = int(rng.integers(10, 21))
        x = rng.integers(0, 2, size=n).tolist()
        return qft(n, x, max_k=6, name=f"cfg5a-{job}", direct=direct)
    if u < 0.8:
        m = int(rng.integers(8, 33))
        return cuccaro_adder(m, name=f"cfg5b-{job}", direct=direct)
    c = config4(100000 + job)
    c.name = f"cfg5c-{job}"
    return c
