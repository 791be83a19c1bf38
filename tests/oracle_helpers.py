"""Helpers shared by the oracle pin tests and the GPU parity tests."""
from __future__ import annotations

import numpy as np

from oracle import dense
from oracle.frame import OracleFrame

AMP_RTOL = 1e-10
AMP_ATOL = 1e-13


def tableau_bits(tab_words: np.ndarray, n: int) -> np.ndarray:
    """[n, 2W] uint64 words -> [n, 2n] 0/1 matrix [x | z]."""
    W = (n + 63) // 64
    out = np.zeros((n, 2 * n), dtype=np.uint8)
    for i in range(n):
        for q in range(n):
            out[i, q] = (int(tab_words[i, q >> 6]) >> (q & 63)) & 1
            out[i, n + q] = (int(tab_words[i, W + (q >> 6)]) >> (q & 63)) & 1
    return out


def sigma_ints(sig_words: np.ndarray) -> list[int]:
    out = []
    for row in sig_words:
        v = 0
        for w, word in enumerate(row):
            v |= int(word) << (64 * w)
        out.append(v)
    return out


def assert_frames_equal(sig_a, amp_a, sig_b, amp_b, what=""):
    """sigma lists bit-exact (same canonical order), amplitudes within the
    1e-10 relative bound."""
    assert list(sig_a) == list(sig_b), f"{what}: phase-vector sets differ ({len(sig_a)} vs {len(sig_b)})"
    a = np.asarray(amp_a, dtype=complex)
    b = np.asarray(amp_b, dtype=complex)
    err = np.abs(a - b)
    bound = AMP_RTOL * np.abs(b) + AMP_ATOL
    assert np.all(err <= bound), f"{what}: amplitude mismatch, worst {np.max(err / bound)} x bound"


def oracle_vs_dense(circ, seed: int = 0, every_gate: bool = True):
    """Run the C oracle gate by gate and the dense checker; compare tableau,
    frame and outcomes after every gate (or only at the end)."""
    n = circ.n
    gates = circ.gates
    psi, M, outs, hist = dense.simulate(n, gates, circ.init_bits, seed=seed, trace=True)
    f = OracleFrame(n, circ.init_bits, seed)
    for gi, g in enumerate(gates):
        f.apply(*g)
        if not every_gate and gi != len(gates) - 1:
            continue
        psi_g, M_g = hist[gi]
        tab, sig, amp = f.read()
        assert np.array_equal(tableau_bits(tab, n), M_g), f"gate {gi}: tableau differs"
        exp = dense.frame_expansion_fast(M_g, psi_g, n)
        assert_frames_equal(sigma_ints(sig), amp, [s for s, _ in exp], [a for _, a in exp],
                            what=f"gate {gi} {g}")
    assert f.outcomes() == outs
    assert not f.fragile
    return f


def oracle_config4(job: int):
    """The oracle's result for uneven circuit `job` (tableau, sigma, amplitudes,
    outcomes, fragile flag); a top-level function so that a process pool can
    run it."""
    from paper_1712_03554_amd import workloads as wl
    c = wl.config4(job)
    f = OracleFrame(c.n, c.init_bits, wl.derive_seed(4, job))
    f.run(c.array())
    tab, sig, amp = f.read()
    return tab, sig, amp, f.outcomes(), f.fragile


def oracle_config2(job: int):
    """As oracle_config4, for the n = 128 Clifford+T circuit `job`."""
    from paper_1712_03554_amd import workloads as wl
    c = wl.config2(job)
    f = OracleFrame(c.n, c.init_bits, wl.derive_seed(2, job))
    f.run(c.array())
    tab, sig, amp = f.read()
    return tab, sig, amp, f.outcomes(), f.fragile


def oracle_stabilizer(n: int, circuit_seed: int, beta: float, seed: int):
    """Oracle frame (tableau, sigma, amp), outcomes and fragile flag of the
    random stabilizer circuit of n qubits (for process pools)."""
    from oracle.frame import OracleFrame
    from paper_1712_03554_amd import workloads as wl
    c = wl.stabilizer_circuit(n, circuit_seed, beta)
    f = OracleFrame(c.n, c.init_bits, seed)
    f.run(c.array())
    return f.read(), f.outcomes(), f.fragile


def oracle_pool(workers: int = 16):
    """A process pool for oracle runs (spawned: no state of the parent's GPU
    runtime is inherited), at most `workers` processes."""
    import multiprocessing as mp
    import os
    from concurrent.futures import ProcessPoolExecutor
    n = max(1, min(workers, os.cpu_count() or 1))
    return ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("spawn"))


def assert_frame_arrays_equal(sig_a, amp_a, sig_b, amp_b, what=""):
    """As assert_frames_equal, on (K, W) word arrays without conversion to
    integers (for frames of millions of elements)."""
    assert sig_a.shape == sig_b.shape, f"{what}: {sig_a.shape[0]} vs {sig_b.shape[0]} elements"
    assert np.array_equal(sig_a, sig_b), f"{what}: phase vectors differ"
    err = np.abs(np.asarray(amp_a) - np.asarray(amp_b))
    bound = AMP_RTOL * np.abs(amp_b) + AMP_ATOL
    assert np.all(err <= bound), f"{what}: amplitude mismatch, worst {np.max(err / bound)} x bound"
