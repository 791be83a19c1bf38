"""The seeded synthetic inputs follow their stated recipes (no GPU needed):
gate counts and kinds, qubit ranges, measured qubits, the Steane encoder's
code state (checked on the dense state vector), the served mix's shares and
size ranges, and distinct seeds."""
import math

import numpy as np
import pytest

from oracle import dense
from paper_1712_03554_amd import workloads as wl

CLIFFORD_DRAWS = (wl.H, wl.S, wl.CNOT)


def _count(c, ops):
    return sum(1 for g in c.gates if g[0] in ops)


@pytest.mark.parametrize("job", [0, 1, 9])
def test_config1_recipe(job):
    c = wl.config1(job)
    assert c.n == 8 and list(c.init_bits) == [0] * 8
    body, tail = c.gates[:-8], c.gates[-8:]
    assert [g[0] for g in tail] == [wl.MEASURE] * 8 and [g[1] for g in tail] == list(range(8))
    assert len(body) == 204 and _count(c, (wl.T,)) == 4
    assert all(g[0] in CLIFFORD_DRAWS + (wl.T,) for g in body)
    assert all(g[1] != g[2] for g in body if g[0] == wl.CNOT)


@pytest.mark.parametrize("n_t", [16, 24])
def test_config2_recipe(n_t):
    for job in range(3):
        c = wl.config2(job, n_t)
        assert c.n == 128 and list(c.init_bits) == [0] * 128
        body, tail = c.gates[:-16], c.gates[-16:]
        assert all(g[0] == wl.MEASURE for g in tail)
        assert len({g[1] for g in tail}) == 16
        assert len(body) == 2000 + n_t and _count(c, (wl.T,)) == n_t
        assert all(g[0] in CLIFFORD_DRAWS + (wl.T,) for g in body)
    # the three Clifford kinds are drawn uniformly
    c = wl.config2(0)
    k = np.array([_count(c, (op,)) for op in CLIFFORD_DRAWS])
    assert np.all(np.abs(k - 2000 / 3) < 5 * math.sqrt(2000 * (1 / 3) * (2 / 3))), k


def test_steane_encoder_prepares_the_logical_plus_state():
    """The encoder part of the Steane circuit (before T and the checks)
    leaves data qubits 0..6 stabilized by the X- and Z-type Hamming checks
    and by the logical X (X on all seven)."""
    base = wl.steane_base()
    t_at = next(i for i, g in enumerate(base.gates) if g[0] == wl.T)
    psi, _, _ = dense.simulate(7, base.gates[:t_at])
    n = 7
    for sup in wl.HAMMING_CHECKS:
        for kind in ("x", "z"):
            x = np.zeros(n, dtype=np.uint8)
            z = np.zeros(n, dtype=np.uint8)
            (x if kind == "x" else z)[list(sup)] = 1
            assert np.allclose(dense.pauli_apply(x, z, psi, n), psi, atol=1e-12), (kind, sup)
    assert np.allclose(dense.pauli_apply(np.ones(n, dtype=np.uint8), np.zeros(n, dtype=np.uint8), psi, n), psi,
                       atol=1e-12)


@pytest.mark.parametrize("trial", [0, 5, 4095])
def test_config3_recipe(trial):
    base = wl.steane_base()
    c = wl.config3(trial)
    assert c.n == 13 and len(c.gates) == len(base.gates) + 1 + 6
    g, q, p = c.fault
    assert 0 <= g < len(base.gates) and 0 <= q < 13 and p in (wl.X, wl.Y, wl.Z)
    assert c.gates[g + 1] == (p, q, 0, 0, 0, 1)
    assert [x[1] for x in c.gates[-6:]] == list(range(7, 13))


def test_config4_recipe():
    ns, ts = [], []
    for job in range(200):
        c = wl.config4(job)
        n_t = _count(c, (wl.T,))
        assert 16 <= c.n <= 256 and 0 <= n_t <= 12
        assert len(c.gates) == 10 * c.n + n_t and _count(c, (wl.MEASURE,)) == 0
        ns.append(c.n)
        ts.append(n_t)
    assert min(ns) < 40 and max(ns) > 230 and set(range(13)) <= set(ts)


def test_config5_mix_shares_and_sizes():
    kinds = {"a": 0, "b": 0, "c": 0}
    for job in range(600):
        c = wl.config5_job(job)
        kind = c.name.split("-")[0][-1]
        kinds[kind] += 1
        if kind == "a":
            assert 10 <= c.n <= 20
            # no rotation beyond k = 6: every phase angle is pi / 2^(k-1) / 2 with k <= 6
            assert all(g[5] <= 2 ** 6 for g in c.gates if g[0] == wl.PHASE)
        elif kind == "b":
            m = (c.n - 2) // 2
            assert c.n % 2 == 0 and 8 <= m <= 32
        else:
            assert 16 <= c.n <= 256
    share = {k: v / 600 for k, v in kinds.items()}
    sd = math.sqrt(0.4 * 0.6 / 600)
    assert abs(share["a"] - 0.4) < 5 * sd and abs(share["b"] - 0.4) < 5 * sd and abs(share["c"] - 0.2) < 5 * sd


@pytest.mark.parametrize("n,beta", [(8, 1.0), (512, 1.0), (1500, 1.0), (2048, 0.08)])
def test_stabilizer_circuit_recipe(n, beta):
    c = wl.stabilizer_circuit(n, 5, beta)
    gates = int(math.ceil(beta * n * math.log2(n)))
    assert len(c.gates) == gates + n
    assert all(g[0] in CLIFFORD_DRAWS for g in c.gates[:gates])
    assert [g[1] for g in c.gates[gates:]] == list(range(n))


def test_seeds_are_distinct():
    for cfg in (1, 2, 3, 4, 5):
        seeds = {wl.derive_seed(cfg, j) for j in range(5000)}
        assert len(seeds) == 5000
    assert len({wl.derive_seed(cfg, 0) for cfg in range(1, 6)}) == 5
