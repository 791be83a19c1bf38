"""Host checks of the benchmark's bookkeeping (no GPU needed): the per-gate
record size used for the phase kernel's bytes, the Clifford gate count, the
segment ends, and the U count (sum over gates of |F| just before the gate)
taken segment by segment against the oracle's gate-by-gate frame sizes."""
import math
import os
import re

import pytest

import bench
from oracle.frame import OracleFrame
from paper_1712_03554_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _dev_define(name):
    text = open(os.path.join(ROOT, "paper_1712_03554_amd", "csrc", "sf_dev.h")).read()
    return int(re.search(rf"#define {name} (\d+)", text).group(1))


@pytest.mark.parametrize("n", [1, 2, 8, 63, 64, 65, 100, 127, 128])
def test_record_stride_is_the_record_layout(n):
    """x and z rows of n slots of W words, SF_DMAX + 1 hull vectors of W
    words and an 8-byte dimension, padded to a 256-byte boundary."""
    W = -(-n // 64)
    raw = 8 * (2 * n * W + (_dev_define("SF_DMAX") + 1) * W) + 8
    s = bench.rec_stride(n)
    assert s % 256 == 0 and raw <= s < raw + 256


def _circuit(gates, n=3):
    c = wl.Circuit(n)
    for g in gates:
        c.add(*g)
    return c


def test_clifford_count_and_segment_ends():
    c = _circuit([(wl.H, 0), (wl.T, 1), (wl.PHASE, 0, 0, 0, 1, 2), (wl.PHASE, 1, 0, 0, 4, 2),
                  (wl.PHASE, 2, 0, 0, 2, 2), (wl.PHASE, 0, 0, 0, 1, 4), (wl.CNOT, 0, 1),
                  (wl.MEASURE, 2), (wl.TDG, 0), (wl.CZ, 1, 2), (wl.PHASE, 1, 0, 0, -1, 2),
                  (wl.SDG, 2), (wl.X, 0), (wl.Y, 1), (wl.Z, 2)])
    # H, S-angle, Z-angle, CNOT, CZ, -pi/2, SDG, X, Y, Z: ten Clifford gates;
    # the identity angle (4 pi/2) is dropped, T, TDG and pi/4 end segments
    assert bench.clifford_gate_count(c, wl) == 10
    assert bench.terminal_indices(c, wl) == [1, 5, 7, 8]
    with pytest.raises(ValueError):
        bench.terminal_indices(_circuit([(wl.TOF, 0, 1, 2)]), wl)
    with pytest.raises(ValueError):
        bench.terminal_indices(_circuit([(wl.CPHASE, 0, 1, 0, 1, 4)]), wl)


def test_random_clifford_t_counts():
    c = wl.config2(0)
    assert bench.clifford_gate_count(c, wl) == 2000
    ends = bench.terminal_indices(c, wl)
    assert len(ends) == 32 and ends[-16:] == list(range(len(c) - 16, len(c)))
    assert all(c.gates[i][0] == wl.T for i in ends[:16])


class _OracleState:
    """The few state calls the U count makes, on the oracle."""

    def __init__(self, circ):
        self.circ = circ

    def reset(self, bits, seed):
        self.f = OracleFrame(self.circ.n, bits, seed)
        self.pos = 0

    def step(self, k):
        for g in self.circ.gates[self.pos:self.pos + k]:
            self.f.apply(*g)
        self.pos += k
        return k

    def frame_size(self):
        return self.f.size

    def dim(self):
        return math.ceil(math.log2(self.f.size))


@pytest.mark.parametrize("make", [lambda: wl.config1(0), lambda: wl.config1(3),
                                  lambda: wl.random_clifford_t(10, 120, 5, 77),
                                  lambda: wl.random_clifford_t(6, 40, 0, 78)])
def test_segment_u_count_matches_gate_by_gate_sizes(make):
    """Frame sizes change only at segment ends, so summing |F| per segment
    gives the gate-by-gate sum; the segment list covers a tail after the
    last terminal gate and circuits without any."""
    c = make()
    seed = 4242
    sizes, meas = [], []
    U, seg_dims = bench.accounting(_OracleState(c), c, seed, wl, sizes=sizes, meas=meas)
    ref = OracleFrame(c.n, c.init_bits, seed).run(c.array())
    assert U == int(ref.sum())
    ends = bench.terminal_indices(c, wl)
    if not ends or ends[-1] != len(c) - 1:
        ends = ends + [len(c) - 1]
    starts = [0] + [e + 1 for e in ends[:-1]]
    assert sizes == [int(ref[s]) for s in starts]
    assert len(seg_dims) == len(ends) and seg_dims[0] == 0
    assert len(meas) == sum(1 for g in c.gates if g[0] == wl.MEASURE)


def _bench(*args):
    import subprocess
    import sys
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, capture_output=True,
                          text=True, timeout=300)


def test_bench_refuses_more_than_one_gpu():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_bench_fails_loudly_without_a_device():
    """No HIP device: the benchmark stops with the library's device error
    instead of measuring anything else."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a HIP device is present")
    r = _bench("--no-cpu", "--no-extra", "--serve-jobs", "0", "--steps", "1", "--warmup", "0")
    assert r.returncode != 0
    assert "SF_E_DEVICE" in r.stderr and '"value"' not in r.stdout
