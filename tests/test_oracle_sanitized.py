"""The frame oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and run on circuits of one to four packed words per
row, and its multiframe simulation (basic COALESCE and COALESCE through the
basis circuit, merging, orthogonalization before measurements) on mixed
circuits and superposed Cuccaro adders: no sanitizer report, and the same
frame sizes and outcomes as the oracle library the other tests load."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.frame import OracleFrame, OracleMultiframe
from paper_1712_03554_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path_factory.mktemp("asan") / "frame_asan")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           os.path.join(ROOT, "oracle", "frame.c"), os.path.join(ROOT, "oracle", "frame_driver.c"), "-lm",
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    return exe


def _circuits():
    out = []
    for n in (5, 63, 64, 65, 128, 129, 200, 256):
        c = wl.random_clifford_t(n, 3 * n if n > 8 else 60, 6, 7300 + n)
        rng = np.random.default_rng(n)
        for g in [(wl.CZ, 0, n - 1, 0, 0, 1), (wl.PHASE, n - 1, 0, 0, 1, 8), (wl.SDG, n // 2, 0, 0, 0, 1),
                  (wl.Y, 0, 0, 0, 0, 1), (wl.X, n - 1, 0, 0, 0, 1), (wl.TDG, n // 3, 0, 0, 0, 1)]:
            c.gates.insert(int(rng.integers(len(c.gates) + 1)), g)
        for q in rng.permutation(n)[: min(n, 6)]:
            c.gates.insert(int(rng.integers(len(c.gates) + 1)), (wl.MEASURE, int(q), 0, 0, 0, 1))
        c.init_bits = rng.integers(0, 2, size=n).tolist()
        out.append(c)
    direct = wl.cuccaro_adder(3, direct=True)
    direct.gates += [(wl.CPHASE_D, 0, 5, 0, 1, 8), (wl.TOF, 1, 2, 3, 0, 1), (wl.CPHASE, 2, 4, 0, 1, 4)]
    out.append(direct)
    return out


@pytest.mark.parametrize("idx", range(9))
def test_oracle_clean_under_sanitizers(sanitized, idx):
    c = _circuits()[idx]
    seed = 11 + idx
    text = f"{c.n} {seed}\n" + " ".join(str(b) for b in c.init_bits) + f"\n{len(c.gates)}\n"
    text += "".join(" ".join(str(int(v)) for v in g) + "\n" for g in c.gates)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sanitized], input=text, capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-2000:]
    got = {k: v for k, _, v in (line.partition(" ") for line in r.stdout.strip().splitlines())}
    ref = OracleFrame(c.n, c.init_bits, seed)
    ref.run(c.array())
    assert int(got["K"]) == ref.size
    assert abs(float(got["norm"]) - 1.0) <= 1e-12
    assert [int(v) for v in got["outcomes"].split()] == ref.outcomes()


def _multi_circuits():
    from tests.test_oracle_multiframe import _random_mix
    out = [_random_mix(seed, 3 + seed % 3, 40) for seed in range(4)]
    for m, direct in ((3, False), (4, False), (3, True)):
        c = wl.cuccaro_adder(m, direct=direct)
        for q in range(c.n):
            c.measure(q)
        out.append(c)
    return out


@pytest.mark.parametrize("general", [False, True])
@pytest.mark.parametrize("idx", range(7))
def test_multiframe_oracle_clean_under_sanitizers(sanitized, idx, general):
    c = _multi_circuits()[idx]
    seed = 31 + idx
    text = f"{c.n} {seed}\n" + " ".join(str(b) for b in c.init_bits) + f"\n{len(c.gates)}\n"
    text += "".join(" ".join(str(int(v)) for v in g) + "\n" for g in c.gates)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sanitized, "general" if general else "multi"], input=text, capture_output=True, text=True,
                       env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-2000:]
    got = {k: v for k, _, v in (line.partition(" ") for line in r.stdout.strip().splitlines())}
    ref = OracleMultiframe(c.n, c.init_bits, seed)
    ref.set_general(general)
    ref.run(c.array())
    assert int(got["K"]) == ref.size and int(got["frames"]) == ref.nframes
    assert abs(float(got["norm"]) - 1.0) <= 1e-12
    assert [int(v) for v in got["outcomes"].split()] == ref.outcomes()
    assert int(got["orthogonal"]) == int(ref.orthogonal())
