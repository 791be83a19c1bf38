"""The library's host code under UndefinedBehaviorSanitizer (needs an MI355X):
the parity tests that drive the host-side runtime (circuit validation and
expansion, planning of batched rounds and their graph form, the serving
loop, ad-hoc measurement, readout, tuning, allocation failures, the
allocation-free entry point, wide frames) run in a child process against
the UBSan build of the library, compared with the oracle as usual.  Any
undefined behaviour aborts the child."""
import os
import subprocess
import sys

import pytest

import paper_1712_03554_amd as sf
from paper_1712_03554_amd import build as lib_build

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PARITY = ["expands_tof_and_cphase", "edge_cases", "invalid_circuits_rejected", "too_large_frame_rejected",
          "budget_rejects_state", "batch_matches_alone", "serve_mix_matches_alone", "serve_budget_cancel",
          "adhoc_measurement", "graph_replays_match_eager", "api_error_paths", "batch_reset_matches",
          "direct_in_batch_and_graph", "small_frames_same_alone", "tuning_roundtrip",
          "batch_mixes_large_and_small_hulls", "word_boundaries_and_max_qubits"]
WIDE = ["wide_limits_and_refusals", "wide_adhoc_measure_and_reset", "wide_frames_in_a_batch"]


def _env():
    env = dict(os.environ)
    env["SFRAME_LIB"] = lib_build.UBSAN_OUT
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:report_error_type=1"
    return env


@pytest.fixture(scope="module")
def ubsan_lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    if not os.path.exists(lib_build.UBSAN_OUT):
        pytest.fail(f"{lib_build.UBSAN_OUT} not built (paper_1712_03554_amd/build.py, ubsan=True)")
    return lib_build.UBSAN_OUT


def test_child_loads_the_sanitized_build(ubsan_lib):
    probe = ("import paper_1712_03554_amd as sf; sf.load_library(); "
             "m = open('/proc/self/maps').read(); "
             "print(sf.LIB_PATH); print('ubsan-runtime' if 'ubsan_standalone' in m else 'no-runtime'); "
             "print('lib-mapped' if sf.LIB_PATH in m else 'lib-missing')")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=_env(), capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = r.stdout.split()
    assert lines == [ubsan_lib, "ubsan-runtime", "lib-mapped"], r.stdout
    assert sf.LIB_PATH != ubsan_lib  # this process keeps the plain build


def test_host_paths_under_ubsan(ubsan_lib):
    sel = ["tests/test_gpu_parity.py", "tests/test_gpu_failures.py", "tests/test_gpu_wide.py",
           "tests/test_zz_no_alloc.py", "-k", " or ".join(PARITY + WIDE + ["allocat", "buffer_too_small", "noalloc"])]
    cmd = [sys.executable, "-u", "-m", "pytest", "-x", "-q", "-m", "gpu", "-p", "no:cacheprovider",
           "--timeout", "240", "--timeout-method", "thread"] + sel
    print("child:", " ".join(cmd), flush=True)
    r = subprocess.run(cmd, cwd=ROOT, env=_env(), capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    print(out[-3000:], flush=True)
    assert "runtime error:" not in out
    assert r.returncode == 0
    assert " passed" in r.stdout and " failed" not in r.stdout
