"""Host-side checks of the C-ABI library (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_1712_03554_amd as sf
from paper_1712_03554_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sframe.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:sf_status|const char\*)\s+(sf_\w+)\(", text, re.M)))


def test_header_declares_binding_exports():
    assert _declared() == sorted(sf.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(sf.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(sf.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_enums_match_header():
    text = open(HEADER).read()
    for i, name in enumerate(wl.OP_NAMES):
        assert re.search(rf"SF_{name}\s*=\s*{i}\b", text), name
    for i, name in enumerate(sf.STATUS_NAMES):
        assert re.search(rf"{name}\s*=\s*{i}\b", text), name


def test_gate_record_layout():
    assert wl.GATE_DTYPE.itemsize == 32
    assert [wl.GATE_DTYPE.fields[k][1] for k in ("op", "q0", "q1", "q2", "num", "den")] == [0, 4, 8, 12, 16, 24]


def test_context_without_device_fails_cleanly():
    """With no HIP device the library reports SF_E_DEVICE instead of crashing."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    if not os.path.exists(sf.LIB_PATH):
        pytest.skip("library not built")
    L = sf.load_library()
    h = ctypes.c_void_p()
    st = L.sf_ctx_create(0, None, None, 0, ctypes.byref(h))
    assert st == sf.SF_E_DEVICE and not h.value


def test_engine_requires_library(monkeypatch, tmp_path):
    monkeypatch.setattr(sf, "_lib", None)
    with pytest.raises(ImportError):
        sf.load_library(str(tmp_path / "missing.so"))


def test_bench_refuses_more_than_one_gpu():
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip())["error"]


def test_basis_word_packing():
    """The batched reset's basis words (lists or an array of bits) equal the
    per-state packing: bit q in word q / 64, position q % 64."""
    import numpy as np
    from paper_1712_03554_amd import _basis_word_rows, _basis_words
    rng = np.random.default_rng(7)
    for n in (1, 13, 63, 64, 65, 128, 200, 256):
        rows = [rng.integers(0, 2, size=n).tolist() for _ in range(6)]
        ref = np.stack([_basis_words(n, r) for r in rows])
        assert np.array_equal(_basis_word_rows(rows, 6), ref)
        assert np.array_equal(_basis_word_rows(np.array(rows, dtype=np.uint8), 6), ref)
        q = int(rng.integers(n))
        one = [0] * n
        one[q] = 1
        w = _basis_word_rows([one], 1)[0]
        assert int(w[q >> 6]) == 1 << (q & 63) and int(w.sum()) == 1 << (q & 63)


def test_packed_bases_pass_through():
    """pack_bases gives the same words, and batch calls take them as they are
    (a plain uint64 array of 0/1 bits is still read as bits)."""
    import numpy as np
    from paper_1712_03554_amd import BasisWords, _basis_word_rows, pack_bases
    rng = np.random.default_rng(8)
    rows = [rng.integers(0, 2, size=130).tolist() for _ in range(5)]
    w = pack_bases(rows)
    assert isinstance(w, BasisWords) and w.shape == (5, 4) and w.dtype == np.uint64
    assert np.array_equal(w, _basis_word_rows(rows, 5))
    again = _basis_word_rows(w, 5)
    assert type(again) is np.ndarray and np.array_equal(again, w)
    bits4 = np.array([[1, 0, 1, 1]] * 5, dtype=np.uint64)
    assert [int(x) for x in _basis_word_rows(bits4, 5)[0]] == [0b1101, 0, 0, 0]
    import pytest
    with pytest.raises(ValueError):
        _basis_word_rows(w, 6)


def test_sanitized_build_keeps_sanitizers_on_the_host():
    """The UBSan build's flags put every sanitizer option behind -Xarch_host
    (device code is never sanitized), make reports fatal, and link the
    shared runtime with a run path to it."""
    from paper_1712_03554_amd import build as lib_build
    fl = lib_build.UBSAN_FLAGS
    for i, f in enumerate(fl):
        if f.startswith("-fsanitize") or f.startswith("-fno-sanitize"):
            assert i > 0 and fl[i - 1] == "-Xarch_host", f
    assert "-fsanitize=undefined" in fl and "-fno-sanitize-recover=undefined" in fl
    assert "-shared-libsan" in fl and any(f.startswith("-Wl,-rpath,") for f in fl)
    assert lib_build.UBSAN_OUT != lib_build.OUT


def test_library_path_override():
    """SFRAME_LIB selects the library file the binding loads (checked in a
    child process, so this one keeps its binding as it is)."""
    import subprocess
    import sys
    code = ("import paper_1712_03554_amd as sf\n"
            "print(sf.LIB_PATH)\n"
            "try:\n    sf.load_library()\nexcept ImportError:\n    print('ImportError')\n")
    env = dict(os.environ, SFRAME_LIB="/nonexistent/libsframe_other.so")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-1000:]
    assert r.stdout.split() == ["/nonexistent/libsframe_other.so", "ImportError"]
    env.pop("SFRAME_LIB")
    r = subprocess.run([sys.executable, "-c", "import paper_1712_03554_amd as sf; print(sf.LIB_PATH)"], cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=120)
    assert r.stdout.strip() == os.path.join(ROOT, "paper_1712_03554_amd", "libsframe.so")


def test_every_declaration_names_its_passage():
    """Each exported call's comment (its own, or the one it shares with the
    calls declared right after it) names the passage of the paper it follows
    (section, definition, equation, example, table, figure, theorem,
    observation, invariant), or says it is not in the paper, or (the
    allocation-free entry point) names the callers it is for."""
    text = open(HEADER).read()
    cite = re.compile(r"sections? \d|definition \d|eqs?\. ?\d|example \d|table \d|figure \d|theorem \d|"
                      r"observation \d|invariant \d|not in the paper|cannot allocate", re.I)
    prev, last, seen = 0, "", []
    for m in re.finditer(r"^(?:sf_status|const char\*)\s+(sf_\w+)\(", text, re.M):
        comments = re.findall(r"/\*.*?\*/", text[prev:m.start()], re.S)
        last = comments[-1] if comments else last
        assert cite.search(last), f"{m.group(1)}: no passage named"
        seen.append(m.group(1))
        prev = m.end()
    assert sorted(seen) == _declared()


def test_header_is_plain_c_and_links(tmp_path):
    """A C99 (pedantic) and a C++ program that include the header and take
    the address of every declared call compile warning-free, and the C one links against
    the built library (every declaration has its definition)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None or shutil.which("g++") is None:
        pytest.skip("no gcc")
    names = _declared()
    body = "#include \"sframe.h\"\n#include <stdio.h>\ntypedef void (*fn_t)(void);\nint main(void) {\n"
    body += "  fn_t fns[] = {\n" + "".join(f"    (fn_t)&{n},\n" for n in names)
    body += "  };\n  printf(\"%d\\n\", (int)(sizeof fns / sizeof fns[0]));\n  return 0;\n}\n"
    src = tmp_path / "use.c"
    src.write_text(body)
    inc = os.path.join(ROOT, "include")
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                        "-I", inc, "-c", str(src), "-o", str(tmp_path / "use.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    srcpp = tmp_path / "use.cpp"
    srcpp.write_text(body.replace("(fn_t)&", "(fn_t)&::"))
    r = subprocess.run(["g++", "-std=c++11", "-Wall", "-Wextra", "-Werror", "-I", inc, "-c", str(srcpp),
                        "-o", str(tmp_path / "usepp.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    if not os.path.exists(sf.LIB_PATH):
        pytest.skip("library not built")
    libdir = os.path.dirname(sf.LIB_PATH)
    r = subprocess.run(["gcc", str(tmp_path / "use.o"), "-o", str(tmp_path / "use"), sf.LIB_PATH,
                        "-Wl,--unresolved-symbols=ignore-in-shared-libs", "-Wl,-rpath," + libdir],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
