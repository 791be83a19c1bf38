"""ctypes wrapper of the C frame oracle (oracle/frame.c) -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the bench's CPU-baseline leg may import this.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "frame.c")
_LIB = os.path.join(_HERE, "_oracle_frame.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile frame.c with gcc (plain -O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.ofr_new.restype = ctypes.c_void_p
        L.ofr_new.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64]
        L.ofr_free.argtypes = [ctypes.c_void_p]
        L.ofr_apply.restype = ctypes.c_int
        L.ofr_apply.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, ctypes.c_int64, ctypes.c_int64]
        L.ofr_size.restype = ctypes.c_size_t
        L.ofr_size.argtypes = [ctypes.c_void_p]
        L.ofr_xblock.restype = ctypes.c_int
        L.ofr_xblock.argtypes = [ctypes.c_void_p]
        L.ofr_fragile.restype = ctypes.c_int
        L.ofr_fragile.argtypes = [ctypes.c_void_p]
        L.ofr_outcomes.restype = ctypes.c_size_t
        L.ofr_outcomes.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
        L.ofr_read.restype = ctypes.c_size_t
        L.ofr_read.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_size_t]
        L.ofr_run.restype = ctypes.c_int
        L.ofr_run.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 4 + [ctypes.c_size_t, ctypes.c_void_p]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class OracleFrame:
    """One single-frame simulation on the CPU."""

    def __init__(self, n: int, init_bits=None, seed: int = 0):
        L = _load()
        self.n = n
        self.W = (n + 63) // 64
        bits = np.zeros(n, dtype=np.uint8) if init_bits is None else np.asarray(init_bits, dtype=np.uint8)
        self._h = L.ofr_new(n, _ptr(bits), ctypes.c_uint64(seed & ((1 << 64) - 1)))
        if not self._h:
            raise ValueError("oracle: bad qubit count")

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ofr_free(self._h)
            self._h = None

    def apply(self, op, q0=0, q1=0, q2=0, num=0, den=1) -> int:
        r = _lib.ofr_apply(self._h, int(op), int(q0), int(q1), int(q2), int(num), int(den))
        if r < 0:
            raise ValueError("oracle: invalid gate")
        return r

    def run(self, gates) -> np.ndarray:
        """Apply a gate array (workloads.GATE_DTYPE); returns |F| before each gate."""
        g = np.asarray(gates)
        ops = np.ascontiguousarray(g["op"], dtype=np.int32)
        q = np.ascontiguousarray(np.stack([g["q0"], g["q1"], g["q2"]], axis=1), dtype=np.int32)
        num = np.ascontiguousarray(g["num"], dtype=np.int64)
        den = np.ascontiguousarray(g["den"], dtype=np.int64)
        sizes = np.zeros(len(g), dtype=np.uint64)
        if _lib.ofr_run(self._h, _ptr(ops), _ptr(q), _ptr(num), _ptr(den), len(g), _ptr(sizes)) < 0:
            raise ValueError("oracle: invalid gate")
        return sizes

    @property
    def size(self) -> int:
        return int(_lib.ofr_size(self._h))

    @property
    def xblock(self) -> int:
        return int(_lib.ofr_xblock(self._h))

    @property
    def fragile(self) -> bool:
        return bool(_lib.ofr_fragile(self._h))

    def outcomes(self) -> list[int]:
        m = _lib.ofr_outcomes(self._h, None, 0)
        out = np.zeros(max(m, 1), dtype=np.uint8)
        _lib.ofr_outcomes(self._h, _ptr(out), m)
        return out[:m].tolist()

    def read(self):
        """(tableau[n, 2W] uint64, sigma[K, W] uint64, amp[K] complex128), canonical order."""
        K = self.size
        tab = np.zeros((self.n, 2 * self.W), dtype=np.uint64)
        sig = np.zeros((max(K, 1), self.W), dtype=np.uint64)
        amp = np.zeros(2 * max(K, 1), dtype=np.float64)
        _lib.ofr_read(self._h, _ptr(tab), _ptr(sig), _ptr(amp), K)
        return tab, sig[:K], (amp[0::2] + 1j * amp[1::2])[:K]


def _load_mf():
    L = _load()
    if getattr(L, "_mf_ready", False):
        return L
    L.omf_new.restype = ctypes.c_void_p
    L.omf_new.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64]
    L.omf_load.restype = ctypes.c_void_p
    L.omf_load.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                           ctypes.c_uint64]
    L.omf_free.argtypes = [ctypes.c_void_p]
    L.omf_apply.restype = ctypes.c_int
    L.omf_apply.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                            ctypes.c_int64, ctypes.c_int64]
    L.omf_run.restype = ctypes.c_int
    L.omf_run.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 4 + [ctypes.c_size_t, ctypes.c_void_p,
                                                                     ctypes.c_void_p]
    for name in ("omf_nframes", "omf_ortho_runs", "omf_coalesce"):
        getattr(L, name).restype = ctypes.c_size_t
        getattr(L, name).argtypes = [ctypes.c_void_p]
    L.omf_frame_size.restype = ctypes.c_size_t
    L.omf_frame_size.argtypes = [ctypes.c_void_p, ctypes.c_size_t]
    L.omf_read.restype = ctypes.c_size_t
    L.omf_read.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_size_t]
    for name in ("omf_fragile", "omf_orthogonal", "omf_orthogonalize"):
        getattr(L, name).restype = ctypes.c_int
        getattr(L, name).argtypes = [ctypes.c_void_p]
    L.omf_add_frame.restype = ctypes.c_int
    L.omf_add_frame.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
    L.omf_set_general.restype = None
    L.omf_set_general.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.omf_outcomes.restype = ctypes.c_size_t
    L.omf_outcomes.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
    L._mf_ready = True
    return L


class OracleMultiframe:
    """A multiframe simulation on the CPU (list of frames, section 4)."""

    def __init__(self, n: int, init_bits=None, seed: int = 0, _handle=None):
        L = _load_mf()
        self.n = n
        self.W = (n + 63) // 64
        if _handle is not None:
            self._h = _handle
        else:
            bits = np.zeros(n, dtype=np.uint8) if init_bits is None else np.asarray(init_bits, dtype=np.uint8)
            self._h = L.omf_new(n, _ptr(bits), ctypes.c_uint64(seed & ((1 << 64) - 1)))
        if not self._h:
            raise ValueError("oracle: bad qubit count")

    @classmethod
    def load(cls, n, tableau, sigma, amp, seed: int = 0):
        """One explicit frame: canonical tableau [n, 2W], sigma [K, W], amp [K] complex."""
        L = _load_mf()
        tab = np.ascontiguousarray(tableau, dtype=np.uint64)
        sig = np.ascontiguousarray(sigma, dtype=np.uint64)
        a = np.ascontiguousarray(np.stack([np.real(amp), np.imag(amp)], axis=1).reshape(-1), dtype=np.float64)
        h = L.omf_load(n, _ptr(tab), _ptr(sig), _ptr(a), len(sig), ctypes.c_uint64(seed))
        return cls(n, _handle=h)

    def add_frame(self, tableau, sigma, amp):
        """Append one explicit frame (frames with equal matrices merge)."""
        tab = np.ascontiguousarray(tableau, dtype=np.uint64)
        sig = np.ascontiguousarray(sigma, dtype=np.uint64)
        a = np.ascontiguousarray(np.stack([np.real(amp), np.imag(amp)], axis=1).reshape(-1), dtype=np.float64)
        _lib.omf_add_frame(self._h, _ptr(tab), _ptr(sig), _ptr(a), len(sig))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.omf_free(self._h)
            self._h = None

    def apply(self, op, q0=0, q1=0, q2=0, num=0, den=1) -> int:
        r = _lib.omf_apply(self._h, int(op), int(q0), int(q1), int(q2), int(num), int(den))
        if r < 0:
            raise ValueError("oracle: invalid gate")
        return r

    def run(self, gates):
        """Apply a gate array; returns (total elements, frames) before each gate."""
        g = np.asarray(gates)
        ops = np.ascontiguousarray(g["op"], dtype=np.int32)
        q = np.ascontiguousarray(np.stack([g["q0"], g["q1"], g["q2"]], axis=1), dtype=np.int32)
        num = np.ascontiguousarray(g["num"], dtype=np.int64)
        den = np.ascontiguousarray(g["den"], dtype=np.int64)
        sizes = np.zeros(len(g), dtype=np.uint64)
        nfr = np.zeros(len(g), dtype=np.uint64)
        if _lib.omf_run(self._h, _ptr(ops), _ptr(q), _ptr(num), _ptr(den), len(g), _ptr(sizes), _ptr(nfr)) < 0:
            raise ValueError("oracle: invalid gate")
        return sizes, nfr

    @property
    def nframes(self) -> int:
        return int(_lib.omf_nframes(self._h))

    @property
    def size(self) -> int:
        return sum(int(_lib.omf_frame_size(self._h, i)) for i in range(self.nframes))

    @property
    def fragile(self) -> bool:
        return bool(_lib.omf_fragile(self._h))

    def orthogonal(self) -> bool:
        return bool(_lib.omf_orthogonal(self._h))

    def orthogonalize(self) -> bool:
        return bool(_lib.omf_orthogonalize(self._h))

    def set_general(self, general: bool = True):
        """Coalesce through the basis circuit (the extension of COALESCE to
        matrices without Z_k rows) instead of the matrix's own Z_k rows."""
        _lib.omf_set_general(self._h, 1 if general else 0)

    def coalesce(self) -> int:
        return int(_lib.omf_coalesce(self._h))

    @property
    def ortho_runs(self) -> int:
        return int(_lib.omf_ortho_runs(self._h))

    def outcomes(self) -> list[int]:
        m = _lib.omf_outcomes(self._h, None, 0)
        out = np.zeros(max(m, 1), dtype=np.uint8)
        _lib.omf_outcomes(self._h, _ptr(out), m)
        return out[:m].tolist()

    def frames(self):
        """[(tableau, sigma, amp)] per frame, frames sorted by matrix."""
        res = []
        for i in range(self.nframes):
            K = int(_lib.omf_frame_size(self._h, i))
            tab = np.zeros((self.n, 2 * self.W), dtype=np.uint64)
            sig = np.zeros((max(K, 1), self.W), dtype=np.uint64)
            amp = np.zeros(2 * max(K, 1), dtype=np.float64)
            _lib.omf_read(self._h, i, _ptr(tab), _ptr(sig), _ptr(amp), K)
            res.append((tab, sig[:K], (amp[0::2] + 1j * amp[1::2])[:K]))
        return res
