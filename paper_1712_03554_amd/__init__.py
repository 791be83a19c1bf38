"""Python binding of libsframe.so (stabilizer-frame simulation on MI355X).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of the library.  Device memory comes from PyTorch's caching allocator
through the library's allocator hook, and work is queued on PyTorch's current
HIP stream.  Importing works without a GPU; creating an Engine needs the built
library and a HIP device and raises otherwise.
"""
from __future__ import annotations

import atexit
import ctypes
import os

import numpy as np

from . import workloads
from .workloads import GATE_DTYPE

_HERE = os.path.dirname(os.path.abspath(__file__))
# SFRAME_LIB names another build of the library (the host-sanitized one)
LIB_PATH = os.environ.get("SFRAME_LIB") or os.path.join(_HERE, "libsframe.so")

SF_OK, SF_E_INVALID, SF_E_OOM, SF_E_DEVICE, SF_E_TOO_LARGE, SF_E_STATE, SF_E_BUFSIZE, SF_E_CANCELLED = range(8)
STATUS_NAMES = ["SF_OK", "SF_E_INVALID", "SF_E_OOM", "SF_E_DEVICE", "SF_E_TOO_LARGE", "SF_E_STATE",
                "SF_E_BUFSIZE", "SF_E_CANCELLED"]

EXPORTS = ["sf_ctx_create", "sf_ctx_destroy", "sf_last_error", "sf_measure", "sf_batch_graph", "sf_autotune",
           "sf_tuning_get", "sf_tuning_set", "sf_batch_reset",
           "sf_graph_set_input", "sf_graph_launch", "sf_graph_destroy", "sf_circuit_load", "sf_circuit_info",
           "sf_circuit_destroy", "sf_state_init", "sf_state_destroy", "sf_step", "sf_run", "sf_sync",
           "sf_outcomes", "sf_frame_size", "sf_read_frame", "sf_state_info", "sf_state_reset",
           "sf_state_dim", "sf_profile", "sf_profile_read", "sf_state_cycles", "sf_batch_run", "sf_batch_run_noalloc",
           "sf_serve_create", "sf_serve_submit", "sf_serve_tick", "sf_serve_poll", "sf_serve_release",
           "sf_serve_cancel", "sf_serve_stats", "sf_serve_destroy"]

KERNEL_KINDS = ["track", "segment", "meas_reduce", "meas_coin", "meas_filter", "readout", "init", "phase", "fit",
                "wide"]


class SFrameError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 8 else status}: {msg}")
        self.status = status


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsframe.so; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libsframe.so not built ({path}); build it with paper_1712_03554_amd/build.py")
    L = ctypes.CDLL(path)
    vp, u64, sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "sf_ctx_create": [ctypes.c_int, vp, vp, u64, P(vp)],
        "sf_ctx_destroy": [vp],
        "sf_circuit_load": [vp, ctypes.c_uint32, vp, sz, P(vp)],
        "sf_circuit_info": [vp, P(u64), P(u64)],
        "sf_circuit_destroy": [vp],
        "sf_state_init": [vp, vp, vp, u64, P(vp)],
        "sf_state_destroy": [vp],
        "sf_step": [vp, sz, P(sz)],
        "sf_run": [vp],
        "sf_measure": [vp, ctypes.c_uint32, P(ctypes.c_int)],
        "sf_batch_graph": [vp, vp, sz, vp, vp, P(vp)],
        "sf_graph_set_input": [vp, sz, vp, u64],
        "sf_graph_launch": [vp],
        "sf_graph_destroy": [vp],
        "sf_autotune": [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp],
        "sf_tuning_get": [vp, vp, vp, P(ctypes.c_int)],
        "sf_tuning_set": [vp, vp, vp, ctypes.c_int],
        "sf_batch_reset": [vp, vp, sz, vp, vp],
        "sf_sync": [vp],
        "sf_outcomes": [vp, vp, sz, P(sz)],
        "sf_frame_size": [vp, P(u64)],
        "sf_read_frame": [vp, vp, vp, vp, sz, P(sz)],
        "sf_state_info": [vp, P(sz), P(ctypes.c_int)],
        "sf_state_reset": [vp, vp, u64],
        "sf_state_dim": [vp, P(ctypes.c_uint32)],
        "sf_profile": [vp, ctypes.c_int],
        "sf_profile_read": [vp, vp, vp, ctypes.c_int],
        "sf_state_cycles": [vp, vp, ctypes.c_int],
        "sf_batch_run": [vp, vp, sz],
        "sf_batch_run_noalloc": [vp, vp, sz],
        "sf_serve_create": [vp, u64, ctypes.c_uint32, ctypes.c_uint32, P(vp)],
        "sf_serve_submit": [vp, vp, vp, u64, P(u64)],
        "sf_serve_tick": [vp, P(ctypes.c_uint32), P(ctypes.c_uint32)],
        "sf_serve_poll": [vp, u64, P(ctypes.c_int), P(vp)],
        "sf_serve_release": [vp, u64],
        "sf_serve_cancel": [vp, u64],
        "sf_serve_stats": [vp, P(u64), P(u64), P(u64), P(u64)],
        "sf_serve_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.sf_last_error.argtypes = [vp]
    L.sf_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


_exiting = False


def _mark_exit():
    # At interpreter exit objects are finalised in no particular order (an
    # Engine may go before its states) and torch's allocator may already be
    # gone; the process is ending, so the library is not called any more.
    global _exiting
    _exiting = True


atexit.register(_mark_exit)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class Engine:
    """A library context bound to one HIP device and stream."""

    def __init__(self, device: int = 0, stream=None, budget_bytes: int = 0, torch_allocator: bool = True,
                 refuse=None):
        """refuse: optional predicate on a request's byte count; requests it
        accepts are answered with NULL (device allocation failure), as an
        allocator that has run out would."""
        self._L = load_library()
        self._keep = []
        self.device = device
        stream_ptr = None
        alloc_ptr = None
        try:
            import torch
        except ImportError:  # pragma: no cover
            torch = None
        if torch is not None and torch.cuda.is_available():
            torch.cuda.set_device(device)
            s = stream if stream is not None else torch.cuda.current_stream(device)
            stream_ptr = ctypes.c_void_p(s.cuda_stream)
            self._torch_stream = s
            if torch_allocator:
                dev = device

                def _alloc(nbytes, stream, user):
                    if refuse is not None and refuse(int(nbytes)):
                        return None
                    try:
                        return torch.cuda.caching_allocator_alloc(int(nbytes), dev, s)
                    except Exception:
                        return None

                def _free(ptr, nbytes, stream, user):
                    try:
                        torch.cuda.caching_allocator_delete(ptr)
                    except Exception:
                        pass

                self._alloc_struct = _Allocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
                alloc_ptr = ctypes.cast(ctypes.pointer(self._alloc_struct), ctypes.c_void_p)
        h = ctypes.c_void_p()
        st = self._L.sf_ctx_create(device, stream_ptr, alloc_ptr, budget_bytes, ctypes.byref(h))
        if st != SF_OK:
            raise SFrameError(st, "sf_ctx_create failed (no HIP device?)")
        self._h = h

    def _check(self, st):
        if st != SF_OK:
            raise SFrameError(st, self._L.sf_last_error(self._h).decode())

    def load(self, n: int, gates) -> "Circuit":
        arr = gates.array() if hasattr(gates, "array") else np.ascontiguousarray(gates, dtype=GATE_DTYPE)
        arr = np.ascontiguousarray(arr, dtype=GATE_DTYPE)
        h = ctypes.c_void_p()
        self._check(self._L.sf_circuit_load(self._h, n, _ptr(arr), len(arr), ctypes.byref(h)))
        return Circuit(self, h, n)

    def batch_run(self, states):
        """Run every remaining gate of the given states as one batch
        (synchronises).  states: a list of State or a StateBatch."""
        sb = states if isinstance(states, StateBatch) else StateBatch(states)
        self._check(self._L.sf_batch_run(self._h, sb.handles(), len(sb)))

    def batch_run_noalloc(self, states):
        """As batch_run, allocating no device memory (sf_batch_run_noalloc)."""
        sb = states if isinstance(states, StateBatch) else StateBatch(states)
        self._check(self._L.sf_batch_run_noalloc(self._h, sb.handles(), len(sb)))

    def batch_reset(self, states, bases=None, seeds=None):
        """Re-initialise the states with one launch.  states: a list of State
        or a StateBatch; bases: basis bit lists, an array of shape
        (states, qubits) of 0/1, or the words of pack_bases; seeds: integers
        (or a uint64 array)."""
        sb = states if isinstance(states, StateBatch) else StateBatch(states)
        ns = len(sb)
        b = None if bases is None else _basis_word_rows(bases, ns)
        sd = None
        if seeds is not None:
            sd = np.asarray(seeds, dtype=np.uint64) if isinstance(seeds, np.ndarray) else \
                np.array([int(x) & ((1 << 64) - 1) for x in seeds] or [0], dtype=np.uint64)
        self._check(self._L.sf_batch_reset(self._h, sb.handles(), ns, _ptr(b), _ptr(sd)))

    def batch_graph(self, states, bases=None, seeds=None) -> "Graph":
        """Record a whole batched run of these states (see sf_batch_graph)."""
        return Graph(self, states, bases, seeds)

    TUNE_DIMS = 31

    def tuning(self) -> dict:
        """The context's launch tuning: {"blocks": [...], "grids": [...] (per
        hull dimension d = 0..30), "phase_waves": int}."""
        b = np.zeros(self.TUNE_DIMS, dtype=np.int32)
        g = np.zeros(self.TUNE_DIMS, dtype=np.int32)
        pw = ctypes.c_int()
        self._check(self._L.sf_tuning_get(self._h, _ptr(b), _ptr(g), ctypes.byref(pw)))
        return {"blocks": b.tolist(), "grids": g.tolist(), "phase_waves": int(pw.value)}

    def set_tuning(self, tun: dict):
        """Install a tuning as returned by tuning() (shapes optional)."""
        pw = int(tun.get("phase_waves", self.tuning()["phase_waves"]))
        if tun.get("blocks") is None:
            self._check(self._L.sf_tuning_set(self._h, None, None, pw))
            return
        b = np.ascontiguousarray(tun["blocks"], dtype=np.int32)
        g = np.ascontiguousarray(tun["grids"], dtype=np.int32)
        if b.shape != (self.TUNE_DIMS,) or g.shape != (self.TUNE_DIMS,):
            raise ValueError(f"tuning tables need {self.TUNE_DIMS} entries")
        self._check(self._L.sf_tuning_set(self._h, _ptr(b), _ptr(g), pw))

    def _device_tag(self) -> str:
        import torch
        p = torch.cuda.get_device_properties(self.device)
        return f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}"

    def save_tuning(self, path: str):
        """Write the tuning with the device it was made on (JSON)."""
        import json
        rec = dict(self.tuning(), device=self._device_tag())
        with open(path, "w") as fh:
            json.dump(rec, fh)

    def load_tuning(self, path: str) -> bool:
        """Install a saved tuning if it was made on this kind of device;
        returns whether it was installed."""
        import json
        try:
            with open(path) as fh:
                rec = json.load(fh)
        except (OSError, ValueError):
            return False
        if rec.get("device") != self._device_tag():
            return False
        self.set_tuning(rec)
        return True

    def autotune(self, d_lo: int = 12, d_hi: int = 24, cache: str = None) -> dict:
        """Pick launch shapes of the elementwise frame kernels; {d: (block, grid, ms)}.
        With cache: a tuning saved there for this kind of device is installed
        instead (the result then holds (block, grid, None)); otherwise the
        tuner runs and its result is saved there."""
        if cache and self.load_tuning(cache):
            t = self.tuning()
            return {d: (t["blocks"][d], t["grids"][d], None) for d in range(d_lo, d_hi + 1)}
        k = d_hi - d_lo + 1
        b = np.zeros(k, dtype=np.int32)
        g = np.zeros(k, dtype=np.int32)
        t = np.zeros(k, dtype=np.float32)
        self._check(self._L.sf_autotune(self._h, d_lo, d_hi, _ptr(b), _ptr(g), _ptr(t)))
        if cache:
            self.save_tuning(cache)
        return {d_lo + i: (int(b[i]), int(g[i]), float(t[i])) for i in range(k)}

    def profile(self, enable: bool, kinds=None):
        """Start (clearing the totals) or stop per-kernel timing; kinds limits
        it to the named kernel kinds (KERNEL_KINDS)."""
        mask = 0 if not enable else (-1 if kinds is None else sum(1 << KERNEL_KINDS.index(k) for k in kinds))
        self._check(self._L.sf_profile(self._h, mask))

    def profile_read(self) -> dict:
        k = len(KERNEL_KINDS)
        ms = np.zeros(k, dtype=np.float64)
        cnt = np.zeros(k, dtype=np.uint64)
        self._check(self._L.sf_profile_read(self._h, _ptr(ms), _ptr(cnt), k))
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(KERNEL_KINDS)}

    def close(self):
        if getattr(self, "_h", None) and not _exiting:
            self._L.sf_ctx_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()


class Circuit:
    def __init__(self, eng: Engine, h, n: int):
        self.eng, self._h, self.n = eng, h, n

    def info(self):
        b, p = ctypes.c_uint64(), ctypes.c_uint64()
        self.eng._check(self.eng._L.sf_circuit_info(self._h, ctypes.byref(b), ctypes.byref(p)))
        return int(b.value), int(p.value)

    def state(self, basis_bits=None, seed: int = 0) -> "State":
        W = (self.n + 63) // 64
        words = None
        if basis_bits is not None:
            words = np.zeros(W, dtype=np.uint64)
            for q, b in enumerate(basis_bits):
                if int(b) & 1:
                    words[q >> 6] |= np.uint64(1 << (q & 63))
        h = ctypes.c_void_p()
        self.eng._check(self.eng._L.sf_state_init(self.eng._h, self._h, _ptr(words),
                                                  ctypes.c_uint64(seed & ((1 << 64) - 1)), ctypes.byref(h)))
        return State(self, h)

    def close(self):
        if getattr(self, "_h", None) and self.eng._h and not _exiting:
            self.eng._L.sf_circuit_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()


class State:
    def __init__(self, circ: Circuit, h, owned: bool = True):
        self.circ, self._h, self._owned = circ, h, owned
        self.n = circ.n
        self.W = (circ.n + 63) // 64
        self._L = circ.eng._L

    def _check(self, st):
        self.circ.eng._check(st)

    def reset(self, basis_bits=None, seed: int = 0):
        words = None
        if basis_bits is not None:
            words = np.zeros(self.W, dtype=np.uint64)
            for q, b in enumerate(basis_bits):
                if int(b) & 1:
                    words[q >> 6] |= np.uint64(1 << (q & 63))
        self._check(self._L.sf_state_reset(self._h, _ptr(words), ctypes.c_uint64(seed & ((1 << 64) - 1))))

    TRACK_PHASES = ["save", "columns", "repair", "index", "sampling", "fit", "cofactor", "total",
                    "repair_check", "repair_rowmul", "repair_replay", "repair_passes",
                    "index_pivots", "index_beta", "index_images", "sampling_points"]

    def track_cycles(self) -> dict:
        c = np.zeros(16, dtype=np.uint64)
        self._check(self._L.sf_state_cycles(self._h, _ptr(c), 16))
        return {k: int(c[i]) for i, k in enumerate(self.TRACK_PHASES)}

    def dim(self) -> int:
        d = ctypes.c_uint32()
        self._check(self._L.sf_state_dim(self._h, ctypes.byref(d)))
        return int(d.value)

    def step(self, max_gates: int) -> int:
        k = ctypes.c_size_t()
        self._check(self._L.sf_step(self._h, max_gates, ctypes.byref(k)))
        return int(k.value)

    def run(self):
        self._check(self._L.sf_run(self._h))

    def measure(self, qubit: int) -> int:
        """Measure a qubit now (between circuit gates); returns the outcome."""
        o = ctypes.c_int()
        self._check(self._L.sf_measure(self._h, qubit, ctypes.byref(o)))
        return int(o.value)

    def sync(self):
        self._check(self._L.sf_sync(self._h))

    def outcomes(self) -> list[int]:
        cnt = ctypes.c_size_t()
        self._check(self._L.sf_outcomes(self._h, None, 0, ctypes.byref(cnt)))
        out = np.zeros(max(1, cnt.value), dtype=np.uint8)
        self._check(self._L.sf_outcomes(self._h, _ptr(out), cnt.value, ctypes.byref(cnt)))
        return out[: cnt.value].tolist()

    def frame_size(self) -> int:
        k = ctypes.c_uint64()
        self._check(self._L.sf_frame_size(self._h, ctypes.byref(k)))
        return int(k.value)

    def info(self):
        done, frag = ctypes.c_size_t(), ctypes.c_int()
        self._check(self._L.sf_state_info(self._h, ctypes.byref(done), ctypes.byref(frag)))
        return int(done.value), bool(frag.value)

    def read_frame(self):
        """(tableau[n, 2W] uint64, sigma[K, W] uint64, amp[K] complex128), canonical order."""
        K = ctypes.c_size_t()
        tab = np.zeros((self.n, 2 * self.W), dtype=np.uint64)
        st = self._L.sf_read_frame(self._h, None, None, None, 0, ctypes.byref(K))
        if st not in (SF_OK, SF_E_BUFSIZE):
            self._check(st)
        k = K.value
        sig = np.zeros((max(k, 1), self.W), dtype=np.uint64)
        amp = np.zeros(2 * max(k, 1), dtype=np.float64)
        self._check(self._L.sf_read_frame(self._h, _ptr(tab), _ptr(sig), _ptr(amp), k, ctypes.byref(K)))
        return tab, sig[:k], (amp[0::2] + 1j * amp[1::2])[:k]

    def close(self):
        if getattr(self, "_h", None) and getattr(self, "_owned", True) and self.circ.eng._h and not _exiting:
            self._L.sf_state_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()


class Server:
    """Continuous-batching request loop over one Engine (see sf_serve_* in sframe.h)."""

    QUEUED, RESIDENT, DONE, CANCELLED, FAILED = range(5)

    def __init__(self, eng: Engine, budget_bytes: int = 0, max_resident: int = 64, tick_segments: int = 0):
        self.eng = eng
        self._L = eng._L
        h = ctypes.c_void_p()
        eng._check(self._L.sf_serve_create(eng._h, budget_bytes, max_resident, tick_segments, ctypes.byref(h)))
        self._h = h
        self._circuits = {}

    def submit(self, circ: Circuit, basis_bits=None, seed: int = 0) -> int:
        words = None
        if basis_bits is not None:
            words = np.zeros((circ.n + 63) // 64, dtype=np.uint64)
            for q, b in enumerate(basis_bits):
                if int(b) & 1:
                    words[q >> 6] |= np.uint64(1 << (q & 63))
        jid = ctypes.c_uint64()
        self.eng._check(self._L.sf_serve_submit(self._h, circ._h, _ptr(words),
                                                ctypes.c_uint64(seed & ((1 << 64) - 1)), ctypes.byref(jid)))
        self._circuits[int(jid.value)] = circ
        return int(jid.value)

    def tick(self):
        r, q = ctypes.c_uint32(), ctypes.c_uint32()
        self.eng._check(self._L.sf_serve_tick(self._h, ctypes.byref(r), ctypes.byref(q)))
        return int(r.value), int(q.value)

    def poll(self, job_id: int):
        """(status, State or None); the State belongs to the server."""
        stt, sh = ctypes.c_int(), ctypes.c_void_p()
        self.eng._check(self._L.sf_serve_poll(self._h, job_id, ctypes.byref(stt), ctypes.byref(sh)))
        st = None
        if stt.value == self.DONE and sh.value:
            st = State(self._circuits[job_id], sh, owned=False)
        return int(stt.value), st

    def release(self, job_id: int):
        self.eng._check(self._L.sf_serve_release(self._h, job_id))
        self._circuits.pop(job_id, None)

    def cancel(self, job_id: int):
        self.eng._check(self._L.sf_serve_cancel(self._h, job_id))

    def stats(self):
        v = [ctypes.c_uint64() for _ in range(4)]
        self.eng._check(self._L.sf_serve_stats(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(["ticks", "admitted", "rejected", "used_bytes"], [int(x.value) for x in v]))

    def close(self):
        if getattr(self, "_h", None) and self.eng._h and not _exiting:
            self._L.sf_serve_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()


class StateBatch:
    """A fixed list of states with their handle array built once (for
    repeated batched runs of many states)."""

    def __init__(self, states):
        self.states = list(states)
        self._arr = (ctypes.c_void_p * max(1, len(self.states)))(*[s._h.value for s in self.states])

    def __len__(self):
        return len(self.states)

    def __iter__(self):
        return iter(self.states)

    def handles(self):
        return ctypes.cast(self._arr, ctypes.c_void_p)


class BasisWords(np.ndarray):
    """Basis bits packed as the batched calls' words (pack_bases)."""


def pack_bases(bases, ns: int = None) -> BasisWords:
    """Basis bits per state (lists, or an array of 0/1 of shape (states, n))
    as the batched calls' words: 4 little-endian 64-bit words per state
    (covering 256 qubits; those calls refuse wider states themselves).  The
    result can be passed as `bases` to batch_reset, which then uses it as is."""
    return _basis_word_rows(bases, len(bases) if ns is None else ns).view(BasisWords)


def _basis_word_rows(bases, ns: int) -> np.ndarray:
    """Basis bits per state (lists, an array of 0/1 of shape (states, n), or
    the words of pack_bases) as 4 little-endian 64-bit words per state."""
    if isinstance(bases, BasisWords):
        if bases.shape[0] < ns:
            raise ValueError(f"packed bases for {bases.shape[0]} states, {ns} given")
        return np.ascontiguousarray(bases.view(np.ndarray))
    bits = np.zeros((max(1, ns), 256), dtype=np.uint8)
    if isinstance(bases, np.ndarray):
        m = min(256, bases.shape[1])
        bits[:bases.shape[0], :m] = bases[:, :m].astype(np.uint8) & 1
    else:
        for i, row in enumerate(bases):
            if row is not None and len(row):
                r = np.asarray(row, dtype=np.uint8)[:256]
                bits[i, :len(r)] = r & 1
    return np.ascontiguousarray(np.packbits(bits, axis=1, bitorder="little").view(np.uint64))


def _basis_words(n: int, bits):
    words = np.zeros(4, dtype=np.uint64)
    if bits is not None:
        for q, b in enumerate(bits[:256]):
            if int(b) & 1:
                words[q >> 6] |= np.uint64(1 << (q & 63))
    return words


class Graph:
    """A recorded batched run; launch() replays it (asynchronously)."""

    def __init__(self, eng: Engine, states, bases=None, seeds=None):
        self.eng, self._L, self.states = eng, eng._L, list(states)
        ns = len(self.states)
        words = [_basis_words(s.n, None if bases is None else bases[i]) for i, s in enumerate(self.states)]
        self._words = words
        ptrs = (ctypes.c_void_p * max(1, ns))(*[w.ctypes.data for w in words])
        sd = np.array([0 if seeds is None else int(seeds[i]) & ((1 << 64) - 1) for i in range(ns)] or [0],
                      dtype=np.uint64)
        arr = (ctypes.c_void_p * max(1, ns))(*[s._h.value for s in self.states])
        h = ctypes.c_void_p()
        eng._check(self._L.sf_batch_graph(eng._h, ctypes.cast(arr, ctypes.c_void_p), ns,
                                          ctypes.cast(ptrs, ctypes.c_void_p), _ptr(sd), ctypes.byref(h)))
        self._h = h

    def set_input(self, i: int, basis_bits=None, seed: int = 0):
        w = _basis_words(self.states[i].n, basis_bits)
        self.eng._check(self._L.sf_graph_set_input(self._h, i, _ptr(w), ctypes.c_uint64(seed & ((1 << 64) - 1))))

    def launch(self):
        self.eng._check(self._L.sf_graph_launch(self._h))

    def close(self):
        if getattr(self, "_h", None) and self.eng._h and not _exiting:
            self._L.sf_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()


def simulate(eng: Engine, circ: "workloads.Circuit", seed: int = 0) -> State:
    """Load, initialise and run a whole circuit; returns the (synchronised) state."""
    c = eng.load(circ.n, circ)
    s = c.state(circ.init_bits, seed)
    s.run()
    s.sync()
    s._circ_ref = c
    return s
