"""ctypes binding of libgrover's C ABI (include/grover.h), with the same function names.

Argument marshalling only: every step of the simulation runs in the library's HIP kernels. PyTorch, when
used (the `Grover` class), only provides device memory for the state and the HIP stream.

The library is loaded after `import torch` so that both share one HIP runtime in the process. Loading fails
loudly when libgrover.so has not been built; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import sys
import threading
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgrover.so")

GROVER_OK = 0
GROVER_E_INVAL = -1
GROVER_E_NOMEM = -2
GROVER_E_HIP = -3
GROVER_E_COOP = -4
GROVER_E_UNSUPPORTED = -5
GROVER_E_PREDICATE = -6
GROVER_E_TIMEOUT = -7

GROVER_F64_REAL, GROVER_C64, GROVER_C128, GROVER_CBF16 = 0, 1, 2, 3
GROVER_ACC_F64, GROVER_ACC_F32, GROVER_ACC_F32_KAHAN = 0, 1, 2
GROVER_UPDATE_F64, GROVER_UPDATE_F32 = 0, 1
GROVER_ORACLE_LIST, GROVER_ORACLE_HASH = 0, 1
GROVER_FORM_AUTO, GROVER_FORM_FUSED, GROVER_FORM_RESIDENT, GROVER_FORM_TWO_PASS, GROVER_FORM_HELD = 0, 1, 2, 3, 4

DTYPES = {"f64": GROVER_F64_REAL, "c64": GROVER_C64, "c128": GROVER_C128, "cbf16": GROVER_CBF16}
ACCUMS = {"f64": GROVER_ACC_F64, "f32": GROVER_ACC_F32, "f32_kahan": GROVER_ACC_F32_KAHAN}
UPDATES = {"f64": GROVER_UPDATE_F64, "f32": GROVER_UPDATE_F32}
FORMS = {"auto": GROVER_FORM_AUTO, "fused": GROVER_FORM_FUSED, "resident": GROVER_FORM_RESIDENT,
         "two_pass": GROVER_FORM_TWO_PASS, "held": GROVER_FORM_HELD}
ELEM_BYTES = {GROVER_F64_REAL: 8, GROVER_C64: 8, GROVER_C128: 16, GROVER_CBF16: 4}
NUMPY_DTYPES = {GROVER_F64_REAL: np.float64, GROVER_C64: np.complex64, GROVER_C128: np.complex128}


def bf16_pairs_to_complex(raw: np.ndarray) -> np.ndarray:
    """Complex bfloat16 storage (uint16 re, im, re, im, ...) -> complex128 (exact)."""
    u = np.ascontiguousarray(raw, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
    f = u.view(np.float32).astype(np.float64)
    return f[0::2] + 1j * f[1::2]


def complex_to_bf16_pairs(psi: np.ndarray) -> np.ndarray:
    """complex -> complex bfloat16 storage, each part rounded once to nearest even: round to odd into
    binary32 (truncate, set the last bit when inexact), then to nearest even into bfloat16."""
    parts = np.empty(2 * psi.size, dtype=np.float64)
    parts[0::2] = np.real(psi)
    parts[1::2] = np.imag(psi)
    t = parts.astype(np.float32)
    away = np.abs(t.astype(np.float64)) > np.abs(parts)
    t[away] = np.nextafter(t[away], np.float32(0))
    u = t.view(np.uint32).copy()
    u[t.astype(np.float64) != parts] |= np.uint32(1)
    u = u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))
    return (u >> np.uint32(16)).astype(np.uint16)

# grover_query keys
Q_FORM, Q_GRID, Q_BLOCK, Q_ELEM_BYTES, Q_N, Q_M, Q_TIMEOUT, Q_PER_CU, Q_FUSED_TEMPORAL = range(9)


# grover_batch_query keys
(BQ_COUNT, BQ_GRID, BQ_SPLIT, BQ_TEAM, BQ_UPDATES, BQ_GRAPH, BQ_BYTES, BQ_N_TEAM, BQ_RESIDENT, BQ_PHASES,
 BQ_STREAMS) = range(11)


# grover_phase_query keys
PQ_BATCH, PQ_GRID, PQ_TEAM, PQ_EVERY, PQ_CHECKPOINTS, PQ_BYTES, PQ_FORM, PQ_HELD_TEAM_F, PQ_HELD_TEAM_A = range(9)
GROVER_PHASE_FORM_AUTO, GROVER_PHASE_FORM_STREAMED, GROVER_PHASE_FORM_HELD = 0, 1, 2


class GroverError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


class grover_config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32),
        ("dtype", ctypes.c_uint32),
        ("oracle_kind", ctypes.c_uint32),
        ("hash_bits", ctypes.c_uint32),
        ("marked", ctypes.POINTER(ctypes.c_uint64)),
        ("m", ctypes.c_uint64),
        ("hash_seed", ctypes.c_uint64),
        ("form", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("accum", ctypes.c_uint32),
        ("update", ctypes.c_uint32),
    ]


class grover_phase_config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32),
        ("batch", ctypes.c_uint32),
        ("iterations", ctypes.c_uint32),
        ("checkpoint_every", ctypes.c_uint32),
        ("marked", ctypes.POINTER(ctypes.c_uint64)),
        ("m", ctypes.c_uint64),
        ("dtype", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
    ]


class grover_batch_config(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_uint64),
        ("n", ctypes.POINTER(ctypes.c_uint32)),
        ("m", ctypes.POINTER(ctypes.c_uint64)),
        ("marked", ctypes.POINTER(ctypes.c_uint64)),
        ("iterations", ctypes.POINTER(ctypes.c_uint64)),
        ("dtype", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("update", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


EXPORTS = [
    "grover_init", "grover_reset", "grover_iterate", "grover_gate_iterate", "grover_apply_hadamard_all",
    "grover_sample", "grover_sample_u53", "grover_norm", "grover_read_state", "grover_write_state",
    "grover_state_device", "grover_marked", "grover_sync", "grover_query", "grover_optimal_iterations",
    "grover_destroy", "grover_status_str", "grover_last_error",
    "grover_gate_iterate_blocked", "grover_apply_hadamard_all_blocked", "grover_iterate_static",
    "grover_stream_probe",
    "grover_batch_init", "grover_batch_set_tiling", "grover_batch_tune", "grover_batch_capture",
    "grover_batch_run", "grover_batch_sync", "grover_batch_state", "grover_batch_read_state",
    "grover_batch_query", "grover_batch_destroy", "grover_batch_last_error",
    "grover_phase_init", "grover_phase_set_team", "grover_phase_set_form", "grover_phase_forward",
    "grover_phase_backward", "grover_phase_sync", "grover_phase_state", "grover_phase_read_state", "grover_phase_query",
    "grover_phase_destroy", "grover_phase_last_error",
]

_lock = threading.Lock()
_lib = None


def load(path: str = LIB_PATH):
    """Load libgrover.so (after torch, so the HIP runtime is shared) and declare its prototypes."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built: run `python -m paper_2005_04635_amd.build` "
                               "(the HIP library is required; there is no fallback)")
        try:
            import torch  # noqa: F401  (shares its HIP runtime with the library)
        except ImportError:
            pass
        lib = ctypes.CDLL(path)
        P, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        pu64 = ctypes.POINTER(ctypes.c_uint64)
        sig = {
            "grover_init": (i32, [ctypes.POINTER(P), ctypes.POINTER(grover_config), P, P, ctypes.c_size_t]),
            "grover_reset": (i32, [P]),
            "grover_iterate": (i32, [P, u64]),
            "grover_gate_iterate": (i32, [P, u64]),
            "grover_apply_hadamard_all": (i32, [P]),
            "grover_gate_iterate_blocked": (i32, [P, u64]),
            "grover_apply_hadamard_all_blocked": (i32, [P]),
            "grover_sample": (i32, [P, u64, u64, P, i32]),
            "grover_sample_u53": (i32, [P, P, i32, u64, P, i32]),
            "grover_norm": (i32, [P, ctypes.POINTER(ctypes.c_double)]),
            "grover_read_state": (i32, [P, P, ctypes.c_size_t]),
            "grover_write_state": (i32, [P, P, ctypes.c_size_t]),
            "grover_state_device": (i32, [P, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_size_t)]),
            "grover_marked": (i32, [P, pu64, u64, pu64]),
            "grover_sync": (i32, [P]),
            "grover_query": (i32, [P, i32, ctypes.POINTER(ctypes.c_int64)]),
            "grover_optimal_iterations": (u64, [u32, u64]),
            "grover_destroy": (None, [P]),
            "grover_iterate_static": (i32, [P, P, u32, u32, P, u64, u64, P]),
            "grover_stream_probe": (i32, [P, P, ctypes.c_size_t, u32, u32, ctypes.POINTER(ctypes.c_float)]),
            "grover_status_str": (ctypes.c_char_p, [i32]),
            "grover_last_error": (ctypes.c_char_p, [P]),
            "grover_batch_init": (i32, [ctypes.POINTER(P), ctypes.POINTER(grover_batch_config), P]),
            "grover_batch_set_tiling": (i32, [P, u32, u32, u32]),
            "grover_batch_tune": (i32, [P, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32),
                                        ctypes.POINTER(ctypes.c_float)]),
            "grover_batch_capture": (i32, [P]),
            "grover_batch_run": (i32, [P]),
            "grover_batch_sync": (i32, [P]),
            "grover_batch_state": (i32, [P, u64, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_size_t)]),
            "grover_batch_read_state": (i32, [P, u64, P, ctypes.c_size_t]),
            "grover_batch_query": (i32, [P, i32, ctypes.POINTER(ctypes.c_int64)]),
            "grover_batch_destroy": (None, [P]),
            "grover_batch_last_error": (ctypes.c_char_p, [P]),
            "grover_phase_init": (i32, [ctypes.POINTER(P), ctypes.POINTER(grover_phase_config), P]),
            "grover_phase_set_team": (i32, [P, u32]),
            "grover_phase_set_form": (i32, [P, u32]),
            "grover_phase_forward": (i32, [P, P, P, P]),
            "grover_phase_backward": (i32, [P, P, P, P]),
            "grover_phase_sync": (i32, [P]),
            "grover_phase_state": (i32, [P, u32, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_size_t)]),
            "grover_phase_read_state": (i32, [P, u32, P, ctypes.c_size_t]),
            "grover_phase_query": (i32, [P, i32, ctypes.POINTER(ctypes.c_int64)]),
            "grover_phase_destroy": (None, [P]),
            "grover_phase_last_error": (ctypes.c_char_p, [P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def _check(ctx, status: int) -> None:
    if status != GROVER_OK:
        lib = load()
        msg = lib.grover_last_error(ctx).decode()
        if not msg or msg == "no context":
            msg = lib.grover_status_str(status).decode()
        raise GroverError(status, msg)


# ------------------------------------------------------------------------- one wrapper per C function
def grover_init(cfg: grover_config, hip_stream: int = 0, state_dev: int = 0, state_bytes: int = 0):
    ctx = ctypes.c_void_p()
    st = load().grover_init(ctypes.byref(ctx), ctypes.byref(cfg), hip_stream or None, state_dev or None,
                            state_bytes)
    _check(None, st)
    return ctx


def grover_reset(ctx) -> None:
    _check(ctx, load().grover_reset(ctx))


def grover_iterate(ctx, k: int) -> None:
    _check(ctx, load().grover_iterate(ctx, k))


def grover_gate_iterate(ctx, k: int) -> None:
    _check(ctx, load().grover_gate_iterate(ctx, k))


def grover_apply_hadamard_all(ctx) -> None:
    _check(ctx, load().grover_apply_hadamard_all(ctx))


def grover_gate_iterate_blocked(ctx, k: int) -> None:
    _check(ctx, load().grover_gate_iterate_blocked(ctx, k))


def grover_apply_hadamard_all_blocked(ctx) -> None:
    _check(ctx, load().grover_apply_hadamard_all_blocked(ctx))


def grover_sample(ctx, shots: int, seed: int, out: int, out_is_device: bool) -> None:
    _check(ctx, load().grover_sample(ctx, shots, seed & (2**64 - 1), out or None, int(out_is_device)))


def grover_sample_u53(ctx, u53: int, u53_is_device: bool, shots: int, out: int, out_is_device: bool) -> None:
    _check(ctx, load().grover_sample_u53(ctx, u53 or None, int(u53_is_device), shots, out or None,
                                         int(out_is_device)))


def grover_norm(ctx) -> float:
    v = ctypes.c_double()
    _check(ctx, load().grover_norm(ctx, ctypes.byref(v)))
    return v.value


def grover_read_state(ctx, host: int, nbytes: int) -> None:
    _check(ctx, load().grover_read_state(ctx, host, nbytes))


def grover_write_state(ctx, host: int, nbytes: int) -> None:
    _check(ctx, load().grover_write_state(ctx, host, nbytes))


def grover_state_device(ctx):
    p, b = ctypes.c_void_p(), ctypes.c_size_t()
    _check(ctx, load().grover_state_device(ctx, ctypes.byref(p), ctypes.byref(b)))
    return p.value, b.value


def grover_marked(ctx, cap: int) -> np.ndarray:
    out = np.zeros(max(cap, 1), dtype=np.uint64)
    count = ctypes.c_uint64()
    _check(ctx, load().grover_marked(ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), cap,
                                     ctypes.byref(count)))
    return out[: min(cap, count.value)].copy()


def grover_sync(ctx) -> None:
    _check(ctx, load().grover_sync(ctx))


def grover_query(ctx, key: int) -> int:
    v = ctypes.c_int64()
    _check(ctx, load().grover_query(ctx, key, ctypes.byref(v)))
    return v.value


def grover_optimal_iterations(n: int, m: int) -> int:
    return int(load().grover_optimal_iterations(n, m))


def grover_destroy(ctx) -> None:
    if ctx:
        load().grover_destroy(ctx)


def grover_iterate_static(hip_stream: int, state_dev: int, n: int, dtype: int, marks_dev: int, m: int, k: int,
                          status_dev: int = 0) -> None:
    _check(None, load().grover_iterate_static(hip_stream or None, state_dev or None, n, dtype, marks_dev or None, m,
                                              k, status_dev or None))


GROVER_PROBE_READ_ONLY, GROVER_PROBE_LAUNCH_PER_PASS, GROVER_PROBE_WRITE_ONLY, GROVER_PROBE_NARROW = 1, 2, 4, 8


def grover_stream_probe(hip_stream: int, buf_dev: int, nbytes: int, passes: int, mode: int = 0) -> float:
    """Milliseconds for `passes` in-place (or read-only) streaming passes over a device buffer."""
    ms = ctypes.c_float()
    _check(None, load().grover_stream_probe(hip_stream or None, buf_dev or None, nbytes, passes, mode,
                                            ctypes.byref(ms)))
    return ms.value


def grover_status_str(status: int) -> str:
    return load().grover_status_str(status).decode()


def grover_last_error(ctx) -> str:
    return load().grover_last_error(ctx).decode()


def _bcheck(b, status: int) -> None:
    if status != GROVER_OK:
        lib = load()
        msg = lib.grover_batch_last_error(b).decode() if b else ""
        if not msg:
            msg = lib.grover_status_str(status).decode()
        raise GroverError(status, msg)


def grover_batch_init(cfg: grover_batch_config, hip_stream: int = 0):
    b = ctypes.c_void_p()
    _bcheck(None, load().grover_batch_init(ctypes.byref(b), ctypes.byref(cfg), hip_stream or None))
    return b


def grover_batch_set_tiling(b, split_n: int, team: int, resident: int = 0) -> None:
    _bcheck(b, load().grover_batch_set_tiling(b, split_n, team, resident))


def grover_batch_tune(b):
    s, t, r, ms = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_float()
    _bcheck(b, load().grover_batch_tune(b, ctypes.byref(s), ctypes.byref(t), ctypes.byref(r), ctypes.byref(ms)))
    return s.value, t.value, r.value, ms.value


def grover_batch_capture(b) -> None:
    _bcheck(b, load().grover_batch_capture(b))


def grover_batch_run(b) -> None:
    _bcheck(b, load().grover_batch_run(b))


def grover_batch_sync(b) -> None:
    _bcheck(b, load().grover_batch_sync(b))


def grover_batch_state(b, i: int):
    p, n = ctypes.c_void_p(), ctypes.c_size_t()
    _bcheck(b, load().grover_batch_state(b, i, ctypes.byref(p), ctypes.byref(n)))
    return p.value, n.value


def grover_batch_read_state(b, i: int, host: int, nbytes: int) -> None:
    _bcheck(b, load().grover_batch_read_state(b, i, host, nbytes))


def grover_batch_query(b, key: int) -> int:
    v = ctypes.c_int64()
    _bcheck(b, load().grover_batch_query(b, key, ctypes.byref(v)))
    return v.value


def grover_batch_destroy(b) -> None:
    if b:
        load().grover_batch_destroy(b)


def grover_batch_last_error(b) -> str:
    return load().grover_batch_last_error(b).decode()


def _pcheck(p, status: int) -> None:
    if status != GROVER_OK:
        lib = load()
        msg = lib.grover_phase_last_error(p).decode() if p else ""
        if not msg:
            msg = lib.grover_status_str(status).decode()
        raise GroverError(status, msg)


def grover_phase_init(cfg: grover_phase_config, hip_stream: int = 0):
    p = ctypes.c_void_p()
    _pcheck(None, load().grover_phase_init(ctypes.byref(p), ctypes.byref(cfg), hip_stream or None))
    return p


def grover_phase_set_team(p, team: int) -> None:
    _pcheck(p, load().grover_phase_set_team(p, team))


def grover_phase_set_form(p, form: int) -> None:
    _pcheck(p, load().grover_phase_set_form(p, form))


def grover_phase_forward(p, phi: int, theta: int, loss: int) -> None:
    _pcheck(p, load().grover_phase_forward(p, phi or None, theta or None, loss or None))


def grover_phase_backward(p, dloss: int, dphi: int, dtheta: int) -> None:
    _pcheck(p, load().grover_phase_backward(p, dloss or None, dphi or None, dtheta or None))


def grover_phase_sync(p) -> None:
    _pcheck(p, load().grover_phase_sync(p))


def grover_phase_state(p, b: int):
    ptr, n = ctypes.c_void_p(), ctypes.c_size_t()
    _pcheck(p, load().grover_phase_state(p, b, ctypes.byref(ptr), ctypes.byref(n)))
    return ptr.value, n.value


def grover_phase_read_state(p, b: int, host: int, nbytes: int) -> None:
    _pcheck(p, load().grover_phase_read_state(p, b, host, nbytes))


def grover_phase_query(p, key: int) -> int:
    v = ctypes.c_int64()
    _pcheck(p, load().grover_phase_query(p, key, ctypes.byref(v)))
    return v.value


def grover_phase_destroy(p) -> None:
    if p:
        load().grover_phase_destroy(p)


def grover_phase_last_error(p) -> str:
    return load().grover_phase_last_error(p).decode()


# --------------------------------------------------------------------------------- convenience class
class Grover:
    """One search instance: a state on the current GPU plus its marked set.

    n          qubits (N = 2^n amplitudes)
    dtype      "f64" (real), "c64", "c128" or "cbf16" (complex bfloat16)
    marks      explicit marked indices (oracle list), or None with hash_seed/hash_bits/m for the predicate
    form       "auto", "fused", "resident", "two_pass" or "held"
    accum      precision of the sum the mean is taken from: "f64", "f32" or "f32_kahan"
    update     precision of the element update: "f64" (rounded once to the storage) or "f32" (complex64
               storage with binary64 sums: binary32 arithmetic from 2S/N rounded to binary32)
    state      optional torch tensor (on the current device) to adopt as the state; otherwise one is made
    The state tensor is `self.state` (torch, 1-D, N elements of the dtype); kernels run on torch's
    current stream at construction.
    """

    def __init__(self, n: int, dtype: str = "c64", marks=None, *, hash_seed: Optional[int] = None,
                 hash_bits: int = 0, m: Optional[int] = None, form: str = "auto", accum: str = "f64",
                 update: str = "f64", state=None):
        import torch

        self.n = n
        self.dtype = DTYPES[dtype]
        N = 1 << n
        tdt = {GROVER_F64_REAL: torch.float64, GROVER_C64: torch.complex64, GROVER_C128: torch.complex128,
               GROVER_CBF16: torch.bfloat16}[self.dtype]
        numel = 2 * N if self.dtype == GROVER_CBF16 else N  # bfloat16: interleaved (re, im)
        self.state = state if state is not None else torch.empty(numel, dtype=tdt, device="cuda")
        if self.state.dtype != tdt or self.state.numel() != numel or not self.state.is_contiguous():
            raise ValueError("state tensor must be contiguous with N elements of the requested dtype")
        self.stream = torch.cuda.current_stream()
        cfg = grover_config()
        cfg.n = n
        cfg.dtype = self.dtype
        cfg.form = FORMS[form]
        cfg.flags = 0
        cfg.accum = ACCUMS[accum]
        cfg.update = UPDATES[update]
        if hash_seed is not None:
            cfg.oracle_kind = GROVER_ORACLE_HASH
            cfg.hash_seed = hash_seed & (2**64 - 1)
            cfg.hash_bits = hash_bits
            cfg.m = int(m if m is not None else 0)
            self._marks = None
        else:
            self._marks = np.ascontiguousarray(np.asarray(marks if marks is not None else [], dtype=np.uint64))
            cfg.oracle_kind = GROVER_ORACLE_LIST
            cfg.m = self._marks.size
            cfg.marked = self._marks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        nbytes = N * ELEM_BYTES[self.dtype]
        self.ctx = grover_init(cfg, self.stream.cuda_stream, self.state.data_ptr(), nbytes)
        self.N = N
        self.nbytes = nbytes

    # -- operations
    def reset(self) -> "Grover":
        grover_reset(self.ctx)
        return self

    def iterate(self, k: int) -> "Grover":
        grover_iterate(self.ctx, k)
        return self

    def gate_iterate(self, k: int) -> "Grover":
        grover_gate_iterate(self.ctx, k)
        return self

    def hadamard_all(self, blocked: bool = False) -> "Grover":
        (grover_apply_hadamard_all_blocked if blocked else grover_apply_hadamard_all)(self.ctx)
        return self

    def gate_iterate_blocked(self, k: int) -> "Grover":
        grover_gate_iterate_blocked(self.ctx, k)
        return self

    def sample(self, shots: int, seed: Optional[int] = None, u53=None, device_out: bool = False):
        """Measurement shots: device-generated uniforms from `seed`, or the given 53-bit uniforms `u53`
        (numpy array or torch device tensor of uint64/int64).  Returns numpy uint64 (host) or a torch
        int64 device tensor (device_out=True)."""
        import torch

        if device_out:
            out = torch.empty(shots, dtype=torch.int64, device=self.state.device)
            optr, odev = out.data_ptr(), True
        else:
            out = np.empty(shots, dtype=np.uint64)
            optr, odev = out.ctypes.data, False
        if u53 is None:
            grover_sample(self.ctx, shots, int(seed or 0), optr, odev)
        elif isinstance(u53, np.ndarray):
            u = np.ascontiguousarray(u53, dtype=np.uint64)
            grover_sample_u53(self.ctx, u.ctypes.data, False, shots, optr, odev)
        else:
            grover_sample_u53(self.ctx, u53.data_ptr(), True, shots, optr, odev)
        return out

    def norm(self) -> float:
        return grover_norm(self.ctx)

    def read_state(self) -> np.ndarray:
        """The state on the host: float64 / complex64 / complex128 arrays, complex128 for bfloat16 storage
        (exact conversion)."""
        if self.dtype == GROVER_CBF16:
            raw = np.empty(2 * self.N, dtype=np.uint16)
            grover_read_state(self.ctx, raw.ctypes.data, self.nbytes)
            return bf16_pairs_to_complex(raw)
        out = np.empty(self.N, dtype=NUMPY_DTYPES[self.dtype])
        grover_read_state(self.ctx, out.ctypes.data, self.nbytes)
        return out

    def write_state(self, psi: np.ndarray) -> "Grover":
        """Write a host state; values are rounded to the storage type (bfloat16: nearest even)."""
        if self.dtype == GROVER_CBF16:
            a = complex_to_bf16_pairs(np.asarray(psi))
        else:
            a = np.ascontiguousarray(psi, dtype=NUMPY_DTYPES[self.dtype])
        grover_write_state(self.ctx, a.ctypes.data, self.nbytes)
        return self

    def marked(self) -> np.ndarray:
        return grover_marked(self.ctx, grover_query(self.ctx, Q_M))

    def sync(self) -> None:
        grover_sync(self.ctx)

    def query(self, key: int) -> int:
        return grover_query(self.ctx, key)

    def close(self) -> None:
        if getattr(self, "ctx", None):
            grover_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            if sys.is_finalizing():  # the HIP runtime may already be torn down
                return
            self.close()
        except BaseException:
            pass


class GroverBatch:
    """Many independent searches (complex64 states) advanced by one persistent launch per run.

    n, m        per-instance qubit counts and marked-list lengths (sequences of equal length)
    marks       per-instance marked lists (a sequence of sequences), concatenated for the library
    iterations  per-instance iteration counts, or None for k_opt(n, m)
    Work goes to torch's current stream at construction.  `run()` restarts every instance from the uniform
    superposition and performs its iterations; `read_state(i)` returns instance i's state (complex64).
    """

    def __init__(self, n, m, marks, iterations=None, update: str = "f64"):
        import torch

        self._n = np.ascontiguousarray(np.asarray(n, dtype=np.uint32))
        self._m = np.ascontiguousarray(np.asarray(m, dtype=np.uint64))
        lists = [np.asarray(x, dtype=np.uint64).ravel() for x in marks]
        if len(lists) != self._n.size or self._m.size != self._n.size:
            raise ValueError("n, m and marks must have one entry per instance")
        self._marks = np.ascontiguousarray(np.concatenate(lists) if lists else np.zeros(0, np.uint64))
        self._iters = None if iterations is None else np.ascontiguousarray(np.asarray(iterations, np.uint64))
        cfg = grover_batch_config()
        cfg.count = self._n.size
        cfg.n = self._n.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        cfg.m = self._m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        if self._marks.size:
            cfg.marked = self._marks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        if self._iters is not None:
            cfg.iterations = self._iters.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        cfg.dtype = GROVER_C64
        cfg.update = UPDATES[update]
        self.stream = torch.cuda.current_stream()
        self.b = grover_batch_init(cfg, self.stream.cuda_stream)
        self.count = int(self._n.size)

    def set_tiling(self, split_n: int, team: int, resident: int = 0) -> "GroverBatch":
        grover_batch_set_tiling(self.b, split_n, team, resident)
        return self

    def tune(self):
        """(split_n, team, resident, milliseconds) of the fastest candidate tiling, which stays selected."""
        return grover_batch_tune(self.b)

    def capture(self) -> "GroverBatch":
        grover_batch_capture(self.b)
        return self

    def run(self) -> "GroverBatch":
        grover_batch_run(self.b)
        return self

    def sync(self) -> None:
        grover_batch_sync(self.b)

    def query(self, key: int) -> int:
        return grover_batch_query(self.b, key)

    def read_state(self, i: int) -> np.ndarray:
        out = np.empty(1 << int(self._n[i]), dtype=np.complex64)
        grover_batch_read_state(self.b, i, out.ctypes.data, out.nbytes)
        return out

    def close(self) -> None:
        if getattr(self, "b", None):
            grover_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            if sys.is_finalizing():
                return
            self.close()
        except BaseException:
            pass


class GroverPhase:
    """B schedules of the generalized iteration (phases phi_j on the marked amplitudes, theta_j in the
    diffusion) over one marked set, with the adjoint gradient; complex64 states on the current GPU.

    n, marks, K, batch   problem shape; checkpoint_every = 0 picks round(sqrt(K))
    `loss(phi, theta)` is differentiable with torch autograd: phi, theta are CUDA float64 tensors of shape
    (batch, K); the result has shape (batch,).  Each forward run must be followed by at most one backward
    run before the next forward (the adjoint sweep reuses the forward run's checkpoints).
    """

    def __init__(self, n: int, marks, K: int, batch: int = 1, checkpoint_every: int = 0):
        import torch

        self._marks = np.ascontiguousarray(np.asarray(marks, dtype=np.uint64).reshape(-1))
        cfg = grover_phase_config()
        cfg.n, cfg.batch, cfg.iterations, cfg.checkpoint_every = n, batch, K, checkpoint_every
        cfg.m = self._marks.size
        if self._marks.size:
            cfg.marked = self._marks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        cfg.dtype = GROVER_C64
        self.stream = torch.cuda.current_stream()
        self.p = grover_phase_init(cfg, self.stream.cuda_stream)
        self.n, self.K, self.batch = n, K, batch
        self.generation = 0

    def _enter(self):
        import torch

        cur = torch.cuda.current_stream()
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)
        return cur

    def _leave(self, cur):
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.wait_stream(self.stream)

    def forward(self, phi, theta):
        """Loss per schedule (torch float64, shape (batch,)) without autograd."""
        import torch

        phi = phi.detach().to(torch.float64).contiguous()
        theta = theta.detach().to(torch.float64).contiguous()
        if phi.shape != (self.batch, self.K) or theta.shape != (self.batch, self.K) or not phi.is_cuda:
            raise ValueError(f"phi and theta must be CUDA tensors of shape ({self.batch}, {self.K})")
        loss = torch.empty(self.batch, dtype=torch.float64, device=phi.device)
        cur = self._enter()
        grover_phase_forward(self.p, phi.data_ptr(), theta.data_ptr(), loss.data_ptr())
        for t in (phi, theta, loss):
            t.record_stream(self.stream)
        self._leave(cur)
        self.generation += 1
        return loss

    def backward(self, dloss):
        """(dphi, dtheta) of sum_b dloss[b] * L_b at the last forward run's phases."""
        import torch

        dloss = dloss.detach().to(torch.float64).contiguous()
        dphi = torch.empty(self.batch, self.K, dtype=torch.float64, device=dloss.device)
        dtheta = torch.empty_like(dphi)
        cur = self._enter()
        grover_phase_backward(self.p, dloss.data_ptr(), dphi.data_ptr(), dtheta.data_ptr())
        for t in (dloss, dphi, dtheta):
            t.record_stream(self.stream)
        self._leave(cur)
        return dphi, dtheta

    def loss(self, phi, theta):
        """Differentiable loss: torch.autograd calls the adjoint kernel for the gradient."""
        return _PhaseLoss.apply(phi, theta, self)

    def set_form(self, form: str) -> "GroverPhase":
        """"auto", "streamed" (states in memory every iteration) or "held" (on chip for all iterations)."""
        forms = {"auto": GROVER_PHASE_FORM_AUTO, "streamed": GROVER_PHASE_FORM_STREAMED,
                 "held": GROVER_PHASE_FORM_HELD}
        grover_phase_set_form(self.p, forms[form])
        return self

    def sync(self) -> None:
        grover_phase_sync(self.p)

    def query(self, key: int) -> int:
        return grover_phase_query(self.p, key)

    def read_state(self, b: int) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=np.complex64)
        grover_phase_read_state(self.p, b, out.ctypes.data, out.nbytes)
        return out

    def close(self) -> None:
        if getattr(self, "p", None):
            grover_phase_destroy(self.p)
            self.p = None

    def __del__(self):
        try:
            if sys.is_finalizing():
                return
            self.close()
        except BaseException:
            pass


def _phase_loss_function():
    import torch

    class PhaseLoss(torch.autograd.Function):
        """L_b(phi_b, theta_b) through libgrover: forward kernel for the value, adjoint kernel for the
        gradient (no intermediate state is kept by torch)."""

        @staticmethod
        def forward(ctx, phi, theta, engine):
            loss = engine.forward(phi, theta)
            ctx.engine = engine
            ctx.generation = engine.generation
            return loss

        @staticmethod
        def backward(ctx, grad_loss):
            engine = ctx.engine
            if engine.generation != ctx.generation:
                raise RuntimeError("another forward run replaced the checkpoints this backward needs")
            dphi, dtheta = engine.backward(grad_loss)
            return dphi, dtheta, None

    return PhaseLoss


class _LazyPhaseLoss:
    _fn = None

    @classmethod
    def apply(cls, *args):
        if cls._fn is None:
            cls._fn = _phase_loss_function()
        return cls._fn.apply(*args)


_PhaseLoss = _LazyPhaseLoss
