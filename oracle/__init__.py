"""Plain CPU FP64 oracle for arXiv:2005.04635 (Python side).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package; the product library never does, and shares no code with it.

The arithmetic lives in `grover_oracle.c` (plain C, binary64, no fused multiply-add). This module only
builds that file with gcc and marshals numpy arrays through ctypes. States are numpy complex128 arrays of
length 2^n, whose memory layout (real, imaginary interleaved) is the one the C code expects.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "grover_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra"]


def build(src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc into a shared library (always recompiles)."""
    tmp = out + ".tmp"
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, src, "-lm"], check=True)
    os.replace(tmp, out)
    return out


def load(path: str = _LIB):
    """Load (building first if absent) the oracle library and declare its prototypes."""
    global _lib
    with _lock:
        if _lib is not None and path == _LIB:
            return _lib
        if not os.path.exists(path):
            build(out=path)
        lib = ctypes.CDLL(path)
        u64, u32, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double
        pd, pu = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64)
        sig = {
            "orc_splitmix64": (u64, [u64, u64]),
            "orc_hash_marks": (u64, [u32, u64, u32, pu, u64]),
            "orc_optimal_iterations": (u64, [u32, u64]),
            "orc_uniform_amplitude": (dbl, [u32]),
            "orc_init_uniform": (None, [u32, pd]),
            "orc_oracle": (None, [pd, pu, u64]),
            "orc_inversion_about_mean": (None, [u32, pd]),
            "orc_grover_iterate": (None, [u32, pd, pu, u64, u64]),
            "orc_grover_search": (None, [u32, pu, u64, u64, pd]),
            "orc_unitary_1q": (ctypes.c_int, [u32, pd, u32, pd]),
            "orc_hadamard_all": (ctypes.c_int, [u32, pd]),
            "orc_conditional_phase_shift": (None, [u32, pd]),
            "orc_gate_iterate": (ctypes.c_int, [u32, pd, pu, u64, u64]),
            "orc_gate_search": (ctypes.c_int, [u32, pu, u64, u64, pd]),
            "orc_norm": (dbl, [u32, pd]),
            "orc_two_class": (None, [u32, u64, u64, pd, pd]),
            "orc_round_to_bits": (dbl, [dbl, ctypes.c_int]),
            "orc_two_class_stored": (None, [u32, u64, u64, ctypes.c_int, pd, pd]),
            "orc_two_class_stored_update": (None, [u32, u64, u64, ctypes.c_int, ctypes.c_int, pd, pd]),
            "orc_grover_iterate_stored": (None, [u32, pd, pu, u64, u64, ctypes.c_int, ctypes.c_int]),
            "orc_sample": (ctypes.c_int, [u32, pd, pu, u64, pu]),
            "orc_uniforms_u53": (None, [u64, u64, pu]),
            "orc_phase_oracle": (None, [pd, pu, u64, dbl]),
            "orc_phase_diffusion": (None, [u32, pd, dbl]),
            "orc_phase_search": (None, [u32, pu, u64, u64, pd, pd, pd]),
            "orc_phase_loss": (dbl, [pd, pu, u64]),
            "orc_phase_grad_tangent": (ctypes.c_int, [u32, pu, u64, u64, pd, pd, pd, pd]),
            "orc_phase_grad_adjoint": (ctypes.c_int, [u32, pu, u64, u64, pd, pd, pd, pd]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        if path == _LIB:
            _lib = lib
        return lib


def _pd(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pu(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _state(psi: np.ndarray) -> np.ndarray:
    if psi.dtype != np.complex128 or not psi.flags.c_contiguous:
        raise TypeError("oracle states are C-contiguous complex128 arrays")
    return psi


def _marks(k) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(k, dtype=np.uint64).reshape(-1))


def _params(phi, theta):
    ph = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).reshape(-1))
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1))
    if ph.size != th.size:
        raise ValueError("phi and theta need one entry per iteration")
    return ph, th


def _n_of(psi: np.ndarray) -> int:
    n = int(psi.size).bit_length() - 1
    if psi.size != 1 << n:
        raise ValueError("state length is not a power of two")
    return n


class Oracle:
    """Thin numpy wrapper around one loaded oracle library (the default one, or a test build)."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    def splitmix64(self, seed: int, j: int) -> int:
        return int(self.lib.orc_splitmix64(seed & (2**64 - 1), j))

    def hash_marks(self, n: int, seed: int, bits: int, cap: int = 1 << 16):
        out = np.zeros(max(cap, 1), dtype=np.uint64)
        count = int(self.lib.orc_hash_marks(n, seed & (2**64 - 1), bits, _pu(out), cap))
        return out[: min(count, cap)].copy(), count

    def optimal_iterations(self, n: int, m: int) -> int:
        return int(self.lib.orc_optimal_iterations(n, m))

    def uniform_amplitude(self, n: int) -> float:
        return float(self.lib.orc_uniform_amplitude(n))

    def init_uniform(self, n: int) -> np.ndarray:
        psi = np.empty(1 << n, dtype=np.complex128)
        self.lib.orc_init_uniform(n, _pd(psi))
        return psi

    def oracle(self, psi: np.ndarray, marks) -> np.ndarray:
        k = _marks(marks)
        self.lib.orc_oracle(_pd(_state(psi)), _pu(k), k.size)
        return psi

    def inversion_about_mean(self, psi: np.ndarray) -> np.ndarray:
        self.lib.orc_inversion_about_mean(_n_of(psi), _pd(_state(psi)))
        return psi

    def iterate(self, psi: np.ndarray, marks, iters: int) -> np.ndarray:
        """Algorithm 5's loop body `iters` times, in place on `psi`."""
        k = _marks(marks)
        self.lib.orc_grover_iterate(_n_of(psi), _pd(_state(psi)), _pu(k), k.size, iters)
        return psi

    def search(self, n: int, marks, iters: int) -> np.ndarray:
        k = _marks(marks)
        psi = np.empty(1 << n, dtype=np.complex128)
        self.lib.orc_grover_search(n, _pu(k), k.size, iters, _pd(psi))
        return psi

    def unitary_1q(self, psi: np.ndarray, q: int, u: np.ndarray) -> np.ndarray:
        uu = np.ascontiguousarray(np.asarray(u, dtype=np.complex128).reshape(2, 2))
        flat = np.array([uu[0, 0].real, uu[0, 0].imag, uu[0, 1].real, uu[0, 1].imag,
                         uu[1, 0].real, uu[1, 0].imag, uu[1, 1].real, uu[1, 1].imag], dtype=np.float64)
        if self.lib.orc_unitary_1q(_n_of(psi), _pd(_state(psi)), q, _pd(flat)) != 0:
            raise MemoryError("oracle scratch allocation failed")
        return psi

    def hadamard_all(self, psi: np.ndarray) -> np.ndarray:
        if self.lib.orc_hadamard_all(_n_of(psi), _pd(_state(psi))) != 0:
            raise MemoryError("oracle scratch allocation failed")
        return psi

    def conditional_phase_shift(self, psi: np.ndarray) -> np.ndarray:
        self.lib.orc_conditional_phase_shift(_n_of(psi), _pd(_state(psi)))
        return psi

    def gate_iterate(self, psi: np.ndarray, marks, iters: int) -> np.ndarray:
        k = _marks(marks)
        if self.lib.orc_gate_iterate(_n_of(psi), _pd(_state(psi)), _pu(k), k.size, iters) != 0:
            raise MemoryError("oracle scratch allocation failed")
        return psi

    def gate_search(self, n: int, marks, iters: int) -> np.ndarray:
        k = _marks(marks)
        psi = np.empty(1 << n, dtype=np.complex128)
        if self.lib.orc_gate_search(n, _pu(k), k.size, iters, _pd(psi)) != 0:
            raise MemoryError("oracle scratch allocation failed")
        return psi

    def norm(self, psi: np.ndarray) -> float:
        return float(self.lib.orc_norm(_n_of(psi), _pd(_state(psi))))

    def two_class(self, n: int, m: int, iters: int):
        a, b = ctypes.c_double(), ctypes.c_double()
        self.lib.orc_two_class(n, m, iters, ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def round_to_bits(self, x: float, p: int) -> float:
        return float(self.lib.orc_round_to_bits(float(x), p))

    def two_class_stored(self, n: int, m: int, iters: int, p: int):
        a, b = ctypes.c_double(), ctypes.c_double()
        self.lib.orc_two_class_stored(n, m, iters, p, ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def two_class_stored_update(self, n: int, m: int, iters: int, p_store: int, p_update: int):
        a, b = ctypes.c_double(), ctypes.c_double()
        self.lib.orc_two_class_stored_update(n, m, iters, p_store, p_update, ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def iterate_stored(self, psi: np.ndarray, marks, iters: int, p_store: int, p_update: int) -> np.ndarray:
        """Iterations with the state stored at p_store bits and the update computed at p_update bits (in
        place); psi must already hold values representable at p_store bits."""
        k = _marks(marks)
        self.lib.orc_grover_iterate_stored(_n_of(psi), _pd(_state(psi)), _pu(k), k.size, iters, p_store, p_update)
        return psi

    def sample(self, psi: np.ndarray, u53: np.ndarray) -> np.ndarray:
        u = np.ascontiguousarray(np.asarray(u53, dtype=np.uint64))
        out = np.empty(u.size, dtype=np.uint64)
        rc = self.lib.orc_sample(_n_of(psi), _pd(_state(psi)), _pu(u), u.size, _pu(out))
        if rc == -2:
            raise ValueError("every probability rounds to zero")
        if rc != 0:
            raise MemoryError("oracle CDF allocation failed")
        return out

    # -- generalized iteration with per-iteration phases (phi_j on the marked entries, theta_j in the
    #    diffusion); phi = theta = pi is Algorithm 3 + Eq. 2
    def phase_oracle(self, psi: np.ndarray, marks, phi: float) -> np.ndarray:
        k = _marks(marks)
        self.lib.orc_phase_oracle(_pd(_state(psi)), _pu(k), k.size, float(phi))
        return psi

    def phase_diffusion(self, psi: np.ndarray, theta: float) -> np.ndarray:
        self.lib.orc_phase_diffusion(_n_of(psi), _pd(_state(psi)), float(theta))
        return psi

    def phase_search(self, n: int, marks, phi, theta) -> np.ndarray:
        k = _marks(marks)
        ph, th = _params(phi, theta)
        psi = np.empty(1 << n, dtype=np.complex128)
        self.lib.orc_phase_search(n, _pu(k), k.size, ph.size, _pd(ph), _pd(th), _pd(psi))
        return psi

    def phase_loss(self, psi: np.ndarray, marks) -> float:
        k = _marks(marks)
        return float(self.lib.orc_phase_loss(_pd(_state(psi)), _pu(k), k.size))

    def phase_grad_tangent(self, n: int, marks, phi, theta):
        return self._phase_grad(self.lib.orc_phase_grad_tangent, n, marks, phi, theta)

    def phase_grad_adjoint(self, n: int, marks, phi, theta):
        return self._phase_grad(self.lib.orc_phase_grad_adjoint, n, marks, phi, theta)

    @staticmethod
    def _phase_grad(fn, n, marks, phi, theta):
        k = _marks(marks)
        ph, th = _params(phi, theta)
        dphi, dtheta = np.empty(ph.size), np.empty(ph.size)
        if fn(n, _pu(k), k.size, ph.size, _pd(ph), _pd(th), _pd(dphi), _pd(dtheta)) != 0:
            raise MemoryError("oracle gradient allocation failed")
        return dphi, dtheta

    def uniforms_u53(self, seed: int, shots: int) -> np.ndarray:
        out = np.empty(shots, dtype=np.uint64)
        self.lib.orc_uniforms_u53(seed & (2**64 - 1), shots, _pu(out))
        return out


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
