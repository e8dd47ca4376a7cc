"""Seeded synthetic inputs for the Grover hot path.

This module is shared by the tests, the benchmark and the CPU oracle's callers. It produces inputs only:
problem sizes, marked index lists, hash seeds, random starting states and the uniform variates that
measurement consumes. It holds none of the arithmetic of the search itself (no oracle sign, no mean,
no update, no CDF).

The paper uses no dataset: its workloads are a 3-qubit example and single-solution searches at
n = 10, 16, 18 and 20 qubits (Simulation Results, Fig. 2 and Table 1). Everything here is synthetic by
construction.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), used as a counter-based generator: output j of the generator seeded with s is
mix64(s + (j + 1) * 0x9E3779B97F4A7C15), mix64 being the published variant with the multipliers
0xBF58476D1CE4E5B9 and 0x94D049BB133111EB.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+count-1 of SplitMix64 seeded with `seed`, as uint64."""
    with np.errstate(over="ignore"):
        j = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + j * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
        return z ^ (z >> np.uint64(31))


def uniforms_u53(seed: int, shots: int) -> np.ndarray:
    """53-bit uniform integers U_j = SplitMix64_j(seed) >> 11 in [0, 2^53), one per measurement shot."""
    return splitmix64(seed, shots) >> np.uint64(11)


def marked_index_from_seed(n: int, seed: int) -> int:
    """One index drawn uniformly from [0, 2^n): the top n bits of output 0 (no modulo bias)."""
    return int(splitmix64(seed, 1)[0]) >> (64 - n) if n > 0 else 0


def distinct_marks(n: int, m: int, seed: int) -> np.ndarray:
    """m distinct indices in [0, 2^n), sorted, drawn from SplitMix64(seed) top bits with rejection."""
    N = 1 << n
    if m > N:
        raise ValueError("m > N")
    if m > N // 2:
        # draw the complement instead so the rejection loop stays short
        rest = set(distinct_marks(n, N - m, seed ^ 0x5DEECE66D).tolist())
        return np.array([i for i in range(N) if i not in rest], dtype=np.uint64)
    out: set[int] = set()
    j = 0
    while len(out) < m:
        batch = splitmix64(seed, 64, start=j)
        j += 64
        for v in batch.tolist():
            idx = v >> (64 - n) if n > 0 else 0
            if idx not in out:
                out.add(idx)
                if len(out) == m:
                    break
    return np.array(sorted(out), dtype=np.uint64)


def random_state(n: int, seed: int, real: bool = False) -> np.ndarray:
    """A normalised random state of 2^n amplitudes (complex128), used to exercise general, non-uniform inputs."""
    N = 1 << n
    u = splitmix64(seed, 2 * N).astype(np.float64) * (2.0 ** -64) - 0.5
    psi = u[0::2] + (0.0 if real else 1j) * u[1::2]
    psi = psi.astype(np.complex128)
    return psi / np.sqrt(np.sum(np.abs(psi) ** 2))


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic search problem.

    name        short identifier
    n           qubit count, N = 2^n amplitudes
    dtype       storage type of the amplitudes: "f64" (real), "c64" (complex64) or "c128" (complex128)
    m           number of marked indices
    marks       explicit marked list (oracle given as a list), or None when a hash predicate defines them
    hash_seed   seed of the hash predicate (low `hash_bits` bits of SplitMix64_i(hash_seed) all zero)
    hash_bits   width of the predicate's zero test
    iterations  Grover iterations, floor(pi/4 * sqrt(N/M))
    shots       measurement shots
    shot_seed   seed of the uniforms that measurement consumes
    """

    name: str
    n: int
    dtype: str
    m: int
    marks: Optional[tuple]
    hash_seed: Optional[int]
    hash_bits: int
    iterations: int
    shots: int
    shot_seed: int


# Plain Grover, n = 10, real FP64, one marked index drawn from a seed, 25 iterations, 10^4 shots.
PLAIN_N10_SEED = 20050463
PLAIN_N10 = Workload(
    name="plain_n10_f64_m1",
    n=10,
    dtype="f64",
    m=1,
    marks=(marked_index_from_seed(10, PLAIN_N10_SEED),),
    hash_seed=None,
    hash_bits=0,
    iterations=25,
    shots=10_000,
    shot_seed=7,
)

# Single large instance, n = 28 complex64, M = 8 marked indices defined by the hash predicate
# (hash(i, seed) mod 2^25 == 0).  The seed is the first one at or above 0x6A09E667F3BCC908 whose predicate
# has exactly 8 hits over 2^28 indices; `oracle/find_hash_seed.py` searched it with the CPU oracle only.
HASH_N28_SEED = 0x6A09E667F3BCC910
HASH_N28 = Workload(
    name="hash_n28_c64_m8",
    n=28,
    dtype="c64",
    m=8,
    marks=None,
    hash_seed=HASH_N28_SEED,
    hash_bits=25,
    iterations=4549,
    shots=1_000_000,
    shot_seed=11,
)

# Precision sweep, n = 26, M = 4 marked indices drawn from a seed, floor(pi/4 sqrt(N/M)) = 3216 iterations;
# the storage type and the accumulator of the mean are the swept settings (dtype here is the reference one).
PRECISION_N26_SEED = 2600426
PRECISION_N26 = Workload(
    name="precision_n26_m4",
    n=26,
    dtype="c128",
    m=4,
    marks=tuple(int(x) for x in distinct_marks(26, 4, PRECISION_N26_SEED)),
    hash_seed=None,
    hash_bits=0,
    iterations=3216,
    shots=0,
    shot_seed=0,
)

WORKLOADS = {w.name: w for w in (PLAIN_N10, HASH_N28, PRECISION_N26)}


@dataclasses.dataclass(frozen=True)
class BatchWorkload:
    """Many independent searches with uneven sizes.

    Instance b takes x = SplitMix64_{3b}(seed), x' = SplitMix64_{3b+1}(seed) and s = SplitMix64_{3b+2}(seed):
    n_b = n_min + (x mod n_span), M_b = 1 + (x' mod m_max), and M_b distinct marked indices drawn by
    `distinct_marks(n_b, M_b, s)`.  Each instance runs its own floor(pi/4 sqrt(N_b / M_b)) iterations from
    the uniform superposition; states are complex64.
    """

    name: str
    count: int
    n_min: int
    n_span: int
    m_max: int
    seed: int

    def instances(self):
        """(n, m, marks) arrays: n uint32[count], m uint64[count], marks = list of uint64 arrays."""
        s = splitmix64(self.seed, 3 * self.count)
        n = (self.n_min + s[0::3] % np.uint64(self.n_span)).astype(np.uint32)
        m = (np.uint64(1) + s[1::3] % np.uint64(self.m_max)).astype(np.uint64)
        marks = [distinct_marks(int(n[b]), int(m[b]), int(s[3 * b + 2])) for b in range(self.count)]
        return n, m, marks

    def write_instances(self, path: str) -> None:
        """One line per instance, "n m mark_1 ... mark_m" (the native driver's batch input format)."""
        n, m, marks = self.instances()
        with open(path, "w") as f:
            for b in range(self.count):
                f.write(" ".join([str(int(n[b])), str(int(m[b]))] + [str(int(x)) for x in marks[b]]) + "\n")


# 4096 searches, n uniform in [8, 20], M uniform in [1, 8].
BATCH_4096 = BatchWorkload(name="batch4096_n8to20_m1to8_c64", count=4096, n_min=8, n_span=13, m_max=8,
                           seed=0x4096C3B5)


def normal_pairs(seed: int, count: int) -> np.ndarray:
    """`count` standard normal variates: Box-Muller on consecutive pairs of 53-bit uniforms of SplitMix64."""
    pairs = (count + 1) // 2
    u = (splitmix64(seed, 2 * pairs) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u1, u2 = u[0::2], u[1::2]
    r = np.sqrt(-2.0 * np.log1p(-u1))
    z = np.empty(2 * pairs)
    z[0::2] = r * np.cos(2.0 * np.pi * u2)
    z[1::2] = r * np.sin(2.0 * np.pi * u2)
    return z[:count]


def phase_schedule(K: int, seed: int, spread: float = 0.1, batch: int = 1):
    """Per-iteration phases phi, theta ~ N(pi, spread^2), shape (batch, K) each (float64)."""
    z = normal_pairs(seed, 2 * batch * K).reshape(batch, 2, K)
    return np.pi + spread * z[:, 0, :], np.pi + spread * z[:, 1, :]


@dataclasses.dataclass(frozen=True)
class PhaseWorkload:
    """A batch of phase schedules for the generalized iteration: n qubits, m marked indices drawn from
    `seed`, K iterations, `batch` schedules with phi, theta ~ N(pi, spread^2) drawn from `seed + 1`."""

    name: str
    n: int
    m: int
    K: int
    batch: int
    spread: float
    seed: int

    def marks(self) -> np.ndarray:
        return distinct_marks(self.n, self.m, self.seed)

    def schedules(self):
        return phase_schedule(self.K, self.seed + 1, self.spread, self.batch)

    def write_file(self, path: str) -> None:
        """"n m K B", the marks, B rows of phi, B rows of theta (the native driver's input format)."""
        phi, theta = self.schedules()
        with open(path, "w") as f:
            f.write(f"{self.n} {self.m} {self.K} {self.batch}\n")
            f.write(" ".join(str(int(x)) for x in self.marks()) + "\n")
            for rows in (phi, theta):
                for r in rows:
                    f.write(" ".join(repr(float(x)) for x in r) + "\n")


# Differentiable generalized search: n = 20, M = 3, K = 64 iterations, 64 schedules, phases N(pi, 0.1).
PHASE_N20 = PhaseWorkload(name="phase_n20_m3_k64_b64", n=20, m=3, K=64, batch=64, spread=0.1, seed=0x5EED2005)
