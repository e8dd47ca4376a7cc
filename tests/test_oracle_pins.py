"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU, no HIP library).

Each test names the passage or the mathematical fact it rests on. Together they are chosen so that a
plausible slip in the oracle (a dropped term, a wrong sign, a wrong divisor, a skipped index, a transposed
operand, a wrong loop count) fails at least one of them; tests/test_oracle_mutants.py checks that claim by
planting such slips in a copy of the oracle.
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest
import scipy.linalg

import workloads
from conftest import GOLDEN

mpmath.mp.dps = 50


# ---------------------------------------------------------------------------------------------- helpers
def closed_form(n: int, m: int, k: int):
    """Boyer-Brassard-Hoyer-Tapp closed form of Grover's amplitudes after k iterations from the uniform state:
    each marked amplitude sin((2k+1) theta)/sqrt(M), each unmarked cos((2k+1) theta)/sqrt(N-M),
    theta = arcsin sqrt(M/N); evaluated at 50 digits."""
    N = mpmath.mpf(2) ** n
    theta = mpmath.asin(mpmath.sqrt(mpmath.mpf(m) / N))
    a = mpmath.sin((2 * k + 1) * theta) / mpmath.sqrt(m) if m > 0 else mpmath.mpf(0)
    b = mpmath.cos((2 * k + 1) * theta) / mpmath.sqrt(N - m) if m < N else mpmath.mpf(0)
    return float(a), float(b)


def dense_diffusion(n: int) -> np.ndarray:
    """Eq. 2 written out: Delta_ii = 2/N - 1, Delta_ij = 2/N for i != j."""
    N = 1 << n
    return np.full((N, N), 2.0 / N) - np.eye(N)


def dense_oracle(n: int, marks) -> np.ndarray:
    """The phase oracle of the Background section as a matrix: diag((-1)^f(x))."""
    s = np.ones(1 << n)
    s[np.asarray(marks, dtype=np.int64)] = -1.0
    return np.diag(s)


def sylvester_hadamard(n: int) -> np.ndarray:
    """H^(x)n = Walsh-Hadamard matrix / sqrt(N) (scipy's Sylvester construction)."""
    return scipy.linalg.hadamard(1 << n).astype(np.float64) / math.sqrt(1 << n)


def read_fig2():
    rows = []
    with open(os.path.join(GOLDEN, "fig2_three_qubit.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                state, pct = line.split()
                rows.append((int(state, 2), float(pct)))
    return dict(rows)


# ------------------------------------------------------------------------------------- worked example
def test_fig2_worked_example(orc):
    """Fig. 2: 3 qubits, solution |101>, after the algorithm's iterations the measured probabilities are
    94.531 % for |101> and 0.781 % for each other state (printed to 3 decimals)."""
    printed = read_fig2()
    k = orc.optimal_iterations(3, 1)
    psi = orc.search(3, [5], k)
    p = np.abs(psi) ** 2 * 100.0
    for i in range(8):
        assert round(p[i], 3) == pytest.approx(printed[i], abs=1e-9), (i, p[i], printed[i])
    # exact values behind the printed ones: 121/128 and 1/128
    assert abs(p[5] / 100 - 121 / 128) < 1e-15
    assert np.all(np.abs(np.delete(p, 5) / 100 - 1 / 128) < 1e-15)


def test_fig2_pins_iteration_count(orc):
    """Fig. 2 fixes floor(pi/4 sqrt(N)) = 2 iterations at N = 8; running the printed loop bound literally
    (iter < pi sqrt(N)/4, i.e. 3 passes) would give 169/512 = 33 %, not the printed 94.531 %."""
    assert orc.optimal_iterations(3, 1) == 2
    psi3 = orc.search(3, [5], 3)
    assert abs(abs(psi3[5]) ** 2 - 169 / 512) < 1e-15
    assert round(abs(psi3[5]) ** 2 * 100, 3) != read_fig2()[5]


def test_iteration_counts_of_the_workloads(orc):
    """floor(pi/4 sqrt(N/M)) at the workload sizes; none lies within 1e-3 of an integer, so binary64 floor is
    safe (checked here at 50 digits)."""
    for n, m, k in [(3, 1, 2), (10, 1, 25), (28, 8, 4549), (26, 4, 3216), (20, 1, 804), (20, 3, 464)]:
        exact = mpmath.pi / 4 * mpmath.sqrt(mpmath.mpf(2) ** n / m)
        assert int(mpmath.floor(exact)) == k
        assert orc.optimal_iterations(n, m) == k
    assert orc.optimal_iterations(10, 0) == 0
    assert workloads.PLAIN_N10.iterations == orc.optimal_iterations(10, 1)
    assert workloads.HASH_N28.iterations == orc.optimal_iterations(28, 8)


# ---------------------------------------------------------------------------------------- closed form
@pytest.mark.parametrize("n,m", [(4, 1), (5, 2), (6, 3), (8, 1), (9, 5), (10, 1), (11, 7), (12, 4)])
def test_closed_form(orc, n, m):
    """Grover's closed form sin((2k+1)theta)/sqrt(M) (marked) and cos((2k+1)theta)/sqrt(N-M) (unmarked),
    for every k up to twice the optimal count (past the peak as well)."""
    marks = workloads.distinct_marks(n, m, seed=1000 * n + m)
    mask = np.zeros(1 << n, dtype=bool)
    mask[marks.astype(np.int64)] = True
    kopt = orc.optimal_iterations(n, m)
    psi = orc.init_uniform(n)
    for k in range(0, 2 * kopt + 2):
        a, b = closed_form(n, m, k)
        assert np.max(np.abs(psi[mask] - a)) < 1e-13, k
        assert np.max(np.abs(psi[~mask] - b)) < 1e-13, k
        assert np.all(psi.imag == 0.0)
        orc.iterate(psi, marks, 1)


@pytest.mark.parametrize("n,m,k", [(20, 1, 804), (20, 3, 464), (26, 4, 3216), (28, 8, 4549), (16, 1, 201)])
def test_two_class_closed_form_large(orc, n, m, k):
    """The oracle's two-class form against the closed form at the paper's and the workloads' sizes."""
    a, b = orc.two_class(n, m, k)
    ea, eb = closed_form(n, m, k)
    assert abs(a - ea) < 1e-12 and abs(b - eb) < 1e-12


@pytest.mark.parametrize("n,m", [(3, 1), (6, 2), (9, 3), (12, 8)])
def test_two_class_equals_full_state(orc, n, m):
    """The two-class form is the full iteration restricted to a two-valued state."""
    marks = workloads.distinct_marks(n, m, seed=n * 31 + m)
    mask = np.zeros(1 << n, dtype=bool)
    mask[marks.astype(np.int64)] = True
    k = orc.optimal_iterations(n, m) + 3
    psi = orc.search(n, marks, k)
    a, b = orc.two_class(n, m, k)
    assert np.max(np.abs(psi[mask] - a)) < 1e-14
    assert np.max(np.abs(psi[~mask] - b)) < 1e-14


# ------------------------------------------------------------------------------ dense definition (Eq. 2)
@pytest.mark.parametrize("n,m,k", [(1, 1, 3), (2, 1, 2), (3, 2, 4), (5, 3, 7), (6, 1, 9), (7, 5, 4)])
def test_dense_eq2_on_general_states(orc, n, m, k):
    """Eq. 2 (Delta = 2J/N - I) times the oracle, as explicit matrices, applied k times to a random complex
    state: pins the mean over all N amplitudes, the divisor N, the absence of conjugation and the order
    (oracle first, then inversion about the mean)."""
    marks = workloads.distinct_marks(n, m, seed=7 * n + m)
    psi0 = workloads.random_state(n, seed=100 + n)
    G = dense_diffusion(n) @ dense_oracle(n, marks)
    want = psi0.copy()
    for _ in range(k):
        want = G @ want
    got = orc.iterate(psi0.copy(), marks, k)
    assert np.max(np.abs(got - want)) < 1e-13


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6])
def test_oracle_and_mean_separately(orc, n):
    """Algorithm 3 alone is the diagonal sign matrix, Algorithm 4 alone is Eq. 2."""
    marks = workloads.distinct_marks(n, max(1, (1 << n) // 3), seed=n)
    psi0 = workloads.random_state(n, seed=200 + n)
    got = orc.oracle(psi0.copy(), marks)
    assert np.array_equal(got, dense_oracle(n, marks) @ psi0)
    got = orc.inversion_about_mean(psi0.copy())
    assert np.max(np.abs(got - dense_diffusion(n) @ psi0)) < 1e-14


# ------------------------------------------------------------------------------- gate level (Alg. 1, 2)
@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_hadamard_all_is_walsh_hadamard(orc, n):
    """n applications of Algorithm 1 with U = H give the Walsh-Hadamard matrix (scipy's Sylvester matrix)."""
    N = 1 << n
    H = sylvester_hadamard(n)
    got = np.empty((N, N), dtype=np.complex128)
    for j in range(N):
        e = np.zeros(N, dtype=np.complex128)
        e[j] = 1.0
        got[:, j] = orc.hadamard_all(e)
    assert np.max(np.abs(got - H)) < 1e-14
    psi = workloads.random_state(n, seed=n)
    twice = orc.hadamard_all(orc.hadamard_all(psi.copy()))
    assert np.max(np.abs(twice - psi)) < 1e-14


@pytest.mark.parametrize("n,q", [(1, 0), (2, 0), (2, 1), (4, 1), (5, 4), (6, 2)])
def test_unitary_1q_matches_kronecker(orc, n, q):
    """Algorithm 1 / Eq. 1 for a general complex unitary U on qubit q equals I (x) ... U ... (x) I acting
    on the state (qubit q = bit q of the index): pins the a12 / a21 orientation and the bit convention."""
    rng = np.random.default_rng(17 + n * 8 + q)
    z = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    U, _ = np.linalg.qr(z)
    full = np.kron(np.kron(np.eye(1 << (n - 1 - q)), U), np.eye(1 << q))
    psi = workloads.random_state(n, seed=300 + n + q)
    got = orc.unitary_1q(psi.copy(), q, U)
    assert np.max(np.abs(got - full @ psi)) < 1e-14


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6])
def test_conditional_phase_shift_gives_eq2(orc, n):
    """Steps 3-5 of the Background list (H^n, 2|0><0| - I, H^n) equal the inversion about the mean, Eq. 2;
    checked column by column through the oracle's own gate routines."""
    N = 1 << n
    got = np.empty((N, N), dtype=np.complex128)
    for j in range(N):
        e = np.zeros(N, dtype=np.complex128)
        e[j] = 1.0
        orc.hadamard_all(e)
        orc.conditional_phase_shift(e)
        orc.hadamard_all(e)
        got[:, j] = e
    assert np.max(np.abs(got - dense_diffusion(n))) < 1e-13
    e0 = np.zeros(N, dtype=np.complex128)
    e0[0] = 1.0
    assert np.array_equal(orc.conditional_phase_shift(e0.copy()), e0)


@pytest.mark.parametrize("n,m", [(1, 1), (2, 1), (3, 1), (4, 2), (6, 3), (8, 1), (8, 5)])
def test_gate_level_equals_proposed(orc, n, m):
    """The conventional simulator (Algorithm 2) and the proposed one (Algorithm 5) reach the same state
    (Discussion: the two are mathematically equivalent)."""
    marks = workloads.distinct_marks(n, m, seed=55 * n + m)
    k = max(orc.optimal_iterations(n, m), 1) + 1
    a = orc.gate_search(n, marks, k)
    b = orc.search(n, marks, k)
    assert np.max(np.abs(a - b)) < 1e-13
    # and both equal the dense matrix power
    G = dense_diffusion(n) @ dense_oracle(n, marks)
    want = np.full(1 << n, 1 / math.sqrt(1 << n), dtype=np.complex128)
    for _ in range(k):
        want = G @ want
    assert np.max(np.abs(b - want)) < 1e-13


# ------------------------------------------------------------------------------------- invariants
def test_uniform_amplitude_correctly_rounded(orc):
    for n in range(0, 40):
        want = float(mpmath.mpf(2) ** (-mpmath.mpf(n) / 2))
        assert orc.uniform_amplitude(n) == want, n


@pytest.mark.parametrize("n", [1, 4, 9, 10])
def test_degenerate_marked_sets(orc, n):
    """M = 0: the uniform state is a fixed point (Eq. 2 maps the uniform vector to itself); bit for bit when
    n is even (the amplitude is a power of two, every partial sum exact), to rounding when n is odd.
    M = N: every iteration only flips the global sign."""
    N = 1 << n
    psi = orc.search(n, [], 7)
    if n % 2 == 0:
        assert np.array_equal(psi, orc.init_uniform(n))
    else:
        assert np.max(np.abs(psi - orc.init_uniform(n))) < 1e-15
    allm = np.arange(N, dtype=np.uint64)
    for k in range(4):
        psi = orc.search(n, allm, k)
        want = (-1) ** k * orc.init_uniform(n)
        if n % 2 == 0:
            assert np.array_equal(psi, want)
        else:
            assert np.max(np.abs(psi - want)) < 1e-15


@pytest.mark.parametrize("n,m", [(5, 1), (9, 3), (13, 2)])
def test_norm_is_one(orc, n, m):
    """Background, Quantum State: sum |c_i|^2 = 1, and the iteration is unitary."""
    marks = workloads.distinct_marks(n, m, seed=n)
    psi = orc.init_uniform(n)
    for _ in range(3):
        orc.iterate(psi, marks, 5)
        assert abs(orc.norm(psi) - 1.0) < 1e-13
    psi = workloads.random_state(n, seed=9)
    assert abs(orc.norm(orc.iterate(psi, marks, 11)) - 1.0) < 1e-13


def test_norm_matches_definition(orc):
    psi = workloads.random_state(7, seed=3) * 1.7
    assert abs(orc.norm(psi) - float(np.sum(np.abs(psi) ** 2))) < 1e-14
    assert orc.norm(np.zeros(8, dtype=np.complex128)) == 0.0


def test_exact_rational_recurrence(orc):
    """Exact dyadic arithmetic of the two-class iteration (Fractions) against the binary64 oracle at n = 10."""
    n, m, k = 10, 1, 25
    N = 1 << n
    A = B = Fraction(1)  # amplitudes scaled by sqrt(N)
    for _ in range(k):
        S = -m * A + (N - m) * B
        A, B = 2 * S / N + A, 2 * S / N - B
    psi = orc.search(n, [3], k)
    scale = 1 / math.sqrt(N)
    assert abs(psi[3].real - float(A) * scale) < 1e-15
    assert abs(psi[0].real - float(B) * scale) < 1e-15


# ------------------------------------------------------------------------------ storage precisions
def test_round_to_bits_binary32(orc):
    """p = 24 is IEEE binary32 round-to-nearest-even (numpy's float32 cast), including ties."""
    rng = np.random.default_rng(5)
    xs = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-30, 30, size=2000),
                         [1 + 2.0 ** -24, 1 + 3 * 2.0 ** -24, -(1 + 2.0 ** -24), 0.1, 1 / 3, 2.0 ** -126]])
    for x in xs:
        assert orc.round_to_bits(float(x), 24) == float(np.float32(x)), x
    assert orc.round_to_bits(0.1, 53) == 0.1


def test_round_to_bits_bfloat16_brute_force(orc):
    """p = 8 is bfloat16 round-to-nearest-even: the nearest of all finite positive bfloat16 values in the
    normal range, ties to the even bit pattern."""
    u = (np.arange(0x0080, 0x7F80, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)  # normals
    rng = np.random.default_rng(6)
    xs = np.concatenate([rng.uniform(1e-6, 1.0, 1500), rng.uniform(1.0, 1e6, 500),
                         (u[1000:1010] + u[1001:1011]) / 2])  # exact ties
    for x in xs:
        i = np.searchsorted(u, x)
        lo, hi = u[i - 1], u[i]
        if x - lo < hi - x or (x - lo == hi - x and (i - 1) % 2 == 0):
            want = lo
        else:
            want = hi
        if u[i] == x:
            want = x
        assert orc.round_to_bits(float(x), 8) == want, x
        assert orc.round_to_bits(-float(x), 8) == -want


@pytest.mark.parametrize("n,m,k", [(10, 1, 25), (20, 3, 464), (28, 8, 4549)])
def test_two_class_stored_at_53_bits_is_two_class(orc, n, m, k):
    assert orc.two_class_stored(n, m, k, 53) == orc.two_class(n, m, k)


def test_two_class_stored_binary32_matches_float32_full_state(orc):
    """At p = 24 the two-class form equals the full iteration with every stored amplitude cast to float32
    (numpy), at n = 12 where the full state is cheap; the two-class structure itself is exact."""
    n, m, k = 12, 2, 30
    marks = workloads.distinct_marks(n, m, seed=2)
    psi = np.full(1 << n, np.float64(np.float32(orc.uniform_amplitude(n))), dtype=np.complex128)
    mask = np.zeros(1 << n, dtype=bool)
    mask[marks.astype(np.int64)] = True
    for _ in range(k):
        orc.iterate(psi, marks, 1)
        psi = psi.real.astype(np.float32).astype(np.float64).astype(np.complex128)
    a, b = orc.two_class_stored(n, m, k, 24)
    assert np.all(psi[mask] == psi[mask][0]) and np.all(psi[~mask] == psi[~mask][0])
    assert abs(psi[mask][0].real - a) <= 2 * 2.0 ** -24 * abs(a)
    assert abs(psi[~mask][0].real - b) <= 2 * 2.0 ** -24 * abs(b)


# ------------------------------------------------- stored amplitudes, update in binary64 or in binary32
@pytest.mark.parametrize("n,m,k", [(7, 3, 5), (9, 1, 12)])
def test_iterate_stored_at_53_bits_is_the_iteration(orc, n, m, k):
    """Storage and update at 53 bits: the stored iteration is Algorithm 5's loop itself, bit for bit, on a
    random complex state (so the imaginary parts are exercised too)."""
    marks = workloads.distinct_marks(n, m, seed=n + 100)
    psi = workloads.random_state(n, seed=n + 200)
    a = orc.iterate(psi.copy(), marks, k)
    b = orc.iterate_stored(psi.copy(), marks, k, 53, 53)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


@pytest.mark.parametrize("p", [8, 24, 53])
def test_two_class_stored_update_at_53_bits(orc, p):
    """An update at 53 bits is the stored two-class iteration with a binary64 update."""
    for n, m, k in [(10, 1, 25), (16, 3, 100)]:
        assert orc.two_class_stored_update(n, m, k, p, 53) == orc.two_class_stored(n, m, k, p)


def float32_run(n: int, marks, k: int, update32: bool) -> np.ndarray:
    """numpy's own arithmetic: the uniform state 2^(-n/2) (even n: exact) stored as complex64; per iteration
    the marked amplitudes negated, the sum S of the stored values taken in binary64, and every amplitude
    replaced by 2S/N - c, either in binary64 and then cast to complex64, or in complex64 arithmetic from
    2S/N cast to complex64 (round to nearest even, each part)."""
    assert n % 2 == 0
    N = 1 << n
    idx = np.asarray(marks, dtype=np.int64)
    psi = np.full(N, np.complex64(2.0 ** (-n // 2)))
    for _ in range(k):
        psi[idx] = -psi[idx]
        mean2 = 2.0 * np.sum(psi.astype(np.complex128)) / N
        if update32:
            psi = np.complex64(mean2) - psi
        else:
            psi = (mean2 - psi.astype(np.complex128)).astype(np.complex64)
    return psi


@pytest.mark.parametrize("update32", [False, True])
@pytest.mark.parametrize("n,m,k", [(12, 2, 30), (10, 1, 25)])
def test_stored_iteration_matches_float32_arithmetic(orc, n, m, k, update32):
    """From the uniform state every stored value is a binary32 number and the state has two values, so
    every partial sum of any order (numpy's and the oracle's pairwise one) is an integer combination of the
    two that fits 53 bits: all sums are exact and the oracle must reproduce numpy's float32 run bit for bit,
    with the update in binary64 (p_update = 53) or in binary32 (p_update = 24); its two-class form too.  The
    two updates end at least one binary32 ulp apart, so the pin tells them apart."""
    N = 1 << n
    marks = workloads.distinct_marks(n, m, seed=3 * n + m)
    want = float32_run(n, marks, k, update32).astype(np.complex128)
    pu = 24 if update32 else 53
    got = orc.iterate_stored(np.full(N, 2.0 ** (-n // 2) + 0j), marks, k, 24, pu)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    a, b = orc.two_class_stored_update(n, m, k, 24, pu)
    mask = np.zeros(N, dtype=bool)
    mask[marks.astype(np.int64)] = True
    assert np.all(want[mask] == a) and np.all(want[~mask] == b)
    other = float32_run(n, marks, k, not update32).astype(np.complex128)
    assert np.max(np.abs(other - want)) >= 2.0 ** -24 * np.max(np.abs(want))


# ------------------------------------------------------------------------------------ random numbers
def test_splitmix64_published_vectors(orc):
    with open(os.path.join(GOLDEN, "splitmix64_vectors.txt")) as f:
        rows = [tuple(int(x) for x in line.split()) for line in f if line.strip() and not line.startswith("#")]
    assert rows
    for seed, j, out in rows:
        assert orc.splitmix64(seed, j) == out
        assert int(workloads.splitmix64(seed, 1, start=j)[0]) == out
    u = orc.uniforms_u53(1234567, 5)
    assert np.array_equal(u, workloads.uniforms_u53(1234567, 5))
    assert np.all(u < (1 << 53))


def test_hash_marks_brute_force(orc):
    """The hash predicate (low bits of SplitMix64_i(seed) all zero) against numpy enumeration."""
    n, seed, bits = 16, 0xDEADBEEF, 6
    h = workloads.splitmix64(seed, 1 << n)
    want = np.nonzero((h & np.uint64((1 << bits) - 1)) == 0)[0].astype(np.uint64)
    got, count = orc.hash_marks(n, seed, bits, cap=1 << 12)
    assert count == want.size and np.array_equal(got, want)
    _, c0 = orc.hash_marks(10, seed, 0, cap=0)
    assert c0 == 1 << 10  # zero-width test: every index is marked


def test_hash_workload_marks(orc):
    """The single-large-instance workload's seed gives exactly 8 marks over 2^28 (stored by make_golden.py)."""
    w = workloads.HASH_N28
    with open(os.path.join(GOLDEN, "hash_marks_n28.txt")) as f:
        stored = [int(x) for x in f if x.strip() and not x.startswith("#")]
    assert len(stored) == w.m
    # re-derive a subset cheaply: each stored index satisfies the predicate (numpy generator)
    for i in stored:
        assert int(workloads.splitmix64(w.hash_seed, 1, start=i)[0]) & ((1 << w.hash_bits) - 1) == 0


# --------------------------------------------------------------------------------------- measurement
@pytest.mark.parametrize("n", [2, 4, 8, 10])
def test_sample_uniform_state_closed_form(orc, n):
    """For the uniform state (even n) every p_i = 2^-n is exact, and inverse transform sampling reduces to
    index = floor(U N / 2^53) = U >> (53 - n)."""
    psi = orc.init_uniform(n)
    u = workloads.uniforms_u53(99, 20000)
    u = np.concatenate([u, np.array([0, (1 << 53) - 1, 1 << 52], dtype=np.uint64)])
    got = orc.sample(psi, u)
    assert np.array_equal(got, u >> np.uint64(53 - n))


@pytest.mark.parametrize("n", [1, 3, 5])
def test_sample_inverse_transform_on_a_grid(orc, n):
    """Inverse transform sampling: over a uniform grid of 2^20 U values the fraction of shots landing on
    index i equals p_i to within the grid spacing plus the 2^-62 quantisation (a single ordered sweep)."""
    psi = workloads.random_state(n, seed=40 + n)
    psi[1] = 0.0  # a zero-probability index is never selected
    psi /= np.sqrt(np.sum(np.abs(psi) ** 2))
    grid = np.arange(1 << 20, dtype=np.uint64) << np.uint64(33)
    got = orc.sample(psi, grid)
    assert np.all(np.diff(got.astype(np.int64)) >= 0)  # monotone in U
    counts = np.bincount(got.astype(np.int64), minlength=1 << n) / float(1 << 20)
    p = np.abs(psi) ** 2
    assert counts[1] == 0.0
    assert np.max(np.abs(counts - p)) <= 2.0 ** -20 + 1e-12


def test_sample_chi_square(orc):
    """10^6 shots from a random 32-state distribution pass a chi-square goodness-of-fit test."""
    import scipy.stats

    psi = workloads.random_state(5, seed=5)
    u = workloads.uniforms_u53(2024, 1_000_000)
    got = orc.sample(psi, u)
    obs = np.bincount(got.astype(np.int64), minlength=32)
    exp = np.abs(psi) ** 2 * u.size
    stat = float(np.sum((obs - exp) ** 2 / exp))
    assert scipy.stats.chi2.sf(stat, df=31) > 1e-4


def test_sample_point_mass(orc):
    psi = np.zeros(16, dtype=np.complex128)
    psi[11] = -1j
    got = orc.sample(psi, workloads.uniforms_u53(1, 1000))
    assert np.all(got == 11)
    with pytest.raises(ValueError):
        orc.sample(np.zeros(16, dtype=np.complex128), np.zeros(3, dtype=np.uint64))
