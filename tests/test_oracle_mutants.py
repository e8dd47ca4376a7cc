"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible slip in a temporary copy of the oracle's C source, builds that copy with
gcc and runs the pin battery of tests/test_oracle_pins.py against it; at least one pin must fail. The
committed oracle is never modified.
"""
from __future__ import annotations

import os
import shutil

import pytest

import oracle
import test_oracle_phase as phase
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "grover_oracle.c")

# (name, original text, planted text): every original must occur exactly once in the source.
MUTANTS = [
    ("update loop skips the last index",
     "for (uint64_t i = 0; i < N; ++i) {\n        psi[2 * i] = real_sum - psi[2 * i];",
     "for (uint64_t i = 0; i < N - 1; ++i) {\n        psi[2 * i] = real_sum - psi[2 * i];"),
    ("mean divided by N/2", "real_sum = (real_sum * 2.0) / ldexp(1.0, (int)n);",
     "real_sum = (real_sum * 2.0) / ldexp(1.0, (int)n - 1);"),
    ("factor two dropped", "real_sum = (real_sum * 2.0) /", "real_sum = (real_sum * 1.0) /"),
    ("inversion sign swapped", "psi[2 * i] = real_sum - psi[2 * i];", "psi[2 * i] = psi[2 * i] - real_sum;"),
    ("imaginary mean conjugated", "m += psi[2 * i + 1];", "m -= psi[2 * i + 1];"),
    ("imaginary mean dropped", "psi[2 * i + 1] = imag_sum - psi[2 * i + 1];",
     "psi[2 * i + 1] = -psi[2 * i + 1];"),
    ("oracle flips only the real part", "        psi[2 * k[i] + 1] = -psi[2 * k[i] + 1];\n", "\n"),
    ("oracle applied after the mean",
     "        orc_oracle(psi, k, m);\n        orc_inversion_about_mean(n, psi);",
     "        orc_inversion_about_mean(n, psi);\n        orc_oracle(psi, k, m);"),
    ("pairwise leaf skips an element", "for (uint64_t i = lo; i < hi; ++i) {\n            r += psi[2 * i];",
     "for (uint64_t i = lo + 1; i < hi; ++i) {\n            r += psi[2 * i];"),
    ("unitary a12/a21 transposed", "c1r = u[2]; c1i = u[3];     /* a12 */", "c1r = u[4]; c1i = u[5];     /* a12 */"),
    ("unitary imaginary cross term sign", "const double a1r = c1r * ar - c1i * ai", "const double a1r = c1r * ar + c1i * ai"),
    ("unitary targets the mirrored qubit", "const uint64_t bit = (uint64_t)1 << q;",
     "const uint64_t bit = (uint64_t)1 << (n - 1 - q);"),
    ("hadamard sign on the wrong entry",
     "ORC_SQRT1_2, 0.0, ORC_SQRT1_2, 0.0, ORC_SQRT1_2, 0.0, -ORC_SQRT1_2, 0.0};",
     "ORC_SQRT1_2, 0.0, -ORC_SQRT1_2, 0.0, ORC_SQRT1_2, 0.0, ORC_SQRT1_2, 0.0};"),
    ("phase shift also negates |0>", "for (uint64_t i = 1; i < N; ++i) {\n        psi[2 * i] = -psi[2 * i];",
     "for (uint64_t i = 0; i < N; ++i) {\n        psi[2 * i] = -psi[2 * i];"),
    ("iteration count rounded up", "return (uint64_t)floor(ORC_PI_4", "return (uint64_t)ceil(ORC_PI_4"),
    ("uniform amplitude off by a factor", "return ldexp(1.0, -(int)(n / 2));", "return ldexp(1.0, -(int)(n / 2) - 1);"),
    ("odd-n amplitude rounded twice", "return ldexp(sqrt(2.0), -(int)((n + 1) / 2));",
     "return 1.0 / sqrt(ldexp(1.0, (int)n));"),
    ("two-class sum sign",
     "double a = orc_uniform_amplitude(n), b = a;\n    for (uint64_t it = 0; it < iters; ++it) {\n"
     "        const double s = (N - (double)m) * b - (double)m * a;",
     "double a = orc_uniform_amplitude(n), b = a;\n    for (uint64_t it = 0; it < iters; ++it) {\n"
     "        const double s = (N - (double)m) * b + (double)m * a;"),
    ("norm drops the imaginary part",
     "s += psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];", "s += psi[2 * i] * psi[2 * i];"),
    ("sampler probability drops the imaginary part",
     "const double p = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];",
     "const double p = psi[2 * i] * psi[2 * i];"),
    ("sampler search uses >=", "if (Q[mid] > t)", "if (Q[mid] >= t)"),
    ("sampler target scaled by 2", "* total) >> 53);", "* total) >> 52);"),
    ("sampler exclusive CDF", "acc += (uint64_t)(p * 0x1p62);\n        Q[i] = acc;",
     "Q[i] = acc;\n        acc += (uint64_t)(p * 0x1p62);"),
    ("splitmix shift changed", "z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;", "z = (z ^ (z >> 31)) * 0xBF58476D1CE4E5B9ull;"),
    ("splitmix counter off by one", "uint64_t z = seed + (j + 1u) *", "uint64_t z = seed + j *"),
    ("hash mask one bit short", "(((uint64_t)1 << bits) - 1u)", "(((uint64_t)1 << (bits - 1)) - 1u)"),
    ("round_to_bits keeps one bit fewer", "const double r = nearbyint(ldexp(m, p));",
     "const double r = nearbyint(ldexp(m, p - 1));"),
    ("round_to_bits truncates", "const double r = nearbyint(ldexp(m, p));", "const double r = trunc(ldexp(m, p));"),
    ("stored two-class skips rounding b", "b = orc_round_to_bits(mean2 - b, p);", "b = mean2 - b;"),
    ("two-class update model keeps the mean in binary64",
     "const double mean2 = orc_round_to_bits((s * 2.0) / N, p_update);", "const double mean2 = (s * 2.0) / N;"),
    ("stored update keeps the mean in binary64",
     "const double mr = orc_round_to_bits((re * 2.0) / ldexp(1.0, (int)n), p_update);",
     "const double mr = (re * 2.0) / ldexp(1.0, (int)n);"),
    ("stored update never rounds to the storage",
     "psi[2 * i] = orc_round_to_bits(orc_round_to_bits(mr - psi[2 * i], p_update), p_store);",
     "psi[2 * i] = orc_round_to_bits(mr - psi[2 * i], p_update);"),
    ("stored iteration skips the oracle", "        orc_oracle(psi, k, m);\n        double re, im;",
     "        double re, im;"),
    ("stored update conjugates the mean", "orc_round_to_bits(mi - psi[2 * i + 1], p_update)",
     "orc_round_to_bits(-mi - psi[2 * i + 1], p_update)"),
    ("phase diffusion conjugates its phase", "const orc_c e = c_expi(theta);", "const orc_c e = c_expi(-theta);"),
    ("phase oracle conjugates its phase", "const orc_c e = c_expi(phi);", "const orc_c e = c_expi(-phi);"),
    ("phase diffusion mean over N/2", "const orc_c mean = {re / ldexp(1.0, (int)n), im / ldexp(1.0, (int)n)};\n    const orc_c e",
     "const orc_c mean = {re / ldexp(1.0, (int)n - 1), im / ldexp(1.0, (int)n)};\n    const orc_c e"),
    ("adjoint theta gradient sign", "dtheta[jj] = 2.0 * g.re;", "dtheta[jj] = -2.0 * g.re;"),
    ("adjoint forgets to undo the oracle", "orc_phase_oracle(lam, k, m, -phi[jj]);", "orc_phase_oracle(lam, k, m, phi[jj]);"),
    ("adjoint applies D instead of its inverse", "orc_phase_diffusion(n, lam, -theta[jj]);",
     "orc_phase_diffusion(n, lam, theta[jj]);"),
    ("adjoint phi gradient takes the real product", "s += t.re;", "s += t.im;"),
    ("tangent theta term conjugated", "t[2 * i + 1] += g.im;", "t[2 * i + 1] -= g.im;"),
    ("tangent phi term skips the diffusion", "        orc_phase_diffusion(n, w, theta[j]);\n", "\n"),
    ("loss derivative sign", "return -2.0 * s;", "return 2.0 * s;"),
    ("phase loss drops the imaginary part",
     "p += psi[2 * k[q]] * psi[2 * k[q]] + psi[2 * k[q] + 1] * psi[2 * k[q] + 1];",
     "p += psi[2 * k[q]] * psi[2 * k[q]];"),
    ("hash marks listed from index 1", "for (uint64_t i = 0; i < N; ++i) {\n        if ((orc_splitmix64",
     "for (uint64_t i = 1; i < N; ++i) {\n        if ((orc_splitmix64"),
]


def battery(orc) -> None:
    """The pin tests, each at a few representative parameters. Raises on the first failing pin."""
    pins.test_fig2_worked_example(orc)
    pins.test_fig2_pins_iteration_count(orc)
    pins.test_iteration_counts_of_the_workloads(orc)
    for n, m in [(5, 2), (9, 5)]:
        pins.test_closed_form(orc, n, m)
    pins.test_two_class_closed_form_large(orc, 20, 3, 464)
    pins.test_two_class_equals_full_state(orc, 9, 3)
    for n, m, k in [(3, 2, 4), (5, 3, 7)]:
        pins.test_dense_eq2_on_general_states(orc, n, m, k)
    pins.test_oracle_and_mean_separately(orc, 3)
    pins.test_hadamard_all_is_walsh_hadamard(orc, 3)
    for n, q in [(2, 0), (4, 1)]:
        pins.test_unitary_1q_matches_kronecker(orc, n, q)
    pins.test_conditional_phase_shift_gives_eq2(orc, 3)
    pins.test_gate_level_equals_proposed(orc, 4, 2)
    pins.test_uniform_amplitude_correctly_rounded(orc)
    pins.test_degenerate_marked_sets(orc, 4)
    pins.test_norm_is_one(orc, 5, 1)
    pins.test_norm_matches_definition(orc)
    pins.test_splitmix64_published_vectors(orc)
    pins.test_hash_marks_brute_force(orc)
    pins.test_sample_uniform_state_closed_form(orc, 4)
    pins.test_sample_inverse_transform_on_a_grid(orc, 3)
    pins.test_sample_point_mass(orc)
    pins.test_round_to_bits_binary32(orc)
    pins.test_round_to_bits_bfloat16_brute_force(orc)
    pins.test_two_class_stored_at_53_bits_is_two_class(orc, 10, 1, 25)
    pins.test_two_class_stored_binary32_matches_float32_full_state(orc)
    pins.test_iterate_stored_at_53_bits_is_the_iteration(orc, 7, 3, 5)
    pins.test_two_class_stored_update_at_53_bits(orc, 24)
    for update32 in (False, True):
        pins.test_stored_iteration_matches_float32_arithmetic(orc, 12, 2, 30, update32)
    phase.test_phases_at_pi_are_the_standard_iteration(orc)
    phase.test_fig2_through_the_generalized_iteration(orc)
    phase.test_dense_matrices_and_torch_autograd(orc, 5, [1, 30], 5, 2)
    phase.test_two_amplitude_reduction_in_50_digits(orc)
    phase.test_inverses_and_unitarity(orc)
    phase.test_tangent_and_adjoint_agree(orc)


def test_battery_passes_on_the_committed_oracle(orc):
    battery(orc)


@pytest.mark.parametrize("name,orig,planted", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_slip(tmp_path, name, orig, planted):
    text = open(SRC).read()
    assert text.count(orig) == 1, f"mutation anchor not unique: {name}"
    src = tmp_path / "grover_oracle.c"
    src.write_text(text.replace(orig, planted))
    shutil.copy(os.path.join(os.path.dirname(SRC), "grover_oracle.h"), tmp_path / "grover_oracle.h")
    lib = oracle.load(oracle.build(src=str(src), out=str(tmp_path / "liboracle_mutant.so")))
    with pytest.raises((AssertionError, ValueError, MemoryError)):
        battery(oracle.Oracle(lib))
