/*
 * Plain CPU FP64 oracle for "Fast simulation of Grover's quantum search on classical computer"
 * (Chattopadhyay and Menon, arXiv:2005.04635).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP library against the paper.  Only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark may load it.  The product library
 * never calls it, and the two share no source, header, table or helper.
 *
 * It is slow and literal on purpose: single thread, no blocking, no fusion, no reordering beyond what
 * the paper's algorithms state.  Every amplitude is IEEE binary64 and the file is compiled with
 * -ffp-contract=off, so no multiply-add is ever fused.
 *
 * State layout (Background, "Quantum State"): a linear array indexed by basis state,
 *   psi[2*i] = Re c_i, psi[2*i + 1] = Im c_i,  0 <= i < N = 2^n,
 * and bit q of the index i is qubit q (the bit arithmetic of Algorithm 1).
 *
 * Readings of the paper that the code relies on (each one pinned by a test under tests/):
 *   - loops run over every basis state, i < N (Algorithm 1 and Algorithm 4 print N-1);
 *   - Algorithm 4 acts on every amplitude of a dense array and divides by N = 2^n;
 *   - the mean is taken of the oracle-flipped state (the oracle runs first, G = (2|psi><psi| - I) O);
 *   - the number of iterations is floor(pi/4 * sqrt(N/M));
 *   - the conditional phase shift is 2|0><0| - I, so the gate-level and proposed paths agree in sign;
 *   - Algorithm 1 accumulates into a zeroed output array (out of place);
 *   - measurement is an inverse transform over an integer CDF (the paper gives no procedure).
 */
#include "grover_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* 1/sqrt(2) and pi/4, correctly rounded to binary64. */
static const double ORC_SQRT1_2 = 0.70710678118654752440084436210484903928483593768847;
static const double ORC_PI_4 = 0.78539816339744830961566084581987572104929234984378;

/* ------------------------------------------------------------------------------------------------ */
/* Counter-based SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output j of the generator seeded with
 * `seed` is mix64(seed + (j + 1) * gamma), gamma = 0x9E3779B97F4A7C15. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t j)
{
    uint64_t z = seed + (j + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Marked set defined by the hash predicate: i is marked when the low `bits` bits of
 * SplitMix64_i(seed) are all zero.  Enumerates every i < 2^n; writes the first `cap` hits in
 * increasing order and returns the total number of hits. */
uint64_t orc_hash_marks(uint32_t n, uint64_t seed, uint32_t bits, uint64_t *out, uint64_t cap)
{
    const uint64_t N = (uint64_t)1 << n;
    const uint64_t mask = bits >= 64 ? ~(uint64_t)0 : (((uint64_t)1 << bits) - 1u);
    uint64_t count = 0;
    for (uint64_t i = 0; i < N; ++i) {
        if ((orc_splitmix64(seed, i) & mask) == 0) {
            if (count < cap)
                out[count] = i;
            ++count;
        }
    }
    return count;
}

/* Number of Grover iterations, floor(pi/4 * sqrt(N/M)); 0 when nothing is marked.
 * (Proposed method, "Simulation of Grover's Search", with M solutions.) */
uint64_t orc_optimal_iterations(uint32_t n, uint64_t m)
{
    if (m == 0)
        return 0;
    return (uint64_t)floor(ORC_PI_4 * sqrt(ldexp(1.0, (int)n) / (double)m));
}

/* The amplitude of H^n|0>, 1/sqrt(N) = 2^(-n/2), correctly rounded:
 * exact for even n, sqrt(2) * 2^(-(n+1)/2) for odd n (sqrt is correctly rounded, the scaling exact). */
double orc_uniform_amplitude(uint32_t n)
{
    if (n % 2 == 0)
        return ldexp(1.0, -(int)(n / 2));
    return ldexp(sqrt(2.0), -(int)((n + 1) / 2));
}

/* psi = H^n |0>, written directly as the uniform superposition (proposed method's initial state). */
void orc_init_uniform(uint32_t n, double *psi)
{
    const uint64_t N = (uint64_t)1 << n;
    const double a = orc_uniform_amplitude(n);
    for (uint64_t i = 0; i < N; ++i) {
        psi[2 * i] = a;
        psi[2 * i + 1] = 0.0;
    }
}

/* Algorithm 3 (n-qubit Oracle): negate the amplitude of every solution state k[0..m-1]. */
void orc_oracle(double *psi, const uint64_t *k, uint64_t m)
{
    for (uint64_t i = 0; i < m; ++i) {
        psi[2 * k[i]] = -psi[2 * k[i]];
        psi[2 * k[i] + 1] = -psi[2 * k[i] + 1];
    }
}

/* Pairwise (cascade) summation of the real and imaginary parts over [lo, hi). */
static void pairwise_sum(const double *psi, uint64_t lo, uint64_t hi, double *re, double *im)
{
    if (hi - lo <= 8) {
        double r = 0.0, m = 0.0;
        for (uint64_t i = lo; i < hi; ++i) {
            r += psi[2 * i];
            m += psi[2 * i + 1];
        }
        *re = r;
        *im = m;
        return;
    }
    const uint64_t mid = lo + (hi - lo) / 2;
    double r0, m0, r1, m1;
    pairwise_sum(psi, lo, mid, &r0, &m0);
    pairwise_sum(psi, mid, hi, &r1, &m1);
    *re = r0 + r1;
    *im = m0 + m1;
}

/* Algorithm 4 (n-qubit Inversion about Mean), Eq. 2 applied to the whole state:
 * with s = sum_i c_i (real and imaginary parts separately, no conjugation),
 * c_i <- 2 s / N - c_i for every basis state. */
void orc_inversion_about_mean(uint32_t n, double *psi)
{
    const uint64_t N = (uint64_t)1 << n;
    double real_sum, imag_sum;
    pairwise_sum(psi, 0, N, &real_sum, &imag_sum);
    real_sum = (real_sum * 2.0) / ldexp(1.0, (int)n);
    imag_sum = (imag_sum * 2.0) / ldexp(1.0, (int)n);
    for (uint64_t i = 0; i < N; ++i) {
        psi[2 * i] = real_sum - psi[2 * i];
        psi[2 * i + 1] = imag_sum - psi[2 * i + 1];
    }
}

/* Algorithm 5 loop body, `iters` times: the oracle, then inversion about the mean. */
void orc_grover_iterate(uint32_t n, double *psi, const uint64_t *k, uint64_t m, uint64_t iters)
{
    for (uint64_t it = 0; it < iters; ++it) {
        orc_oracle(psi, k, m);
        orc_inversion_about_mean(n, psi);
    }
}

/* Algorithm 5 (proposed n-qubit Grover's search): uniform superposition, then `iters` iterations. */
void orc_grover_search(uint32_t n, const uint64_t *k, uint64_t m, uint64_t iters, double *psi)
{
    orc_init_uniform(n, psi);
    orc_grover_iterate(n, psi, k, m, iters);
}

/* Algorithm 1 (1-qubit unitary on target qubit q), Eq. 1:
 *   U|0> = a11|0> + a21|1>,  U|1> = a12|0> + a22|1>.
 * u = {Re a11, Im a11, Re a12, Im a12, Re a21, Im a21, Re a22, Im a22}.
 * Every basis state scatters its two contributions into a zeroed output, which then replaces psi.
 * Returns 0, or -1 when the scratch array cannot be allocated. */
int orc_unitary_1q(uint32_t n, double *psi, uint32_t q, const double u[8])
{
    const uint64_t N = (uint64_t)1 << n;
    double *out = (double *)calloc(2 * N, sizeof(double));
    if (!out)
        return -1;
    const uint64_t bit = (uint64_t)1 << q;
    for (uint64_t b = 0; b < N; ++b) {
        const double ar = psi[2 * b], ai = psi[2 * b + 1];
        const uint64_t zero = b & ~bit; /* the state with the target qubit |0> */
        const uint64_t one = b | bit;   /* the state with the target qubit |1> */
        double c1r, c1i, c2r, c2i;      /* coefficients of |0> and |1> in U|x_q> */
        if (!(b & bit)) {
            c1r = u[0]; c1i = u[1];     /* a11 */
            c2r = u[4]; c2i = u[5];     /* a21 */
        } else {
            c1r = u[2]; c1i = u[3];     /* a12 */
            c2r = u[6]; c2i = u[7];     /* a22 */
        }
        /* a1 = c1 * psi[b], a2 = c2 * psi[b] (complex products) */
        const double a1r = c1r * ar - c1i * ai, a1i = c1r * ai + c1i * ar;
        const double a2r = c2r * ar - c2i * ai, a2i = c2r * ai + c2i * ar;
        out[2 * zero] += a1r;
        out[2 * zero + 1] += a1i;
        out[2 * one] += a2r;
        out[2 * one + 1] += a2i;
    }
    memcpy(psi, out, 2 * N * sizeof(double));
    free(out);
    return 0;
}

/* H^(x)n as n applications of Algorithm 1 with U = H = (1/sqrt 2) [[1, 1], [1, -1]]. */
int orc_hadamard_all(uint32_t n, double *psi)
{
    const double h[8] = {ORC_SQRT1_2, 0.0, ORC_SQRT1_2, 0.0, ORC_SQRT1_2, 0.0, -ORC_SQRT1_2, 0.0};
    for (uint32_t q = 0; q < n; ++q)
        if (orc_unitary_1q(n, psi, q, h) != 0)
            return -1;
    return 0;
}

/* Conditional phase shift 2|0><0| - I (Background, step 4): |0> keeps its amplitude, every other basis
 * state is negated. */
void orc_conditional_phase_shift(uint32_t n, double *psi)
{
    const uint64_t N = (uint64_t)1 << n;
    for (uint64_t i = 1; i < N; ++i) {
        psi[2 * i] = -psi[2 * i];
        psi[2 * i + 1] = -psi[2 * i + 1];
    }
}

/* Algorithm 2 loop body (conventional simulator), `iters` times:
 * oracle, H^n, conditional phase shift, H^n. */
int orc_gate_iterate(uint32_t n, double *psi, const uint64_t *k, uint64_t m, uint64_t iters)
{
    for (uint64_t it = 0; it < iters; ++it) {
        orc_oracle(psi, k, m);
        if (orc_hadamard_all(n, psi) != 0)
            return -1;
        orc_conditional_phase_shift(n, psi);
        if (orc_hadamard_all(n, psi) != 0)
            return -1;
    }
    return 0;
}

/* Algorithm 2 (conventional n-qubit Grover's search): psi = |0>^n, H^n, then `iters` iterations. */
int orc_gate_search(uint32_t n, const uint64_t *k, uint64_t m, uint64_t iters, double *psi)
{
    const uint64_t N = (uint64_t)1 << n;
    memset(psi, 0, 2 * N * sizeof(double));
    psi[0] = 1.0;
    if (orc_hadamard_all(n, psi) != 0)
        return -1;
    return orc_gate_iterate(n, psi, k, m, iters);
}

/* Squared norm sum_i |c_i|^2 (Background, "Quantum State": it equals 1), pairwise summed. */
static double pairwise_norm(const double *psi, uint64_t lo, uint64_t hi)
{
    if (hi - lo <= 8) {
        double s = 0.0;
        for (uint64_t i = lo; i < hi; ++i)
            s += psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
        return s;
    }
    const uint64_t mid = lo + (hi - lo) / 2;
    return pairwise_norm(psi, lo, mid) + pairwise_norm(psi, mid, hi);
}

double orc_norm(uint32_t n, const double *psi)
{
    return pairwise_norm(psi, 0, (uint64_t)1 << n);
}

/* Two-class form of Algorithm 5 from the uniform state.  Starting from the uniform superposition every
 * marked amplitude stays equal to every other marked one (value a), and likewise every unmarked one
 * (value b), so one iteration is
 *   s = (N - M) b - M a        (sum of the oracle-flipped state),
 *   a <- 2 s / N + a,  b <- 2 s / N - b.
 * This is the same update as orc_grover_iterate restricted to that two-valued state, usable at any n. */
void orc_two_class(uint32_t n, uint64_t m, uint64_t iters, double *a_out, double *b_out)
{
    const double N = ldexp(1.0, (int)n);
    double a = orc_uniform_amplitude(n), b = a;
    for (uint64_t it = 0; it < iters; ++it) {
        const double s = (N - (double)m) * b - (double)m * a;
        const double mean2 = (s * 2.0) / N;
        a = mean2 + a;
        b = mean2 - b;
    }
    *a_out = a;
    *b_out = b;
}

/* x rounded to the nearest binary floating-point number with p significand bits, ties to even, exponent
 * unbounded (p = 53: binary64 itself; p = 24: binary32; p = 8: bfloat16, over their normal ranges). */
double orc_round_to_bits(double x, int p)
{
    if (x == 0.0 || !isfinite(x))
        return x;
    int e;
    const double m = frexp(x, &e); /* x = m 2^e, 0.5 <= |m| < 1 */
    const double r = nearbyint(ldexp(m, p)); /* default rounding mode: to nearest, ties to even */
    return ldexp(r, e - p);
}

/* The two-class form of the iteration with the amplitudes stored at p significand bits: the uniform
 * amplitude and every updated amplitude are rounded to p bits, the sum and the update are binary64.  This
 * is what a device that stores amplitudes in that precision and accumulates in binary64 computes when
 * started from the uniform superposition, up to the summation order of the sum. */
void orc_two_class_stored(uint32_t n, uint64_t m, uint64_t iters, int p, double *a_out, double *b_out)
{
    const double N = ldexp(1.0, (int)n);
    double a = orc_round_to_bits(orc_uniform_amplitude(n), p), b = a;
    for (uint64_t it = 0; it < iters; ++it) {
        const double s = (N - (double)m) * b - (double)m * a;
        const double mean2 = (s * 2.0) / N;
        a = orc_round_to_bits(mean2 + a, p);
        b = orc_round_to_bits(mean2 - b, p);
    }
    *a_out = a;
    *b_out = b;
}

/* Measurement (Background, step 6) by inverse transform over an integer CDF:
 *   p_i = Re^2 + Im^2 (binary64),  q_i = floor(p_i * 2^62),  Q_i = q_0 + ... + q_i,
 *   t_j = floor(U_j * Q_{N-1} / 2^53) for a 53-bit uniform integer U_j,
 *   shot j returns the smallest i with Q_i > t_j.
 * Returns 0, -1 when the CDF cannot be allocated, -2 when every probability rounds to zero. */
int orc_sample(uint32_t n, const double *psi, const uint64_t *u53, uint64_t shots, uint64_t *out)
{
    const uint64_t N = (uint64_t)1 << n;
    uint64_t *Q = (uint64_t *)malloc(N * sizeof(uint64_t));
    if (!Q)
        return -1;
    uint64_t acc = 0;
    for (uint64_t i = 0; i < N; ++i) {
        const double p = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
        acc += (uint64_t)(p * 0x1p62);
        Q[i] = acc;
    }
    const uint64_t total = Q[N - 1];
    if (total == 0) {
        free(Q);
        return -2;
    }
    for (uint64_t j = 0; j < shots; ++j) {
        const uint64_t t = (uint64_t)(((unsigned __int128)u53[j] * total) >> 53);
        uint64_t lo = 0, hi = N - 1;
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (Q[mid] > t)
                hi = mid;
            else
                lo = mid + 1;
        }
        out[j] = lo;
    }
    free(Q);
    return 0;
}

/* Uniforms from the oracle's own SplitMix64: U_j = SplitMix64_j(seed) >> 11. */
void orc_uniforms_u53(uint64_t seed, uint64_t shots, uint64_t *out)
{
    for (uint64_t j = 0; j < shots; ++j)
        out[j] = orc_splitmix64(seed, j) >> 11;
}
