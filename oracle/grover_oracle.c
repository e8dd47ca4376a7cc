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

/* The two-class form with a reduced-precision update as well as reduced-precision storage: the new
 * amplitude is computed at p_update significand bits from 2s/N rounded to p_update bits, then stored at
 * p_store bits,
 *   mean2 = fl_u(2 s / N),  a <- fl_s(fl_u(mean2 + a)),  b <- fl_s(fl_u(mean2 - b)),
 * with s = (N - M) b - M a in binary64.  p_update = 53 is orc_two_class_stored (the update in binary64);
 * p_update = 24 is an update in binary32: the exact difference of two binary32 values rounded to binary64
 * and then to binary32 equals its single rounding to binary32, since 53 >= 2 * 24 + 2. */
void orc_two_class_stored_update(uint32_t n, uint64_t m, uint64_t iters, int p_store, int p_update, double *a_out,
                                 double *b_out)
{
    const double N = ldexp(1.0, (int)n);
    double a = orc_round_to_bits(orc_uniform_amplitude(n), p_store), b = a;
    for (uint64_t it = 0; it < iters; ++it) {
        const double s = (N - (double)m) * b - (double)m * a;
        const double mean2 = orc_round_to_bits((s * 2.0) / N, p_update);
        a = orc_round_to_bits(orc_round_to_bits(mean2 + a, p_update), p_store);
        b = orc_round_to_bits(orc_round_to_bits(mean2 - b, p_update), p_store);
    }
    *a_out = a;
    *b_out = b;
}

/* Algorithm 5's loop body on a state whose amplitudes are stored at p_store significand bits, with the
 * second loop of Algorithm 4 computed at p_update bits: the oracle (Algorithm 3; a negation is exact), the
 * sum of the first loop in binary64 (pairwise), then for every basis state
 *   c_i <- fl_s(fl_u(fl_u(2 s / N) - c_i))
 * for the real and the imaginary part.  With p_store = p_update = 53 this is orc_grover_iterate; p_update
 * = 53 is an update in binary64 rounded once to the storage, p_update = 24 an update in binary32.  psi
 * must hold values representable at p_store bits (the state as stored). */
void orc_grover_iterate_stored(uint32_t n, double *psi, const uint64_t *k, uint64_t m, uint64_t iters, int p_store,
                               int p_update)
{
    const uint64_t N = (uint64_t)1 << n;
    for (uint64_t it = 0; it < iters; ++it) {
        orc_oracle(psi, k, m);
        double re, im;
        pairwise_sum(psi, 0, N, &re, &im);
        const double mr = orc_round_to_bits((re * 2.0) / ldexp(1.0, (int)n), p_update);
        const double mi = orc_round_to_bits((im * 2.0) / ldexp(1.0, (int)n), p_update);
        for (uint64_t i = 0; i < N; ++i) {
            psi[2 * i] = orc_round_to_bits(orc_round_to_bits(mr - psi[2 * i], p_update), p_store);
            psi[2 * i + 1] = orc_round_to_bits(orc_round_to_bits(mi - psi[2 * i + 1], p_update), p_store);
        }
    }
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

/* ------------------------------------------------------------------------------------------------ */
/* Generalized iteration with per-iteration phases.  The paper fixes both phases at pi (the oracle of
 * Algorithm 3 negates, Eq. 2 inverts about the mean); this is the usual phase-matched generalization, a
 * convention of this project:
 *   O(phi):   c_i <- e^{i phi} c_i for every marked i;
 *   D(theta): c <- ((1 - e^{i theta}) |psi><psi| - I) c with |psi> the uniform superposition, i.e.
 *             c_i <- (1 - e^{i theta}) * mean(c) - c_i with mean(c) = (sum_j c_j) / N.
 * At phi = theta = pi these are Algorithm 3 and Eq. 2.  Iteration j applies D(theta_j) O(phi_j), from the
 * uniform superposition, for j = 1 .. K.  The loss is L = 1 - sum over marked i of |c_i|^2. */

typedef struct {
    double re, im;
} orc_c;

static orc_c c_mul(orc_c a, orc_c b)
{
    orc_c r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}

static orc_c c_expi(double x)
{
    orc_c r = {cos(x), sin(x)};
    return r;
}

static orc_c c_at(const double *psi, uint64_t i)
{
    orc_c r = {psi[2 * i], psi[2 * i + 1]};
    return r;
}

static void c_put(double *psi, uint64_t i, orc_c v)
{
    psi[2 * i] = v.re;
    psi[2 * i + 1] = v.im;
}

void orc_phase_oracle(double *psi, const uint64_t *k, uint64_t m, double phi)
{
    const orc_c e = c_expi(phi);
    for (uint64_t q = 0; q < m; ++q)
        c_put(psi, k[q], c_mul(e, c_at(psi, k[q])));
}

void orc_phase_diffusion(uint32_t n, double *psi, double theta)
{
    const uint64_t N = (uint64_t)1 << n;
    double re, im;
    pairwise_sum(psi, 0, N, &re, &im);
    const orc_c mean = {re / ldexp(1.0, (int)n), im / ldexp(1.0, (int)n)};
    const orc_c e = c_expi(theta);
    const orc_c one_minus_e = {1.0 - e.re, -e.im};
    const orc_c f = c_mul(one_minus_e, mean);
    for (uint64_t i = 0; i < N; ++i) {
        psi[2 * i] = f.re - psi[2 * i];
        psi[2 * i + 1] = f.im - psi[2 * i + 1];
    }
}

void orc_phase_search(uint32_t n, const uint64_t *k, uint64_t m, uint64_t K, const double *phi,
                      const double *theta, double *psi)
{
    orc_init_uniform(n, psi);
    for (uint64_t j = 0; j < K; ++j) {
        orc_phase_oracle(psi, k, m, phi[j]);
        orc_phase_diffusion(n, psi, theta[j]);
    }
}

double orc_phase_loss(const double *psi, const uint64_t *k, uint64_t m)
{
    double p = 0.0;
    for (uint64_t q = 0; q < m; ++q)
        p += psi[2 * k[q]] * psi[2 * k[q]] + psi[2 * k[q] + 1] * psi[2 * k[q] + 1];
    return 1.0 - p;
}

/* dL/dp = -2 Re sum over marked i of conj(c_i) t_i, t = dc/dp at the end of the run. */
static double loss_derivative(const double *psi, const double *t, const uint64_t *k, uint64_t m)
{
    double s = 0.0;
    for (uint64_t q = 0; q < m; ++q)
        s += psi[2 * k[q]] * t[2 * k[q]] + psi[2 * k[q] + 1] * t[2 * k[q] + 1];
    return -2.0 * s;
}

/* Gradient of the loss by forward-mode differentiation: for each parameter p the tangent t = dc/dp is
 * carried beside c.  Iteration j maps (c, t) to (D O c, D O t + dD/dp O c + D dO/dp c), where the only
 * nonzero parameter derivatives are, for p = phi_j, dO/dphi = i e^{i phi} on the marked entries, and for
 * p = theta_j, dD/dtheta c = -i e^{i theta} mean(c) 1 (D is affine in |psi><psi|).  Both operators are
 * linear, so the tangent obeys the same step.  Cost O(K^2 N); returns -1 when memory is short. */
int orc_phase_grad_tangent(uint32_t n, const uint64_t *k, uint64_t m, uint64_t K, const double *phi,
                           const double *theta, double *dphi, double *dtheta)
{
    const uint64_t N = (uint64_t)1 << n;
    double *c = malloc(2 * N * sizeof(double)), *t = malloc(2 * N * sizeof(double));
    double *w = malloc(2 * N * sizeof(double));
    if (!c || !t || !w) {
        free(c);
        free(t);
        free(w);
        return -1;
    }
    for (uint64_t p = 0; p < 2 * K; ++p) {
        const uint64_t jp = p % K;     /* iteration the parameter belongs to */
        const int is_theta = p >= K;   /* parameters 0..K-1 are phi, K..2K-1 theta */
        orc_init_uniform(n, c);
        memset(t, 0, 2 * N * sizeof(double));
        for (uint64_t j = 0; j < K; ++j) {
            if (j != jp) {
                orc_phase_oracle(c, k, m, phi[j]);
                orc_phase_diffusion(n, c, theta[j]);
                orc_phase_oracle(t, k, m, phi[j]);
                orc_phase_diffusion(n, t, theta[j]);
                continue;
            }
            if (!is_theta) {
                /* d/dphi of D O c = D (i e^{i phi} P_M c): w = i e^{i phi} c on marked, 0 elsewhere */
                memset(w, 0, 2 * N * sizeof(double));
                const orc_c ie = c_mul((orc_c){0.0, 1.0}, c_expi(phi[j]));
                for (uint64_t q = 0; q < m; ++q)
                    c_put(w, k[q], c_mul(ie, c_at(c, k[q])));
                /* D applied to w: D w = (1 - e^{i theta}) mean(w) - w */
                orc_phase_diffusion(n, w, theta[j]);
                orc_phase_oracle(t, k, m, phi[j]);
                orc_phase_diffusion(n, t, theta[j]);
                for (uint64_t i = 0; i < 2 * N; ++i)
                    t[i] += w[i];
                orc_phase_oracle(c, k, m, phi[j]);
                orc_phase_diffusion(n, c, theta[j]);
            } else {
                /* d/dtheta of D y with y = O c: -i e^{i theta} mean(y) in every entry */
                orc_phase_oracle(c, k, m, phi[j]);
                double re, im;
                pairwise_sum(c, 0, N, &re, &im);
                const orc_c mean = {re / ldexp(1.0, (int)n), im / ldexp(1.0, (int)n)};
                const orc_c g = c_mul(c_mul((orc_c){0.0, -1.0}, c_expi(theta[j])), mean);
                orc_phase_diffusion(n, c, theta[j]);
                orc_phase_oracle(t, k, m, phi[j]);
                orc_phase_diffusion(n, t, theta[j]);
                for (uint64_t i = 0; i < N; ++i) {
                    t[2 * i] += g.re;
                    t[2 * i + 1] += g.im;
                }
            }
        }
        (is_theta ? dtheta : dphi)[jp] = loss_derivative(c, t, k, m);
    }
    free(c);
    free(t);
    free(w);
    return 0;
}

/* Gradient of the loss by reverse-mode differentiation with every intermediate state stored (memory
 * (K + 1) N complex values).  With lambda = dL/d(conj c) (lambda = -c on the marked entries after the last
 * iteration, 0 elsewhere) and y_j = O(phi_j) c_{j-1}:
 *   dL/dtheta_j = 2 Re( conj(sum lambda_j) * (-i e^{i theta_j}) * mean(y_j) ),
 *   nu_j = D(theta_j)^H lambda_j,   dL/dphi_j = 2 Re( sum over marked of conj(nu_j) * i * y_j ),
 *   lambda_{j-1} = O(phi_j)^H nu_j,
 * where D^H = D(-theta) and O^H = O(-phi).  Returns -1 when memory is short. */
int orc_phase_grad_adjoint(uint32_t n, const uint64_t *k, uint64_t m, uint64_t K, const double *phi,
                           const double *theta, double *dphi, double *dtheta)
{
    const uint64_t N = (uint64_t)1 << n;
    double *states = malloc((K + 1) * 2 * N * sizeof(double));
    double *lam = malloc(2 * N * sizeof(double)), *y = malloc(2 * N * sizeof(double));
    if (!states || !lam || !y) {
        free(states);
        free(lam);
        free(y);
        return -1;
    }
    orc_init_uniform(n, states);
    for (uint64_t j = 0; j < K; ++j) {
        double *next = states + (j + 1) * 2 * N;
        memcpy(next, states + j * 2 * N, 2 * N * sizeof(double));
        orc_phase_oracle(next, k, m, phi[j]);
        orc_phase_diffusion(n, next, theta[j]);
    }
    memset(lam, 0, 2 * N * sizeof(double));
    const double *last = states + K * 2 * N;
    for (uint64_t q = 0; q < m; ++q)
        c_put(lam, k[q], (orc_c){-last[2 * k[q]], -last[2 * k[q] + 1]});
    for (uint64_t jj = K; jj-- > 0;) {
        memcpy(y, states + jj * 2 * N, 2 * N * sizeof(double));
        orc_phase_oracle(y, k, m, phi[jj]);
        double yr, yi, lr, li;
        pairwise_sum(y, 0, N, &yr, &yi);
        pairwise_sum(lam, 0, N, &lr, &li);
        const orc_c mean_y = {yr / ldexp(1.0, (int)n), yi / ldexp(1.0, (int)n)};
        const orc_c conj_sum_lam = {lr, -li};
        const orc_c g = c_mul(c_mul(conj_sum_lam, c_mul((orc_c){0.0, -1.0}, c_expi(theta[jj]))), mean_y);
        dtheta[jj] = 2.0 * g.re;
        orc_phase_diffusion(n, lam, -theta[jj]); /* nu = D(-theta) lambda */
        double s = 0.0;
        for (uint64_t q = 0; q < m; ++q) {
            const orc_c nu = c_at(lam, k[q]);
            const orc_c conj_nu = {nu.re, -nu.im};
            const orc_c t = c_mul(conj_nu, c_mul((orc_c){0.0, 1.0}, c_at(y, k[q])));
            s += t.re;
        }
        dphi[jj] = 2.0 * s;
        orc_phase_oracle(lam, k, m, -phi[jj]); /* lambda_{j-1} = O(-phi) nu */
    }
    free(states);
    free(lam);
    free(y);
    return 0;
}
