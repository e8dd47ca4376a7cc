/*
 * Plain CPU FP64 oracle for arXiv:2005.04635 — TEST INFRASTRUCTURE ONLY (see grover_oracle.c).
 * This header belongs to the oracle alone; the HIP library neither includes it nor links it.
 */
#ifndef GROVER_ORACLE_H
#define GROVER_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

uint64_t orc_splitmix64(uint64_t seed, uint64_t j);
uint64_t orc_hash_marks(uint32_t n, uint64_t seed, uint32_t bits, uint64_t *out, uint64_t cap);
uint64_t orc_optimal_iterations(uint32_t n, uint64_t m);
double orc_uniform_amplitude(uint32_t n);
void orc_init_uniform(uint32_t n, double *psi);
void orc_oracle(double *psi, const uint64_t *k, uint64_t m);
void orc_inversion_about_mean(uint32_t n, double *psi);
void orc_grover_iterate(uint32_t n, double *psi, const uint64_t *k, uint64_t m, uint64_t iters);
void orc_grover_search(uint32_t n, const uint64_t *k, uint64_t m, uint64_t iters, double *psi);
int orc_unitary_1q(uint32_t n, double *psi, uint32_t q, const double u[8]);
int orc_hadamard_all(uint32_t n, double *psi);
void orc_conditional_phase_shift(uint32_t n, double *psi);
int orc_gate_iterate(uint32_t n, double *psi, const uint64_t *k, uint64_t m, uint64_t iters);
int orc_gate_search(uint32_t n, const uint64_t *k, uint64_t m, uint64_t iters, double *psi);
double orc_norm(uint32_t n, const double *psi);
void orc_two_class(uint32_t n, uint64_t m, uint64_t iters, double *a_out, double *b_out);
double orc_round_to_bits(double x, int p);
void orc_two_class_stored(uint32_t n, uint64_t m, uint64_t iters, int p, double *a_out, double *b_out);
void orc_two_class_stored_update(uint32_t n, uint64_t m, uint64_t iters, int p_store, int p_update, double *a_out,
                                 double *b_out);
void orc_grover_iterate_stored(uint32_t n, double *psi, const uint64_t *k, uint64_t m, uint64_t iters, int p_store,
                               int p_update);
int orc_sample(uint32_t n, const double *psi, const uint64_t *u53, uint64_t shots, uint64_t *out);
void orc_uniforms_u53(uint64_t seed, uint64_t shots, uint64_t *out);
void orc_phase_oracle(double *psi, const uint64_t *k, uint64_t m, double phi);
void orc_phase_diffusion(uint32_t n, double *psi, double theta);
void orc_phase_search(uint32_t n, const uint64_t *k, uint64_t m, uint64_t K, const double *phi,
                      const double *theta, double *psi);
double orc_phase_loss(const double *psi, const uint64_t *k, uint64_t m);
int orc_phase_grad_tangent(uint32_t n, const uint64_t *k, uint64_t m, uint64_t K, const double *phi,
                           const double *theta, double *dphi, double *dtheta);
int orc_phase_grad_adjoint(uint32_t n, const uint64_t *k, uint64_t m, uint64_t K, const double *phi,
                           const double *theta, double *dphi, double *dtheta);

#ifdef __cplusplus
}
#endif

#endif
