// Shared between the generalized-iteration kernels (k_phase.hip) and their host side (api_phase.hip).
#pragma once

#include "internal.h"

namespace grover {

// Barrier words of one team of the phase kernels: as GridSync, with room for eight reduced values.
struct PhaseSync {
    uint64_t flag;
    uint32_t error;
    uint32_t pad0[61];
    uint32_t arrive0;
    uint32_t pad1[63];
    uint32_t arrive1;
    uint32_t pad2[63];
    uint64_t sum[2][8];  // bit patterns of binary64 values
    uint64_t pad3[16];
};
static_assert(sizeof(PhaseSync) == 1024, "barrier words on separate lines");

struct PhaseLaunch {
    void *state, *lambda, *ckpt;
    const uint64_t *marks;
    uint64_t m;
    uint64_t nvec;
    double N;
    float amp;
    uint32_t B, K, every, nck;
    const double *phi, *theta;
    double *loss, *aux;
    const double *dloss;
    double *dphi, *dtheta;
    PhaseSync *sync;
    uint64_t *partials;
    uint32_t team_size;
    uint32_t teams_alloc;  // barrier objects zeroed before the launch
    uint32_t probe;
    uint32_t held;  // 1: the on-chip kernels (team_size set from the state size)
    int grid;
    uint64_t timeout_ticks;
    hipStream_t stream;
};

// Largest state (vectors) the on-chip kernels hold per thread: forward 16 vectors, adjoint 8 of the state
// and 8 of the adjoint state.
constexpr uint64_t kPhaseHeldForwardVecs = 16 * 1024;
constexpr uint64_t kPhaseHeldAdjointVecs = 8 * 1024;

const void *phase_kernel_fn(bool adjoint, bool held);
hipError_t launch_phase(const PhaseLaunch &L, bool adjoint);

}  // namespace grover
