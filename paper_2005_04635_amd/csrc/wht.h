// Blocked Walsh-Hadamard transform of the gate-level path (k_wht.hip), used by api.hip.
#pragma once

#include "internal.h"

namespace grover {

// H^n with the normalisation 2^(-n/2), in ceil((n - L) / H) + 1 LDS-blocked passes.
hipError_t launch_hadamard_all_blocked(grover_ctx *c);
// H^n (2|0><0| - I) H^n as two unnormalised transforms: the phase shift fused into the first one's last
// pass, the exact scale 2^(-n) into the second one's.
hipError_t launch_gate_diffusion_blocked(grover_ctx *c);

}  // namespace grover
