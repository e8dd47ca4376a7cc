// Shared between the batched kernel (k_batch.hip) and its host side (api_batch.hip).
#pragma once

#include "internal.h"

namespace grover {

constexpr int kBatchMaxPhases = 12;
constexpr int kBatchRegE = 8;                         // 16-byte vectors a thread holds in registers
constexpr int kBatchLdsE = 8;                         // ... and in its own slots of LDS (128 KiB per workgroup)
constexpr int kBatchHoldE = kBatchRegE + kBatchLdsE;  // 16 vectors = 32 complex64 amplitudes per thread

// One instance of a batch (device table, written by the host).
struct BatchInstance {
    uint64_t state_off;  // first 16-byte vector of the instance's state in the batch buffer
    uint64_t nvec;       // N / 2 (complex64: two amplitudes per vector)
    uint64_t marks_off;  // first entry of its sorted marked list in the concatenated marks
    uint64_t m;
    uint64_t iters;
    double N;
    double amp;  // 2^(-n/2) in binary64 (rounded to the storage type by the fill)
};

// A run is a sequence of phases.  Phase p has a queue of instances (ordered by decreasing work), a team
// size team[p] (workgroups per instance; non-increasing from one phase to the next, each a divisor of the
// previous one, so a team of phase p + 1 lies inside one team of phase p) and a mode: resident[p] > 0 holds
// each instance's state on chip in the team's workgroups (at most that many 16-byte vectors per thread, the
// first kBatchRegE in registers, the rest in LDS), 0 streams it from memory every iteration.  Team size 1 is
// one workgroup per instance (on chip when the state fits kBatchHoldE vectors per thread, else streamed).
struct BatchLaunch {
    void *state;
    const uint64_t *marks;
    const BatchInstance *inst;
    const uint32_t *queue;  // the phases' queues, concatenated
    uint64_t qoff[kBatchMaxPhases + 1];
    uint32_t team[kBatchMaxPhases];
    uint32_t resident[kBatchMaxPhases];
    uint32_t nphases;
    uint32_t probe;              // 1: one barrier of the whole grid, nothing else (residency check)
    uint32_t streams;            // 0: every state is held on chip (the kernel without the streamed paths)
    uint32_t update;             // grover_update of the element update
    unsigned long long *heads;   // one per phase
    GridSync *sync;              // [phase][grid]
    uint64_t *partials;          // [phase][grid * 8]: team slots [2][T][4]
    int grid;
    uint64_t timeout_ticks;
    hipStream_t stream;
};

// The persistent kernel with the streamed paths (streams = 1) or without them (0: every state on chip), with
// the update in binary32 (u32) or binary64.
const void *batch_kernel_fn(bool streams, bool u32);
hipError_t launch_batch(const BatchLaunch &L);

}  // namespace grover
