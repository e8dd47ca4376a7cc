// Batched searches in one persistent launch (many independent instances of Algorithm 5, complex64 states,
// binary64 sums, the update in binary64 or binary32).  The grid (one workgroup per CU, all co-resident) works through a sequence of
// phases, each with its own queue ordered by decreasing work N * k and its own team size T:
//   - in a phase with T > 1 the grid is split into teams of T consecutive workgroups; a team's leader takes
//     the next instance and publishes it through the team barrier, and the team iterates it with one team
//     barrier per iteration (which also reduces the sum).  The state is either held on chip by the team
//     for all iterations (resident phases: the instance fits T * 1024 threads * the phase's vectors per
//     thread, up to 8 in registers and 8 more in LDS) or streamed from memory every iteration, exactly as
//     the fused single-instance kernel does;
//   - in a phase with T = 1 every workgroup takes instances alone: held on chip (registers and LDS) when
//     the state fits (n <= 15), otherwise streamed with workgroup-level sums only.
// Team sizes do not increase from one phase to the next and each divides the previous one, so the members
// of a team always come from one team of the previous phase (they finish it together) and no grid-wide
// barrier is needed between phases.  Which phases exist and their parameters is the tiling the host
// chooses; each instance starts from the uniform superposition.
#include "batch.h"
#include "held.h"
#include "stream.h"

namespace grover {
namespace {

constexpr int kRegE = kHeldRegE;
constexpr int kLdsE = kHeldLdsE;
constexpr int kHoldE = kHeldHoldE;
static_assert(kHeldRegE == kBatchRegE && kHeldLdsE == kBatchLdsE, "the batch tiling assumes the held layout");

struct BatchArgs {
    float4 *state;
    const uint64_t *marks;
    const BatchInstance *inst;
    const uint32_t *queue;
    uint64_t qoff[kBatchMaxPhases + 1];
    uint32_t team[kBatchMaxPhases];
    uint32_t resident[kBatchMaxPhases];
    uint32_t nphases;
    uint32_t probe;
    unsigned long long *heads;
    GridSync *sync;
    uint64_t *partials;
    uint64_t timeout_ticks;
};

// Workgroup sum of (a, b) for every thread with one workgroup barrier: wave totals, then every thread adds
// the wave values by the same fixed tree (the same bits everywhere).  The wave values alternate between two
// buffers by `parity`: a buffer is rewritten two calls later, after the next call's barrier, which every
// thread reaches only after reading it.
__device__ inline void block_allsum(double &a, double &b, unsigned parity, TeamShared<double> &sh)
{
    const unsigned lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    double *red = sh.red[parity & 1u];
    a = wave_total(a);
    b = wave_total(b);
    if (lane == 0) {
        red[2 * wave] = a;
        red[2 * wave + 1] = b;
    }
    __syncthreads();
    add_wave_values(red, a, b);
}

// Sets an error word (the team's, which its members' barrier waits poll, or the workgroup's own), which
// the host reads after the run and reports as a failure.
__device__ inline void flag_error(GridSync *word)
{
    if (threadIdx.x == 0)
        __hip_atomic_store(&word->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline float4 uniform_vec(double amp)
{
    const float af = float(amp);
    return make_float4(af, 0.0f, af, 0.0f);
}

// One instance streamed by the T workgroups of a team.  Returns false when a barrier gave up.
template <bool U32>
__device__ bool run_team_streamed(const BatchArgs &a, const BatchInstance &I, const Team &tm, uint64_t &gen,
                                  TeamShared<double> &sh, uint32_t *table)
{
    const Share<C64> share{a.state + I.state_off, I.nvec, a.marks + I.marks_off, I.m, tm.rank, tm.size};
    const bool use_table = build_mark_table(share, table);
    AccF64 acc0;
    stream_pass<C64, AccF64, kFill>(share, table, use_table, 0.0, 0.0, uniform_vec(I.amp), acc0);
    double sr = acc0.r, si = acc0.i;
    if (!team_sum<double>(sr, si, tm, ++gen, sh))
        return false;
    const float4 none{};
    for (uint64_t it = 0; it < I.iters; ++it) {
        const double mr = (sr * 2.0) / I.N, mi = (si * 2.0) / I.N;
        AccF64 acc;
        stream_pass<C64, AccF64, kUpdate, U32>(share, table, use_table, mr, mi, none, acc);
        sr = acc.r;
        si = acc.i;
        if (!team_sum<double>(sr, si, tm, ++gen, sh))
            return false;
    }
    return true;
}

// One instance held on chip by a team for all its iterations: member `rank` owns the contiguous vectors
// [rank * per, (rank + 1) * per), per = nvec / T a power of two <= kHoldE * 1024, thread `tid` the vectors
// rank * per + e * 1024 + tid, e < ne = per / 1024 (or, when per < 1024, the one vector tid < per): the
// first kRegE in registers, the others in the thread's own slots of LDS (held[(e - kRegE) * 1024 + tid]; no
// other thread touches them, so no workgroup barrier is needed around them).  Marked bits travel packed, two
// per vector.  `reduce` is the team's (or the workgroup's) sum; the state is written to memory once, at
// the end.  Returns false when a barrier gave up.
template <bool U32, class Reduce>
__device__ bool run_held(const BatchArgs &a, const BatchInstance &I, uint64_t base, uint64_t per, float4 *held,
                         TeamShared<double> &sh, Reduce reduce)
{
    float4 *st = a.state + I.state_off + base;
    const uint64_t *marks = a.marks + I.marks_off;
    const unsigned tid = threadIdx.x;
    const unsigned ne = per >= kStreamBlock ? unsigned(per / kStreamBlock) : 1u;  // 1, 2, 4, 8 or 16
    const bool active = tid < per;
    const float4 fill = uniform_vec(I.amp);
    // 2/N is a power of two, so S * (2/N) rounds to the same binary64 value as 2S / N
    const double scale = 2.0 / I.N;
    uint32_t mask = 0u;
    AccF64 acc0;
    if (active) {
#pragma unroll 1
        for (unsigned e = 0; e < ne; ++e) {
            const uint64_t v = uint64_t(e) * kStreamBlock + tid;
            const unsigned bits = marked_bits<2>(marks, 0, I.m, (base + v) * 2u);
            mask |= uint32_t(bits) << (2 * e);
            accum_vec<C64>(fill, bits, acc0);
            if (e >= unsigned(kRegE))
                held[(e - kRegE) * kStreamBlock + tid] = fill;
        }
    }
    float4 x[kRegE];
#pragma unroll
    for (int e = 0; e < kRegE; ++e)
        x[e] = fill;
    double sr = acc0.r, si = acc0.i;
    if (!reduce(sr, si))
        return false;
    for (uint64_t it = 0; it < I.iters; ++it) {
        const double mr = sr * scale, mi = si * scale;
        AccF64 acc;
        if (active) {
            if (mask != 0u)
                negate_marked(x, held, mask);
            if constexpr (U32)
                held_sweep(x, held, ne, float(mr), float(mi), acc);
            else
                held_sweep(x, held, ne, mr, mi, acc);
            if (mask != 0u)
                correct_marked(x, held, mask, acc);
        }
        sr = acc.r;
        si = acc.i;
        if (!reduce(sr, si))
            return false;
    }
    if (active) {
#pragma unroll
        for (int e = 0; e < kHoldE; ++e)
            if (unsigned(e) < ne)
                st[uint64_t(e) * kStreamBlock + tid] = e < kRegE ? x[e] : held[(e - kRegE) * kStreamBlock + tid];
    }
    return true;
}

// One instance iterated by one workgroup, its state streamed from memory.
template <bool U32>
__device__ void run_single_streamed(const BatchArgs &a, const BatchInstance &I, TeamShared<double> &sh,
                                    uint32_t *table)
{
    const Share<C64> share{a.state + I.state_off, I.nvec, a.marks + I.marks_off, I.m, 0, 1};
    const bool use_table = build_mark_table(share, table);
    AccF64 acc0;
    stream_pass<C64, AccF64, kFill>(share, table, use_table, 0.0, 0.0, uniform_vec(I.amp), acc0);
    double sr = acc0.r, si = acc0.i;
    unsigned parity = 0;
    block_allsum(sr, si, parity++, sh);
    const float4 none{};
    for (uint64_t it = 0; it < I.iters; ++it) {
        const double mr = (sr * 2.0) / I.N, mi = (si * 2.0) / I.N;
        AccF64 acc;
        stream_pass<C64, AccF64, kUpdate, U32>(share, table, use_table, mr, mi, none, acc);
        sr = acc.r;
        si = acc.i;
        block_allsum(sr, si, parity++, sh);
    }
}

// kStreams = false compiles the kernel without the streamed paths, for tilings that hold every state on
// chip: the held loops then get the registers to themselves.  The host launches that instantiation only
// when no phase streams, so its streamed branches are never taken; were one taken, the kernel would report
// it through the error word instead of computing.  U32: the update in binary32 from 2S/N rounded to
// binary32; otherwise in binary64.
template <bool kStreams, bool U32>
__global__ __launch_bounds__(kStreamBlock) void batch_kernel(BatchArgs a)
{
    __shared__ TeamShared<double> sh;
    __shared__ uint32_t table[kMarkWords];
    __shared__ uint64_t taken;
    __shared__ float4 held[kLdsE * kStreamBlock];  // on-chip state beyond the registers (128 KiB)
    const uint32_t grid = gridDim.x;
    if (a.probe) {
        const Team tm{a.sync, a.partials, grid, blockIdx.x, a.timeout_ticks};
        double zr = 0.0, zi = 0.0;
        (void)team_sum<double>(zr, zi, tm, 1u, sh);
        return;
    }
    for (uint32_t p = 0; p < a.nphases; ++p) {
        const uint64_t q0 = a.qoff[p], count = a.qoff[p + 1] - q0;
        const unsigned T = a.team[p];
        const unsigned teams = grid / T, team_id = blockIdx.x / T;
        if (count == 0 || team_id >= teams)
            continue;
        if (T == 1) {
            for (;;) {
                if (threadIdx.x == 0)
                    taken = atomicAdd(&a.heads[p], 1ull);
                __syncthreads();
                // the index is the same in every lane; saying so keeps the instance's fields in scalar registers
                const uint64_t q = __builtin_amdgcn_readfirstlane(uint32_t(taken)) |
                                   (uint64_t(__builtin_amdgcn_readfirstlane(uint32_t(taken >> 32))) << 32);
                __syncthreads();
                if (q >= count)
                    break;
                const BatchInstance I = a.inst[a.queue[q0 + q]];
                unsigned parity = 0;
                if (I.nvec <= uint64_t(kHoldE) * kStreamBlock)
                    (void)run_held<U32>(a, I, 0, I.nvec, held, sh, [&](double &r, double &i) {
                        block_allsum(r, i, parity++, sh);
                        return true;
                    });
                else if (kStreams)
                    run_single_streamed<U32>(a, I, sh, table);
                else
                    flag_error(a.sync + uint64_t(p) * grid + blockIdx.x);
            }
            continue;
        }
        const Team tm{a.sync + uint64_t(p) * grid + team_id,
                      a.partials + uint64_t(p) * 8u * grid + uint64_t(team_id) * 8u * T, T, blockIdx.x % T,
                      a.timeout_ticks};
        uint64_t gen = 0;
        for (;;) {
            // the leader takes the next instance and contributes its index to a team sum (exact in binary64:
            // one integer below 2^53 plus zeros), which hands it to every member
            double zr = 0.0, zi = 0.0;
            if (tm.rank == 0 && threadIdx.x == 0)
                zr = double(atomicAdd(&a.heads[p], 1ull));
            if (!team_sum<double>(zr, zi, tm, ++gen, sh))
                return;
            const uint64_t qv = uint64_t(zr);  // the same in every lane (a team sum); made scalar below
            const uint64_t q = __builtin_amdgcn_readfirstlane(uint32_t(qv)) |
                               (uint64_t(__builtin_amdgcn_readfirstlane(uint32_t(qv >> 32))) << 32);
            if (q >= count)
                break;
            const BatchInstance I = a.inst[a.queue[q0 + q]];
            bool ok;
            if (a.resident[p]) {
                const uint64_t per = I.nvec / T;
                ok = run_held<U32>(a, I, uint64_t(tm.rank) * per, per, held, sh,
                                   [&](double &r, double &i) { return team_sum<double>(r, i, tm, ++gen, sh); });
            } else if (kStreams) {
                ok = run_team_streamed<U32>(a, I, tm, gen, sh, table);
            } else {
                flag_error(tm.sync);
                ok = false;
            }
            if (!ok)
                return;
        }
    }
}

// Zeroes the phase heads, the team barriers and the member slots (whose generation tags the barriers
// compare against) before a run — a kernel, not a memset, so that the pair of launches can be captured into
// a graph and replayed.
__global__ void batch_reset_kernel(unsigned long long *heads, uint64_t nheads, uint64_t *sync_words, uint64_t nwords,
                                   uint64_t *slots, uint64_t nslots)
{
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    if (i < nheads)
        heads[i] = 0ull;
    for (uint64_t w = i; w < nwords; w += stride)
        sync_words[w] = 0u;
    for (uint64_t w = i; w < nslots; w += stride)
        slots[w] = 0u;
}

}  // namespace

const void *batch_kernel_fn(bool streams, bool u32)
{
    if (u32)
        return streams ? reinterpret_cast<const void *>(&batch_kernel<true, true>)
                       : reinterpret_cast<const void *>(&batch_kernel<false, true>);
    return streams ? reinterpret_cast<const void *>(&batch_kernel<true, false>)
                   : reinterpret_cast<const void *>(&batch_kernel<false, false>);
}

hipError_t launch_batch(const BatchLaunch &L)
{
    BatchArgs a;
    a.state = static_cast<float4 *>(L.state);
    a.marks = L.marks;
    a.inst = L.inst;
    a.queue = L.queue;
    for (int p = 0; p <= kBatchMaxPhases; ++p)
        a.qoff[p] = L.qoff[p];
    for (int p = 0; p < kBatchMaxPhases; ++p) {
        a.team[p] = L.team[p];
        a.resident[p] = L.resident[p];
    }
    a.nphases = L.nphases;
    a.probe = L.probe;
    a.heads = L.heads;
    a.sync = L.sync;
    a.partials = L.partials;
    a.timeout_ticks = L.timeout_ticks;
    unsigned long long *heads = L.heads;
    uint64_t nheads = kBatchMaxPhases;
    uint64_t *words = reinterpret_cast<uint64_t *>(L.sync);
    uint64_t nwords = uint64_t(kBatchMaxPhases) * uint64_t(L.grid) * sizeof(GridSync) / sizeof(uint64_t);
    uint64_t *slots = L.partials;
    uint64_t nslots = uint64_t(kBatchMaxPhases) * uint64_t(L.grid) * 8u;
    void *ra[] = {&heads, &nheads, &words, &nwords, &slots, &nslots};
    hipError_t e = hipLaunchKernel(reinterpret_cast<const void *>(&batch_reset_kernel), dim3(256), dim3(256), ra, 0,
                                   L.stream);
    if (e != hipSuccess)
        return e;
    void *args[] = {&a};
    return hipLaunchCooperativeKernel(batch_kernel_fn(L.streams != 0u, L.update != 0u), dim3(L.grid),
                                      dim3(kStreamBlock), args, 0, L.stream);
}

}  // namespace grover
