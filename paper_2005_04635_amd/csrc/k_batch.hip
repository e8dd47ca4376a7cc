// Batched searches in one persistent launch (many independent instances of Algorithm 5, complex64 states,
// binary64 sums).  The grid (one workgroup per CU, all co-resident) works through two queues, each ordered
// by decreasing work N * k:
//   1. team queue: the grid is split into teams of T consecutive workgroups; a team takes one instance at a
//      time and iterates it exactly as the fused single-instance kernel does, with a team barrier per
//      iteration (T = grid size is grid-per-instance);
//   2. single queue: once the team queue is empty, every workgroup takes instances alone — held in
//      registers for the whole run when the state fits (n <= 14), otherwise streamed with workgroup-level
//      sums only (workgroup-per-instance).
// Which instances go to the team queue (n >= split) and T are the tiling the host's autotuner chooses.
// Each instance starts from the uniform superposition, written by the instance's own first pass.
#include "stream.h"

namespace grover {
namespace {

constexpr int kResE = 8;  // 16-byte vectors per thread for a register-held state: N <= 2 * 8 * 1024

struct BatchArgs {
    float4 *state;
    const uint64_t *marks;
    const BatchInstance *inst;
    const uint32_t *queue_team;
    uint64_t n_team;
    const uint32_t *queue_single;
    uint64_t n_single;
    unsigned long long *heads;  // [0] next team-queue entry, [1] next single-queue entry
    GridSync *team_sync;        // one per team
    uint64_t *team_partials;    // [teams][2][T][2]
    uint64_t *team_mail;        // one 256-byte line per team: the instance its leader took
    uint32_t team_size;
    uint64_t timeout_ticks;
};

__device__ inline void block_allsum(double &a, double &b, TeamShared<double> &sh)
{
    block_sum2(a, b, sh.red);
    if (threadIdx.x == 0) {
        sh.sum[0] = a;
        sh.sum[1] = b;
    }
    __syncthreads();
    a = sh.sum[0];
    b = sh.sum[1];
    __syncthreads();
}

__device__ inline float4 uniform_vec(double amp)
{
    const float af = float(amp);
    return make_float4(af, 0.0f, af, 0.0f);
}

// One instance iterated by the T workgroups of a team.  Returns false when a barrier gave up.
__device__ bool run_team_instance(const BatchArgs &a, const BatchInstance &I, const Team &tm, uint64_t &gen,
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
        stream_pass<C64, AccF64, kUpdate>(share, table, use_table, mr, mi, none, acc);
        sr = acc.r;
        si = acc.i;
        if (!team_sum<double>(sr, si, tm, ++gen, sh))
            return false;
    }
    return true;
}

// One instance iterated by one workgroup, its state streamed from memory.
__device__ void run_single_streamed(const BatchArgs &a, const BatchInstance &I, TeamShared<double> &sh,
                                    uint32_t *table)
{
    const Share<C64> share{a.state + I.state_off, I.nvec, a.marks + I.marks_off, I.m, 0, 1};
    const bool use_table = build_mark_table(share, table);
    AccF64 acc0;
    stream_pass<C64, AccF64, kFill>(share, table, use_table, 0.0, 0.0, uniform_vec(I.amp), acc0);
    double sr = acc0.r, si = acc0.i;
    block_allsum(sr, si, sh);
    const float4 none{};
    for (uint64_t it = 0; it < I.iters; ++it) {
        const double mr = (sr * 2.0) / I.N, mi = (si * 2.0) / I.N;
        AccF64 acc;
        stream_pass<C64, AccF64, kUpdate>(share, table, use_table, mr, mi, none, acc);
        sr = acc.r;
        si = acc.i;
        block_allsum(sr, si, sh);
    }
}

// One instance held in the registers of one workgroup for all its iterations (vector v = e * block + tid).
__device__ void run_single_resident(const BatchArgs &a, const BatchInstance &I, TeamShared<double> &sh)
{
    float4 *st = a.state + I.state_off;
    const uint64_t *marks = a.marks + I.marks_off;
    const unsigned tid = threadIdx.x;
    float4 x[kResE];
    unsigned bits[kResE];
    const float4 fill = uniform_vec(I.amp);
    AccF64 acc0;
#pragma unroll
    for (int e = 0; e < kResE; ++e) {
        const uint64_t v = uint64_t(e) * kStreamBlock + tid;
        bits[e] = 0u;
        if (v < I.nvec) {
            x[e] = fill;
            bits[e] = marked_bits<2>(marks, 0, I.m, v * 2u);
            accum_vec<C64>(x[e], bits[e], acc0);
        }
    }
    double sr = acc0.r, si = acc0.i;
    block_allsum(sr, si, sh);
    for (uint64_t it = 0; it < I.iters; ++it) {
        const double mr = (sr * 2.0) / I.N, mi = (si * 2.0) / I.N;
        AccF64 acc;
#pragma unroll
        for (int e = 0; e < kResE; ++e)
            if (uint64_t(e) * kStreamBlock + tid < I.nvec)
                update_vec<C64>(x[e], mr, mi, bits[e], acc);
        sr = acc.r;
        si = acc.i;
        block_allsum(sr, si, sh);
    }
#pragma unroll
    for (int e = 0; e < kResE; ++e) {
        const uint64_t v = uint64_t(e) * kStreamBlock + tid;
        if (v < I.nvec)
            st[v] = x[e];
    }
}

__global__ __launch_bounds__(kStreamBlock) void batch_kernel(BatchArgs a)
{
    __shared__ TeamShared<double> sh;
    __shared__ uint32_t table[kMarkWords];
    __shared__ uint64_t taken;
    // 1. team queue
    const unsigned T = a.team_size;
    const unsigned teams = T > 1 ? gridDim.x / T : 0u;
    const unsigned team_id = blockIdx.x / (T > 0 ? T : 1u);
    if (team_id < teams) {
        const Team tm{a.team_sync + team_id, a.team_partials + uint64_t(team_id) * 4u * T, T, blockIdx.x % T,
                      a.timeout_ticks};
        uint64_t *mail = a.team_mail + uint64_t(team_id) * 32u;
        uint64_t gen = 0;
        for (;;) {
            // the leader takes the next instance; the barrier that follows publishes it to the team
            if (tm.rank == 0 && threadIdx.x == 0)
                __hip_atomic_store(mail, uint64_t(atomicAdd(&a.heads[0], 1ull)), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            double zr = 0.0, zi = 0.0;
            if (!team_sum<double>(zr, zi, tm, ++gen, sh))
                return;
            if (threadIdx.x == 0)
                taken = __hip_atomic_load(mail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            const uint64_t q = taken;
            __syncthreads();
            if (q >= a.n_team)
                break;
            if (!run_team_instance(a, a.inst[a.queue_team[q]], tm, gen, sh, table))
                return;
        }
    }
    // 2. single queue
    for (;;) {
        if (threadIdx.x == 0)
            taken = atomicAdd(&a.heads[1], 1ull);
        __syncthreads();
        const uint64_t q = taken;
        __syncthreads();
        if (q >= a.n_single)
            break;
        const BatchInstance I = a.inst[a.queue_single[q]];
        if (I.nvec <= uint64_t(kResE) * kStreamBlock)
            run_single_resident(a, I, sh);
        else
            run_single_streamed(a, I, sh, table);
    }
}

// Zeroes the queue heads and the team barriers before a run (a kernel, not a memset, so that the pair of
// launches can be captured into a graph and replayed).
__global__ void batch_reset_kernel(unsigned long long *heads, uint64_t *sync_words, uint64_t nwords)
{
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < 2)
        heads[i] = 0ull;
    for (uint64_t w = i; w < nwords; w += uint64_t(gridDim.x) * blockDim.x)
        sync_words[w] = 0u;
}

}  // namespace

const void *batch_kernel_fn() { return reinterpret_cast<const void *>(&batch_kernel); }

hipError_t launch_batch(const BatchLaunch &L)
{
    BatchArgs a;
    a.state = static_cast<float4 *>(L.state);
    a.marks = L.marks;
    a.inst = L.inst;
    a.queue_team = L.queue_team;
    a.n_team = L.n_team;
    a.queue_single = L.queue_single;
    a.n_single = L.n_single;
    a.heads = L.heads;
    a.team_sync = L.team_sync;
    a.team_partials = L.team_partials;
    a.team_mail = L.team_mail;
    a.team_size = L.team_size;
    a.timeout_ticks = L.timeout_ticks;
    unsigned long long *heads = L.heads;
    uint64_t *words = reinterpret_cast<uint64_t *>(L.team_sync);
    uint64_t nwords = uint64_t(L.teams_alloc) * sizeof(GridSync) / sizeof(uint64_t);
    void *ra[] = {&heads, &words, &nwords};
    hipError_t e = hipLaunchKernel(reinterpret_cast<const void *>(&batch_reset_kernel), dim3(64), dim3(256), ra, 0,
                                   L.stream);
    if (e != hipSuccess)
        return e;
    void *args[] = {&a};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&batch_kernel), dim3(L.grid),
                                      dim3(kStreamBlock), args, 0, L.stream);
}

}  // namespace grover
