// Single-state held form of grover_iterate (complex64 storage, binary64 sums): the state stays on chip for
// all k iterations of one call (Algorithm 5's loop of Algorithm 3's oracle sign and Eq. 2 / Algorithm 4's
// inversion about the mean), held by a team of T workgroups (T a power of two, one launch of exactly T
// workgroups).  Member `rank` owns the vectors [rank * per, (rank + 1) * per), per = nvec / T; thread tid
// the vectors rank * per + e * 1024 + tid, e < ne = per / 1024 (or the one vector tid < per when per <
// 1024), the first 8 in registers and the rest in its LDS slots.  The launch loads the state, forms the
// oracle-signed sum of it in the order the iterations add theirs (so consecutive calls compose bit for bit),
// runs k iterations with one team barrier each, and stores the state back.  Where the state is small
// enough (nvec / T <= 8 vectors per thread for T <= 64) only registers are used.
#include "held.h"

namespace grover {
namespace {

struct HeldIterArgs {
    float4 *state;
    const uint64_t *marks;
    uint64_t m;
    uint64_t nvec;
    uint64_t iters;
    double scale;  // 2 / N, a power of two: S * scale rounds as 2S / N
    GridSync *sync;
    uint64_t *partials;  // team slots [2][T][4]
    uint64_t gen0;
    uint64_t timeout_ticks;
    uint32_t probe;  // 1: one team barrier only (residency check)
};

// kTogether: a lane of the team barrier waits for its 2 to 4 member slots together (teams of more than 64
// workgroups; n = 21 and 22: 5.29 vs 5.84 ms and 8.59 vs 9.58 ms per optimal search on MI355X).  Teams of
// at most 64 use the kernel without it, whose code keeps fewer registers in flight (with it n = 18 took
// 1.61 instead of 1.43 ms).
// U32: the update in binary32 from 2S/N rounded to binary32; otherwise in binary64.
template <bool kTogether, bool U32>
__global__ __launch_bounds__(kStreamBlock) void held_iterate_kernel(HeldIterArgs a)
{
    __shared__ TeamShared<double> sh;
    __shared__ float4 held[kHeldLdsE * kStreamBlock];
    const Team tm{a.sync, a.partials, gridDim.x, blockIdx.x, a.timeout_ticks};
    uint64_t gen = a.gen0;
    if (a.probe) {
        double zr = 0.0, zi = 0.0;
        (void)team_sum<double, kTogether>(zr, zi, tm, ++gen, sh);
        return;
    }
    const unsigned tid = threadIdx.x;
    const uint64_t per = a.nvec / gridDim.x, base = uint64_t(blockIdx.x) * per;
    const unsigned ne = per >= kStreamBlock ? unsigned(per / kStreamBlock) : 1u;
    const bool active = tid < per;
    float4 *st = a.state + base;
    float4 x[kHeldRegE];
    uint32_t mask = 0u;
    AccF64 acc0;
    if (active) {
#pragma unroll 1
        for (unsigned e = 0; e < ne; ++e) {
            const uint64_t v = uint64_t(e) * kStreamBlock + tid;
            mask |= uint32_t(marked_bits<2>(a.marks, 0, a.m, (base + v) * 2u)) << (2 * e);
        }
#pragma unroll
        for (int e = 0; e < kHeldRegE; ++e)
            if (unsigned(e) < ne)
                x[e] = st[uint64_t(e) * kStreamBlock + tid];
        if (ne > unsigned(kHeldRegE))
#pragma unroll
            for (int e = 0; e < kHeldLdsE; ++e)
                held[e * kStreamBlock + tid] = st[uint64_t(kHeldRegE + e) * kStreamBlock + tid];
        held_accumulate(x, held, ne, acc0);
        if (mask != 0u)
            correct_marked(x, held, mask, acc0);
    }
    double sr = acc0.r, si = acc0.i;
    if (!team_sum<double, kTogether>(sr, si, tm, ++gen, sh))
        return;
    for (uint64_t it = 0; it < a.iters; ++it) {
        const double mr = sr * a.scale, mi = si * a.scale;
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
        if (!team_sum<double, kTogether>(sr, si, tm, ++gen, sh))
            return;
    }
    if (active) {
#pragma unroll
        for (int e = 0; e < kHeldRegE; ++e)
            if (unsigned(e) < ne)
                st[uint64_t(e) * kStreamBlock + tid] = x[e];
        if (ne > unsigned(kHeldRegE))
#pragma unroll
            for (int e = 0; e < kHeldLdsE; ++e)
                st[uint64_t(kHeldRegE + e) * kStreamBlock + tid] = held[e * kStreamBlock + tid];
    }
}

}  // namespace

// Team size of the held form for a complex64 state of nvec vectors on a device whose largest power-of-two
// team is max_team; 0 when the state does not fit.  While a team of at most 128 workgroups can hold the state
// in registers (8 vectors per thread), the state is spread over the team that gives each thread about two
// vectors, up to 64 workgroups (never fewer than the registers need): the update's VALU work per iteration
// shrinks, while the team barrier costs about the same up to 64 members.  Larger states take 16 vectors per
// thread, 8 of them in LDS.  One optimal search on MI355X, chosen team against the fewest workgroups that
// hold the state in registers: n = 14 4 vs 1 workgroup 0.264 vs 0.330 ms, n = 15 8 vs 2 0.413 vs 0.496 ms,
// n = 17 32 vs 8 0.984 vs 1.008 ms, n = 18 64 vs 16 1.436 vs 1.572 ms, n = 19 64 vs 32 2.188 vs 2.361 ms,
// n = 21 128 with 8 per thread vs 64 with 16 5.81 vs 5.93 ms (n = 16: 16 vs 4 0.650 vs 0.692 ms, where 64
// took 0.619 ms and 32 0.671 ms).
uint32_t held_team_size(uint64_t nvec, uint32_t max_team)
{
    auto pow2 = [](uint64_t x) {
        uint64_t t = 1;
        while (t < x)
            t <<= 1;
        return t;
    };
    const uint64_t t8 = pow2((nvec + uint64_t(kHeldRegE) * kStreamBlock - 1) / (uint64_t(kHeldRegE) * kStreamBlock));
    if (t8 <= 128 && t8 <= max_team) {
        uint64_t t2 = pow2((nvec + 2u * kStreamBlock - 1) / (2u * kStreamBlock));  // about two vectors per thread
        if (t2 > 64)
            t2 = 64;
        if (t2 > max_team)
            t2 = max_team;
        return uint32_t(t8 > t2 ? t8 : t2);
    }
    const uint64_t t16 = pow2((nvec + uint64_t(kHeldHoldE) * kStreamBlock - 1) / (uint64_t(kHeldHoldE) * kStreamBlock));
    return t16 <= max_team ? uint32_t(t16) : 0u;
}

hipError_t launch_held_iterate(grover_ctx *c, uint64_t k, uint64_t timeout_ticks, bool probe)
{
    HeldIterArgs a;
    a.state = static_cast<float4 *>(c->state);
    a.marks = c->marks_dev;
    a.m = c->marks.size();
    a.nvec = c->N / 2;
    a.iters = k;
    a.scale = 2.0 / double(c->N);
    a.sync = c->sync;
    a.partials = c->partials;
    a.gen0 = c->generation;
    a.timeout_ticks = timeout_ticks;
    a.probe = probe ? 1u : 0u;
    void *args[] = {&a};
    const bool u32 = c->update == GROVER_UPDATE_F32;
    const void *fn = c->held_team > 64u
                         ? (u32 ? reinterpret_cast<const void *>(&held_iterate_kernel<true, true>)
                                : reinterpret_cast<const void *>(&held_iterate_kernel<true, false>))
                         : (u32 ? reinterpret_cast<const void *>(&held_iterate_kernel<false, true>)
                                : reinterpret_cast<const void *>(&held_iterate_kernel<false, false>));
    const hipError_t e = hipLaunchCooperativeKernel(fn, dim3(c->held_team), dim3(kStreamBlock), args, 0, c->stream);
    if (e == hipSuccess)
        c->generation += probe ? 1u : k + 1u;
    return e;
}

}  // namespace grover
