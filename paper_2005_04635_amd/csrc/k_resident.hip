// On-chip iteration for small states (n <= 14): one workgroup of 1024 threads loads the whole state into
// registers once, runs all k iterations of Algorithm 5's loop body there (oracle sign, sum, update), and
// writes it back once.  The only synchronisation per iteration is the one workgroup barrier of the sum, so
// small searches (e.g. n = 10, 25 iterations) cost one launch instead of 2k passes over memory.
#include "internal.h"

namespace grover {
namespace {

constexpr int kBlock = kResidentBlock;

struct ResidentArgs {
    void *state;
    uint64_t nvec;
    double N;
    const uint64_t *marks;
    uint64_t m;
    uint64_t iters;
};

constexpr int kWaves = kBlock / kWave;

// Sum of (a, b) over the workgroup, left with the same bits in every thread: wave totals into the LDS slots
// of parity p, one workgroup barrier, then every thread adds the wave values in wave order.  A slot set is
// written again two calls later, after the next call's barrier, which every thread reaches only after its
// reads here, so one barrier per call suffices.
__device__ inline void workgroup_sum(double &a, double &b, double (*red)[2 * kWaves], int p)
{
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    a = wave_total(a);
    b = wave_total(b);
    if (lane == 0) {
        red[p][2 * wave] = a;
        red[p][2 * wave + 1] = b;
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        sa += red[p][2 * w];
        sb += red[p][2 * w + 1];
    }
    a = sa;
    b = sb;
}

// E = 16-byte vectors per thread; vector v = e * kBlock + threadIdx.x (coalesced load and store).  U32: the
// update in binary32 from 2S/N rounded to binary32 (complex64 only); otherwise binary64.
template <class T, int E, bool U32>
__global__ __launch_bounds__(kBlock) void resident_iterate_kernel(ResidentArgs a)
{
    using V = typename T::vec;
    __shared__ double red[2][2 * kWaves];
    V *st = static_cast<V *>(a.state);
    const unsigned tid = threadIdx.x;
    V x[E];
    unsigned bits[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint64_t v = uint64_t(e) * kBlock + tid;
        if (v < a.nvec) {
            x[e] = st[v];
            bits[e] = marked_bits<T::EPV>(a.marks, 0, a.m, v * T::EPV);
        } else {
            bits[e] = 0u;
        }
    }
    AccF64 acc0;
#pragma unroll
    for (int e = 0; e < E; ++e)
        if (uint64_t(e) * kBlock + tid < a.nvec)
            accum_vec<T>(x[e], bits[e], acc0);
    double sr = acc0.r, si = acc0.i;
    workgroup_sum(sr, si, red, 0);
    for (uint64_t it = 0; it < a.iters; ++it) {
        const double mr = (sr * 2.0) / a.N, mi = (si * 2.0) / a.N;
        AccF64 acc;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (uint64_t(e) * kBlock + tid < a.nvec) {
                if constexpr (U32)
                    update_vec_f32(x[e], float(mr), float(mi), bits[e], acc);
                else
                    update_vec<T>(x[e], mr, mi, bits[e], acc);
            }
        sr = acc.r;
        si = acc.i;
        workgroup_sum(sr, si, red, int((it + 1) & 1u));
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint64_t v = uint64_t(e) * kBlock + tid;
        if (v < a.nvec)
            st[v] = x[e];
    }
}

template <class T, bool U32 = false>
const void *pick(uint64_t vec_per_thread)
{
    switch (vec_per_thread) {
    case 1: return reinterpret_cast<const void *>(&resident_iterate_kernel<T, 1, U32>);
    case 2: return reinterpret_cast<const void *>(&resident_iterate_kernel<T, 2, U32>);
    case 4: return reinterpret_cast<const void *>(&resident_iterate_kernel<T, 4, U32>);
    case 8: return reinterpret_cast<const void *>(&resident_iterate_kernel<T, 8, U32>);
    case 16: return reinterpret_cast<const void *>(&resident_iterate_kernel<T, 16, U32>);
    default: return nullptr;
    }
}

}  // namespace

hipError_t launch_resident_iterate(grover_ctx *c, uint64_t k)
{
    ResidentArgs a;
    a.state = c->state;
    a.nvec = c->N / elems_per_vec(c->dtype);
    a.N = double(c->N);
    a.marks = c->marks_dev;
    a.m = c->marks.size();
    a.iters = k;
    uint64_t per = (a.nvec + kBlock - 1) / kBlock;
    uint64_t e = 1;
    while (e < per)
        e <<= 1;
    const void *fn = nullptr;
    switch (c->dtype) {
    case GROVER_F64_REAL: fn = pick<F64Real>(e); break;
    case GROVER_C64: fn = c->update == GROVER_UPDATE_F32 ? pick<C64, true>(e) : pick<C64>(e); break;
    case GROVER_C128: fn = pick<C128>(e); break;
    }
    if (!fn)
        return hipErrorInvalidValue;
    void *args[] = {&a};
    return hipLaunchKernel(fn, dim3(1), dim3(kBlock), args, 0, c->stream);
}

}  // namespace grover
