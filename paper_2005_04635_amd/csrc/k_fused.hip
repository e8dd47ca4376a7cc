// Fused persistent iteration (proposed method, Algorithms 3-5 of arXiv:2005.04635).
//
// One cooperative launch runs k Grover iterations.  Each workgroup owns a fixed set of tiles of the state
// for the whole launch (so every amplitude stays with one workgroup, hence one XCD and its L2), and each
// iteration is a single streaming pass over it:
//
//   read c_i, flip the sign of marked amplitudes (Algorithm 3), write c_i' = 2S/N - s_i c_i (Algorithm 4's
//   second loop), and add s_i c_i' into an accumulator — which is Algorithm 4's first loop for the NEXT
//   iteration, already applied to the next iteration's oracle-flipped state.
//
// The per-workgroup accumulators then meet at a grid barrier: every workgroup publishes its partial, the
// last one to arrive adds all partials in workgroup order (so the sum is reproducible run to run) and
// releases the others with the new S.  One read and one write of the state per iteration is the minimum:
// S depends on every amplitude, so no amplitude can be updated twice before all have been read once.
//
// A prologue pass computes S of the incoming state with the same per-thread order as the fused
// accumulation, which makes iterate(a); iterate(b) equal iterate(a + b) bit for bit.
//
// Template parameters: T = storage type (F64Real, C64, C128, CBF16), A = accumulator of the sum (AccF64,
// AccF32, AccF32Kahan; the grid tree runs in A's precision).  The update itself is always binary64.  The
// streaming pass and the barrier are shared with the batched kernel (stream.h); here the whole grid is
// one team.
#include "stream.h"

namespace grover {
namespace {

struct FusedArgs {
    void *state;
    uint64_t nvec;  // N / EPV
    double N;
    const uint64_t *marks;
    uint64_t m;
    uint64_t *partials;  // [2][grid][2] binary64 bit patterns
    GridSync *sync;
    uint64_t iters;
    uint64_t gen0;
    uint64_t timeout_ticks;
};

// CHECK only names a second, code-identical instantiation used for the residency check at context
// creation, so that profiles list it apart from the iteration launches.
template <class T, class A, bool CHECK>
__global__ __launch_bounds__(kStreamBlock) void fused_iterate_kernel(FusedArgs a)
{
    using Val = typename A::value;
    __shared__ TeamShared<Val> sh;
    __shared__ uint32_t table[kMarkWords];
    const Team team{a.sync, a.partials, gridDim.x, blockIdx.x, a.timeout_ticks};
    const Share<T> share{static_cast<typename T::vec *>(a.state), a.nvec, a.marks, a.m, blockIdx.x, gridDim.x};
    const bool use_table = build_mark_table(share, table);
    const typename T::vec none{};
    A acc0;
    stream_pass<T, A, kAccumulate>(share, table, use_table, 0.0, 0.0, none, acc0);
    Val sr = acc0.res_r(), si = acc0.res_i();
    if (!team_sum<Val>(sr, si, team, a.gen0 + 1u, sh))
        return;
    for (uint64_t it = 0; it < a.iters; ++it) {
        const double mr = (double(sr) * 2.0) / a.N, mi = (double(si) * 2.0) / a.N;
        A acc;
        stream_pass<T, A, kUpdate>(share, table, use_table, mr, mi, none, acc);
        sr = acc.res_r();
        si = acc.res_i();
        if (!team_sum<Val>(sr, si, team, a.gen0 + 2u + it, sh))
            return;
    }
}

template <class A, bool CHECK>
const void *pick_storage(uint32_t dtype)
{
    switch (dtype) {
    case GROVER_F64_REAL: return reinterpret_cast<const void *>(&fused_iterate_kernel<F64Real, A, CHECK>);
    case GROVER_C64: return reinterpret_cast<const void *>(&fused_iterate_kernel<C64, A, CHECK>);
    case GROVER_C128: return reinterpret_cast<const void *>(&fused_iterate_kernel<C128, A, CHECK>);
    case GROVER_CBF16: return reinterpret_cast<const void *>(&fused_iterate_kernel<CBF16, A, CHECK>);
    default: return nullptr;
    }
}

template <bool CHECK>
const void *kernel_for(uint32_t dtype, uint32_t accum)
{
    switch (accum) {
    case GROVER_ACC_F64: return pick_storage<AccF64, CHECK>(dtype);
    case GROVER_ACC_F32: return pick_storage<AccF32, CHECK>(dtype);
    case GROVER_ACC_F32_KAHAN: return pick_storage<AccF32Kahan, CHECK>(dtype);
    default: return nullptr;
    }
}

}  // namespace

hipError_t fused_configure(grover_ctx *c, int *per_cu, int *block, int64_t *forced_grid)
{
    const void *k = kernel_for<false>(c->dtype, c->accum);
    if (!k)
        return hipErrorInvalidValue;
    c->fused_kernel = k;
    c->fused_check_kernel = kernel_for<true>(c->dtype, c->accum);
    c->fused_tile = kStreamTile;
    int coop = 0;
    hipError_t e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c->device);
    if (e != hipSuccess)
        return e;
    if (!coop)
        return hipErrorCooperativeLaunchTooLarge;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k, kStreamBlock, 0);
    if (e != hipSuccess)
        return e;
    *block = kStreamBlock;
    *forced_grid = 0;
    if (const char *env = getenv("GROVER_FUSED_GRID")) {
        const long long want = atoll(env);
        if (want > 0) {
            if (want > int64_t(*per_cu) * c->cu_count)
                return hipErrorCooperativeLaunchTooLarge;
            *forced_grid = want;
        }
    }
    return hipSuccess;
}

uint64_t fused_tiles(const grover_ctx *c)
{
    const uint64_t nvec = c->N / elems_per_vec(c->dtype);
    return (nvec + c->fused_tile - 1) / c->fused_tile;
}

hipError_t launch_fused_iterate(grover_ctx *c, uint64_t k, uint64_t timeout_ticks, bool check)
{
    FusedArgs a;
    a.state = c->state;
    a.nvec = c->N / elems_per_vec(c->dtype);
    a.N = double(c->N);
    a.marks = c->marks_dev;
    a.m = c->marks.size();
    a.partials = reinterpret_cast<uint64_t *>(c->partials);
    a.sync = c->sync;
    a.iters = k;
    a.gen0 = c->generation;
    a.timeout_ticks = timeout_ticks;
    void *args[] = {&a};
    const void *fn = check ? c->fused_check_kernel : c->fused_kernel;
    const hipError_t e = hipLaunchCooperativeKernel(fn, dim3(c->grid), dim3(c->block), args, 0, c->stream);
    if (e == hipSuccess)
        c->generation += k + 1u;
    return e;
}

}  // namespace grover
