// Fused persistent iteration (proposed method, Algorithms 3-5 of arXiv:2005.04635).
//
// One cooperative launch runs k Grover iterations.  Each workgroup owns a fixed, contiguous run of tiles
// of the state for the whole launch (so every amplitude stays with one workgroup, hence one XCD and its
// L2), and each iteration is a single streaming pass over it:
//
//   read c_i, flip the sign of marked amplitudes (Algorithm 3), write c_i' = 2S/N - s_i c_i (Algorithm 4's
//   second loop), and add s_i c_i' into a binary64 accumulator — which is Algorithm 4's first loop for the
//   NEXT iteration, already applied to the next iteration's oracle-flipped state.
//
// The per-workgroup accumulators then meet at a grid barrier: every workgroup publishes its partial, the
// last one to arrive adds all partials in workgroup order (so the sum is reproducible run to run) and
// releases the others with the new S.  One read and one write of the state per iteration is the minimum:
// S depends on every amplitude, so no amplitude can be updated twice before all have been read once.
//
// A prologue pass computes S of the incoming state with the same per-thread order as the fused
// accumulation, which makes iterate(a); iterate(b) equal iterate(a + b) bit for bit.
#include "internal.h"

namespace grover {
namespace {

constexpr int kBlock = 256;
constexpr int kUnroll = 4;
constexpr int kTile = kBlock * kUnroll;  // 16-byte vectors per tile

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

struct Shared {
    double red[2 * (kBlock / kWave)];
    double sum[2];
    int last;
    int abort;
};

// Grid-wide sum of (xr, xi) for barrier generation `gen`.  Returns false when the wait gave up (timeout,
// or another workgroup gave up); every thread of the workgroup gets the same answer and the sum in (xr, xi).
__device__ bool grid_sum(double &xr, double &xi, const FusedArgs &a, uint64_t gen, Shared &sh)
{
    const unsigned p = unsigned(gen & 1u);
    block_sum2(xr, xi, sh.red);
    if (threadIdx.x == 0) {
        uint64_t *dst = a.partials + (uint64_t(p) * gridDim.x + blockIdx.x) * 2u;
        __hip_atomic_store(dst, (uint64_t)__double_as_longlong(xr), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(dst + 1, (uint64_t)__double_as_longlong(xi), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        const unsigned old =
            __hip_atomic_fetch_add(&a.sync->arrive[p], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        sh.last = (old == gridDim.x - 1u);
        sh.abort = 0;
    }
    __syncthreads();
    if (sh.last) {
        // Every partial of this barrier is published.  Add them in workgroup order.
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        double sr = 0.0, si = 0.0;
        for (unsigned w = threadIdx.x; w < gridDim.x; w += blockDim.x) {
            const uint64_t *src = a.partials + (uint64_t(p) * gridDim.x + w) * 2u;
            sr += __longlong_as_double(
                (long long)__hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            si += __longlong_as_double(
                (long long)__hip_atomic_load(src + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        }
        block_sum2(sr, si, sh.red);
        if (threadIdx.x == 0) {
            __hip_atomic_store(&a.sync->sum[p][0], (uint64_t)__double_as_longlong(sr), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.sync->sum[p][1], (uint64_t)__double_as_longlong(si), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.sync->arrive[p], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.sync->flag, gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            sh.sum[0] = sr;
            sh.sum[1] = si;
        }
    } else if (threadIdx.x == 0) {
        const uint64_t t0 = wall_clock64();
        bool ok = true;
        while (__hip_atomic_load(&a.sync->flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < gen) {
            if (__hip_atomic_load(&a.sync->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                ok = false;
                break;
            }
            if (uint64_t(wall_clock64()) - t0 > a.timeout_ticks) {
                __hip_atomic_store(&a.sync->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = false;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        if (ok) {
            sh.sum[0] = __longlong_as_double(
                (long long)__hip_atomic_load(&a.sync->sum[p][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            sh.sum[1] = __longlong_as_double(
                (long long)__hip_atomic_load(&a.sync->sum[p][1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        } else {
            sh.abort = 1;
        }
    }
    __syncthreads();
    const bool ok = sh.abort == 0;
    xr = sh.sum[0];
    xi = sh.sum[1];
    __syncthreads();  // sh is reused by the next barrier
    return ok;
}

// One pass over tiles [t_lo, t_hi) of the state.  UPDATE: c' = 2S/N - s c written back and s c' summed;
// otherwise s c summed.  The per-thread order of the sum is identical in both modes.
template <class T, bool NT, bool UPDATE>
__device__ inline void chunk_pass(const FusedArgs &a, uint64_t t_lo, uint64_t t_hi, uint64_t m_lo,
                                  uint64_t m_hi, double mr, double mi, double &ar, double &ai)
{
    using V = typename T::vec;
    V *st = static_cast<V *>(a.state);
    const unsigned tid = threadIdx.x;
    uint64_t mp = m_lo;
    uint64_t next_mark = mp < m_hi ? a.marks[mp] : ~uint64_t(0);
    for (uint64_t t = t_lo; t < t_hi; ++t) {
        const uint64_t v0 = t * kTile;
        const uint64_t end_elem = (v0 + kTile) * T::EPV;
        if (v0 + kTile <= a.nvec && next_mark >= end_elem) {
            // Full tile without marked amplitudes.
            V x[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                x[u] = load16<NT>(st + v0 + u * kBlock + tid);
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (UPDATE) {
                    update_vec<T>(x[u], mr, mi, 0u, ar, ai);
                    store16<NT>(x[u], st + v0 + u * kBlock + tid);
                } else {
                    accum_vec<T>(x[u], 0u, ar, ai);
                }
            }
        } else {
            // Ragged tail of the state, or marked amplitudes inside this tile.
            const uint64_t mq = lower_bound_u64(a.marks, mp, m_hi, end_elem);
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint64_t v = v0 + u * kBlock + tid;
                if (v < a.nvec) {
                    V x = st[v];
                    const unsigned bits = mp < mq ? marked_bits<T::EPV>(a.marks, mp, mq, v * T::EPV) : 0u;
                    if (UPDATE) {
                        update_vec<T>(x, mr, mi, bits, ar, ai);
                        st[v] = x;
                    } else {
                        accum_vec<T>(x, bits, ar, ai);
                    }
                }
            }
            mp = mq;
            next_mark = mp < m_hi ? a.marks[mp] : ~uint64_t(0);
        }
    }
}

template <class T, bool NT>
__global__ __launch_bounds__(kBlock) void fused_iterate_kernel(FusedArgs a)
{
    __shared__ Shared sh;
    const uint64_t ntiles = (a.nvec + kTile - 1) / kTile;
    const uint64_t t_lo = ntiles * blockIdx.x / gridDim.x;
    const uint64_t t_hi = ntiles * (blockIdx.x + 1u) / gridDim.x;
    const uint64_t e_lo = t_lo * kTile * T::EPV;
    const uint64_t e_hi = t_hi * kTile * T::EPV;
    const uint64_t m_lo = lower_bound_u64(a.marks, 0, a.m, e_lo);
    const uint64_t m_hi = lower_bound_u64(a.marks, m_lo, a.m, e_hi);

    double sr = 0.0, si = 0.0;
    chunk_pass<T, NT, false>(a, t_lo, t_hi, m_lo, m_hi, 0.0, 0.0, sr, si);
    if (!grid_sum(sr, si, a, a.gen0 + 1u, sh))
        return;
    for (uint64_t it = 0; it < a.iters; ++it) {
        const double mr = (sr * 2.0) / a.N, mi = (si * 2.0) / a.N;
        double ar = 0.0, ai = 0.0;
        chunk_pass<T, NT, true>(a, t_lo, t_hi, m_lo, m_hi, mr, mi, ar, ai);
        if (!grid_sum(ar, ai, a, a.gen0 + 2u + it, sh))
            return;
        sr = ar;
        si = ai;
    }
}

// Streaming hint for the state's loads and stores: nontemporal unless GROVER_FUSED_NT=0.
bool use_nontemporal()
{
    const char *env = getenv("GROVER_FUSED_NT");
    return !(env && env[0] == '0');
}

template <bool NT>
const void *kernel_nt(uint32_t dtype)
{
    switch (dtype) {
    case GROVER_F64_REAL: return reinterpret_cast<const void *>(&fused_iterate_kernel<F64Real, NT>);
    case GROVER_C64: return reinterpret_cast<const void *>(&fused_iterate_kernel<C64, NT>);
    case GROVER_C128: return reinterpret_cast<const void *>(&fused_iterate_kernel<C128, NT>);
    default: return nullptr;
    }
}

const void *kernel_for(uint32_t dtype)
{
    return use_nontemporal() ? kernel_nt<true>(dtype) : kernel_nt<false>(dtype);
}

}  // namespace

hipError_t fused_configure(grover_ctx *c, int *grid, int *block)
{
    const void *k = kernel_for(c->dtype);
    if (!k)
        return hipErrorInvalidValue;
    int coop = 0;
    hipError_t e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c->device);
    if (e != hipSuccess)
        return e;
    if (!coop)
        return hipErrorCooperativeLaunchTooLarge;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kBlock, 0);
    if (e != hipSuccess)
        return e;
    const int64_t max_grid = int64_t(per_cu) * c->cu_count;
    const uint64_t epv = c->dtype == GROVER_C128 ? 1 : 2;
    const uint64_t nvec = c->N / epv;
    const uint64_t ntiles = (nvec + kTile - 1) / kTile;
    int64_t g = max_grid;
    if (const char *env = getenv("GROVER_FUSED_GRID")) {
        const long long want = atoll(env);
        if (want > 0)
            g = want;
    } else if (uint64_t(g) > ntiles) {
        g = int64_t(ntiles);
    }
    if (g < 1)
        g = 1;
    if (g > max_grid)
        return hipErrorCooperativeLaunchTooLarge;
    *grid = int(g);
    *block = kBlock;
    return hipSuccess;
}

hipError_t launch_fused_iterate(grover_ctx *c, uint64_t k)
{
    FusedArgs a;
    a.state = c->state;
    a.nvec = c->N / (c->dtype == GROVER_C128 ? 1 : 2);
    a.N = double(c->N);
    a.marks = c->marks_dev;
    a.m = c->marks.size();
    a.partials = reinterpret_cast<uint64_t *>(c->partials);
    a.sync = c->sync;
    a.iters = k;
    a.gen0 = c->generation;
    a.timeout_ticks = c->timeout_ticks;
    void *args[] = {&a};
    const hipError_t e = hipLaunchCooperativeKernel(kernel_for(c->dtype), dim3(c->grid), dim3(c->block), args,
                                                    0, c->stream);
    if (e == hipSuccess)
        c->generation += k + 1u;
    return e;
}

}  // namespace grover
