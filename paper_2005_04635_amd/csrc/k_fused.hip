// Fused persistent iteration (proposed method, Algorithms 3-5 of arXiv:2005.04635).
//
// One cooperative launch runs k Grover iterations.  Each workgroup owns a fixed set of tiles of the state
// for the whole launch (so every amplitude stays with one workgroup, hence one XCD and its L2), and each
// iteration is a single streaming pass over it:
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

template <int BLOCK>
struct Shared {
    double red[2 * (BLOCK / kWave)];
    double sum[2];
    int last;
    int abort;
};

__device__ inline uint32_t *arrive_word(GridSync *s, unsigned p) { return p ? &s->arrive1 : &s->arrive0; }

// Grid-wide sum of (xr, xi) for barrier generation `gen`.  Returns false when the wait gave up (timeout,
// or another workgroup gave up); every thread of the workgroup gets the same answer and the sum in (xr, xi).
//
// Memory ordering: a workgroup publishes its partial and then increments the arrival counter with release
// semantics; the workgroup whose increment completes the count acquires, adds the partials in workgroup
// order, stores the sum and releases the generation flag; the others poll the flag with relaxed loads and
// acquire once it has advanced.  Acquire/release at agent scope make the data visible across the XCDs'
// separate L2s.  (Letting every workgroup poll the counter and add the partials itself was measured
// slower on MI355X: the polls contend with the increments.)
template <int BLOCK>
__device__ bool grid_sum(double &xr, double &xi, const FusedArgs &a, uint64_t gen, Shared<BLOCK> &sh)
{
    const unsigned p = unsigned(gen & 1u);
    block_sum2(xr, xi, sh.red);
    if (threadIdx.x == 0) {
        uint64_t *dst = a.partials + (uint64_t(p) * gridDim.x + blockIdx.x) * 2u;
        __hip_atomic_store(dst, (uint64_t)__double_as_longlong(xr), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(dst + 1, (uint64_t)__double_as_longlong(xi), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        const unsigned old =
            __hip_atomic_fetch_add(arrive_word(a.sync, p), 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        sh.last = (old == gridDim.x - 1u);
        sh.abort = 0;
    }
    __syncthreads();
    if (sh.last) {
        // Every partial of this barrier is published.  Add them in workgroup order.
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        double sr = 0.0, si = 0.0;
        for (unsigned w = threadIdx.x; w < gridDim.x; w += BLOCK) {
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
            __hip_atomic_store(arrive_word(a.sync, p), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.sync->flag, gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            sh.sum[0] = sr;
            sh.sum[1] = si;
        }
    } else if (threadIdx.x == 0) {
        const uint64_t t0 = wall_clock64();
        bool ok = true;
        while (__hip_atomic_load(&a.sync->flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen) {
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
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
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

// First index q >= start with marks[q] >= x in the sorted list marks[0, m), given that every entry before
// `start` is < x: exponential steps from `start`, then a binary search in the last step.  Tiles are visited
// in increasing order, so each search starts where the previous tile's ended and costs O(log gap).
__device__ inline uint64_t gallop_lower_bound(const uint64_t *marks, uint64_t start, uint64_t m, uint64_t x)
{
    if (start >= m || marks[start] >= x)
        return start;
    uint64_t lo = start, step = 1;  // invariant: marks[lo] < x
    while (lo + step < m && marks[lo + step] < x) {
        lo += step;
        step <<= 1;
    }
    const uint64_t hi = lo + step < m ? lo + step : m;
    return lower_bound_u64(marks, lo + 1, hi, x);
}

// Marks of one tile held in registers: up to kTileMarks entries of the sorted slice marks[lo, hi), padded
// with ~0 (never equal to an amplitude index).  Longer slices fall back to a binary search per vector.
constexpr int kTileMarks = 8;

template <int EPV>
__device__ inline unsigned bits_from_regs(const uint64_t (&mk)[kTileMarks], uint64_t i)
{
    unsigned bits = 0;
#pragma unroll
    for (int q = 0; q < kTileMarks; ++q) {
        const uint64_t d = mk[q] - i;  // wraps to a huge value when mk[q] < i
        bits |= d < uint64_t(EPV) ? 1u << unsigned(d) : 0u;
    }
    return bits;
}

constexpr int kMarkWords = 1024;  // LDS bitmap of this workgroup's tiles that hold marked amplitudes

// One pass over this workgroup's tiles t = blockIdx.x + j G, j = 0, 1, ... (G = gridDim.x).  At any moment
// the grid streams one contiguous window of the state, spread over all HBM channels, while each tile still
// belongs to the same workgroup (hence XCD) in every iteration.  (Alternating the direction between passes,
// to start on lines the memory-side cache might still hold, measured no faster on MI355X.)  UPDATE:
// c' = 2S/N - s c written back and s c' summed; otherwise s c summed.  The per-thread order of the sum is
// identical in both modes.  `slow_tiles` (when `table`) flags the workgroup's tiles holding marked
// amplitudes; without a table every tile is checked against the marked list.
template <class T, bool NT, int BLOCK, int UNROLL, bool UPDATE>
__device__ inline void chunk_pass(const FusedArgs &a, const uint32_t *slow_tiles, bool table, double mr, double mi,
                                  double &ar, double &ai)
{
    constexpr int kTile = BLOCK * UNROLL;  // 16-byte vectors per tile
    using V = typename T::vec;
    V *st = static_cast<V *>(a.state);
    const unsigned tid = threadIdx.x;
    const uint64_t ntiles = (a.nvec + kTile - 1) / kTile;
    const uint64_t cnt = blockIdx.x < ntiles ? (ntiles - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
    uint64_t mp = 0;  // marked entries before this position lie in tiles already visited
    for (uint64_t j = 0; j < cnt; ++j) {
        const uint64_t t = blockIdx.x + j * gridDim.x;
        const uint64_t v0 = t * kTile;
        const bool full = v0 + kTile <= a.nvec;
        const bool marked = table ? ((slow_tiles[j >> 5] >> (j & 31)) & 1u) != 0u : a.m > 0;
        if (full && !marked) {
            V x[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u)
                x[u] = load16<NT>(st + v0 + u * BLOCK + tid);
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                if (UPDATE) {
                    update_vec<T>(x[u], mr, mi, 0u, ar, ai);
                    store16<NT>(x[u], st + v0 + u * BLOCK + tid);
                } else {
                    accum_vec<T>(x[u], 0u, ar, ai);
                }
            }
        } else {
            // Ragged tail of the state, or a tile that may hold marked amplitudes: the same vector loads,
            // then each amplitude's sign from the tile's slice [mp, mq) of the sorted marked list.
            mp = gallop_lower_bound(a.marks, mp, a.m, v0 * T::EPV);
            const uint64_t mq = gallop_lower_bound(a.marks, mp, a.m, (v0 + kTile) * T::EPV);
            const bool in_regs = mq - mp <= uint64_t(kTileMarks);
            uint64_t mk[kTileMarks];
#pragma unroll
            for (int q = 0; q < kTileMarks; ++q)
                mk[q] = in_regs && mp + q < mq ? a.marks[mp + q] : ~uint64_t(0);
            V x[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const uint64_t v = v0 + u * BLOCK + tid;
                if (v < a.nvec)
                    x[u] = load16<NT>(st + v);
            }
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const uint64_t v = v0 + u * BLOCK + tid;
                if (v < a.nvec) {
                    const unsigned bits = in_regs ? bits_from_regs<T::EPV>(mk, v * T::EPV)
                                                  : marked_bits<T::EPV>(a.marks, mp, mq, v * T::EPV);
                    if (UPDATE) {
                        update_vec<T>(x[u], mr, mi, bits, ar, ai);
                        store16<NT>(x[u], st + v);
                    } else {
                        accum_vec<T>(x[u], bits, ar, ai);
                    }
                }
            }
            mp = mq;
        }
    }
}

template <class T, bool NT, int BLOCK, int UNROLL, bool CHECK = false>
__global__ __launch_bounds__(BLOCK) void fused_iterate_kernel(FusedArgs a)
{
    constexpr int kTile = BLOCK * UNROLL;
    __shared__ Shared<BLOCK> sh;
    __shared__ uint32_t slow_tiles[kMarkWords];
    // Table of this workgroup's tiles that hold marked amplitudes, built once per launch.
    const uint64_t ntiles = (a.nvec + kTile - 1) / kTile;
    const uint64_t cnt = blockIdx.x < ntiles ? (ntiles - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
    const bool table = cnt <= uint64_t(kMarkWords) * 32u && a.m <= uint64_t(64) * BLOCK;
    if (table) {
        for (unsigned w = threadIdx.x; w < kMarkWords; w += BLOCK)
            slow_tiles[w] = 0u;
        __syncthreads();
        for (uint64_t q = threadIdx.x; q < a.m; q += BLOCK) {
            const uint64_t t = a.marks[q] / T::EPV / kTile;
            if (t % gridDim.x == blockIdx.x) {
                const uint64_t j = t / gridDim.x;
                atomicOr(&slow_tiles[j >> 5], 1u << (j & 31));
            }
        }
        __syncthreads();
    }
    double sr = 0.0, si = 0.0;
    chunk_pass<T, NT, BLOCK, UNROLL, false>(a, slow_tiles, table, 0.0, 0.0, sr, si);
    if (!grid_sum<BLOCK>(sr, si, a, a.gen0 + 1u, sh))
        return;
    for (uint64_t it = 0; it < a.iters; ++it) {
        const double mr = (sr * 2.0) / a.N, mi = (si * 2.0) / a.N;
        double ar = 0.0, ai = 0.0;
        chunk_pass<T, NT, BLOCK, UNROLL, true>(a, slow_tiles, table, mr, mi, ar, ai);
        if (!grid_sum<BLOCK>(ar, ai, a, a.gen0 + 2u + it, sh))
            return;
        sr = ar;
        si = ai;
    }
}

// Launch variant: workgroup size, unroll (16-byte vectors per thread per tile) and the streaming hint.
// Defaults are set by measurement on MI355X; GROVER_FUSED_BLOCK / _UNROLL / _NT override them.
struct Variant {
    int block = 1024;
    int unroll = 4;
    bool nt = true;
};

Variant variant()
{
    Variant v;
    if (const char *e = getenv("GROVER_FUSED_BLOCK"))
        v.block = atoi(e);
    if (const char *e = getenv("GROVER_FUSED_UNROLL"))
        v.unroll = atoi(e);
    if (const char *e = getenv("GROVER_FUSED_NT"))
        v.nt = e[0] != '0';
    return v;
}

template <class T, bool NT, int BLOCK, bool CHECK>
const void *pick_unroll(int unroll)
{
    switch (unroll) {
    case 2: return reinterpret_cast<const void *>(&fused_iterate_kernel<T, NT, BLOCK, 2, CHECK>);
    case 4: return reinterpret_cast<const void *>(&fused_iterate_kernel<T, NT, BLOCK, 4, CHECK>);
    case 8: return reinterpret_cast<const void *>(&fused_iterate_kernel<T, NT, BLOCK, 8, CHECK>);
    default: return nullptr;
    }
}

template <class T, bool NT, bool CHECK>
const void *pick_block(int block, int unroll)
{
    switch (block) {
    case 256: return pick_unroll<T, NT, 256, CHECK>(unroll);
    case 512: return pick_unroll<T, NT, 512, CHECK>(unroll);
    case 1024: return pick_unroll<T, NT, 1024, CHECK>(unroll);
    default: return nullptr;
    }
}

template <class T, bool CHECK>
const void *pick(const Variant &v)
{
    return v.nt ? pick_block<T, true, CHECK>(v.block, v.unroll) : pick_block<T, false, CHECK>(v.block, v.unroll);
}

template <bool CHECK>
const void *kernel_for(uint32_t dtype, const Variant &v)
{
    switch (dtype) {
    case GROVER_F64_REAL: return pick<F64Real, CHECK>(v);
    case GROVER_C64: return pick<C64, CHECK>(v);
    case GROVER_C128: return pick<C128, CHECK>(v);
    default: return nullptr;
    }
}

}  // namespace

hipError_t fused_configure(grover_ctx *c, int *per_cu, int *block, int64_t *forced_grid)
{
    const Variant v = variant();
    const void *k = kernel_for<false>(c->dtype, v);
    if (!k)
        return hipErrorInvalidValue;
    c->fused_kernel = k;
    c->fused_check_kernel = kernel_for<true>(c->dtype, v);
    c->fused_tile = uint64_t(v.block) * v.unroll;
    int coop = 0;
    hipError_t e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c->device);
    if (e != hipSuccess)
        return e;
    if (!coop)
        return hipErrorCooperativeLaunchTooLarge;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k, v.block, 0);
    if (e != hipSuccess)
        return e;
    *block = v.block;
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
    const uint64_t nvec = c->N / (c->dtype == GROVER_C128 ? 1 : 2);
    return (nvec + c->fused_tile - 1) / c->fused_tile;
}

hipError_t launch_fused_iterate(grover_ctx *c, uint64_t k, uint64_t timeout_ticks, bool check)
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
    a.timeout_ticks = timeout_ticks;
    void *args[] = {&a};
    const void *fn = check ? c->fused_check_kernel : c->fused_kernel;
    const hipError_t e = hipLaunchCooperativeKernel(fn, dim3(c->grid), dim3(c->block), args, 0, c->stream);
    if (e == hipSuccess)
        c->generation += k + 1u;
    return e;
}

}  // namespace grover
