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
// AccF32, AccF32Kahan; the grid tree runs in A's precision).  The update itself is always binary64.
#include "internal.h"

namespace grover {
namespace {

constexpr int kBlock = 1024;  // one workgroup per CU: fewest barrier participants, 16 waves per CU
constexpr int kUnroll = 4;    // 16-byte vectors per thread per tile
constexpr int kTile = kBlock * kUnroll;

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

template <class V>
struct Shared {
    V red[2 * (kBlock / kWave)];
    V sum[2];
    int last;
    int abort;
};

__device__ inline uint32_t *arrive_word(GridSync *s, unsigned p) { return p ? &s->arrive1 : &s->arrive0; }

__device__ inline uint64_t load_bits(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void store_bits(uint64_t *p, double x)
{
    __hip_atomic_store(p, (uint64_t)__double_as_longlong(x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide sum of (xr, xi) for barrier generation `gen`, in the arithmetic of V (binary64 or binary32;
// partials travel as binary64, which holds a binary32 exactly).  Returns false when the wait gave up
// (timeout, or another workgroup gave up); every thread of the workgroup gets the same answer and the sum
// in (xr, xi).
//
// Memory ordering: a workgroup publishes its partial and then increments the arrival counter with release
// semantics; the workgroup whose increment completes the count acquires, adds the partials in workgroup
// order, stores the sum and releases the generation flag; the others poll the flag with relaxed loads and
// acquire once it has advanced.  Acquire/release at agent scope make the data visible across the XCDs'
// separate L2s.  (Letting every workgroup poll the counter and add the partials itself was measured
// slower on MI355X: the polls contend with the increments.)
template <class V>
__device__ bool grid_sum(V &xr, V &xi, const FusedArgs &a, uint64_t gen, Shared<V> &sh)
{
    const unsigned p = unsigned(gen & 1u);
    block_sum2(xr, xi, sh.red);
    if (threadIdx.x == 0) {
        uint64_t *dst = a.partials + (uint64_t(p) * gridDim.x + blockIdx.x) * 2u;
        store_bits(dst, double(xr));
        store_bits(dst + 1, double(xi));
        const unsigned old =
            __hip_atomic_fetch_add(arrive_word(a.sync, p), 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        sh.last = (old == gridDim.x - 1u);
        sh.abort = 0;
    }
    __syncthreads();
    if (sh.last) {
        // Every partial of this barrier is published.  Add them in workgroup order.
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        V sr = V(0), si = V(0);
        for (unsigned w = threadIdx.x; w < gridDim.x; w += kBlock) {
            const uint64_t *src = a.partials + (uint64_t(p) * gridDim.x + w) * 2u;
            sr += V(__longlong_as_double((long long)load_bits(src)));
            si += V(__longlong_as_double((long long)load_bits(src + 1)));
        }
        block_sum2(sr, si, sh.red);
        if (threadIdx.x == 0) {
            store_bits(&a.sync->sum[p][0], double(sr));
            store_bits(&a.sync->sum[p][1], double(si));
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
            sh.sum[0] = V(__longlong_as_double((long long)load_bits(&a.sync->sum[p][0])));
            sh.sum[1] = V(__longlong_as_double((long long)load_bits(&a.sync->sum[p][1])));
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
// amplitudes; without a table every tile is checked against the marked list.  Loads and stores carry the
// nontemporal hint (+6 % measured on MI355X).
template <class T, class A, bool UPDATE>
__device__ inline void chunk_pass(const FusedArgs &a, const uint32_t *slow_tiles, bool table, double mr, double mi,
                                  A &acc)
{
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
            V x[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                x[u] = load16<true>(st + v0 + u * kBlock + tid);
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (UPDATE) {
                    update_vec<T>(x[u], mr, mi, 0u, acc);
                    store16<true>(x[u], st + v0 + u * kBlock + tid);
                } else {
                    accum_vec<T>(x[u], 0u, acc);
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
            V x[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint64_t v = v0 + u * kBlock + tid;
                if (v < a.nvec)
                    x[u] = load16<true>(st + v);
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint64_t v = v0 + u * kBlock + tid;
                if (v < a.nvec) {
                    const unsigned bits = in_regs ? bits_from_regs<T::EPV>(mk, v * T::EPV)
                                                  : marked_bits<T::EPV>(a.marks, mp, mq, v * T::EPV);
                    if (UPDATE) {
                        update_vec<T>(x[u], mr, mi, bits, acc);
                        store16<true>(x[u], st + v);
                    } else {
                        accum_vec<T>(x[u], bits, acc);
                    }
                }
            }
            mp = mq;
        }
    }
}

// CHECK only names a second, code-identical instantiation used for the residency check at context
// creation, so that profiles list it apart from the iteration launches.
template <class T, class A, bool CHECK>
__global__ __launch_bounds__(kBlock) void fused_iterate_kernel(FusedArgs a)
{
    using Val = typename A::value;
    __shared__ Shared<Val> sh;
    __shared__ uint32_t slow_tiles[kMarkWords];
    // Table of this workgroup's tiles that hold marked amplitudes, built once per launch.
    const uint64_t ntiles = (a.nvec + kTile - 1) / kTile;
    const uint64_t cnt = blockIdx.x < ntiles ? (ntiles - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
    const bool table = cnt <= uint64_t(kMarkWords) * 32u && a.m <= uint64_t(64) * kBlock;
    if (table) {
        for (unsigned w = threadIdx.x; w < kMarkWords; w += kBlock)
            slow_tiles[w] = 0u;
        __syncthreads();
        for (uint64_t q = threadIdx.x; q < a.m; q += kBlock) {
            const uint64_t t = a.marks[q] / T::EPV / kTile;
            if (t % gridDim.x == blockIdx.x) {
                const uint64_t j = t / gridDim.x;
                atomicOr(&slow_tiles[j >> 5], 1u << (j & 31));
            }
        }
        __syncthreads();
    }
    A acc0;
    chunk_pass<T, A, false>(a, slow_tiles, table, 0.0, 0.0, acc0);
    Val sr = acc0.res_r(), si = acc0.res_i();
    if (!grid_sum<Val>(sr, si, a, a.gen0 + 1u, sh))
        return;
    for (uint64_t it = 0; it < a.iters; ++it) {
        const double mr = (double(sr) * 2.0) / a.N, mi = (double(si) * 2.0) / a.N;
        A acc;
        chunk_pass<T, A, true>(a, slow_tiles, table, mr, mi, acc);
        sr = acc.res_r();
        si = acc.res_i();
        if (!grid_sum<Val>(sr, si, a, a.gen0 + 2u + it, sh))
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
    c->fused_tile = kTile;
    int coop = 0;
    hipError_t e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c->device);
    if (e != hipSuccess)
        return e;
    if (!coop)
        return hipErrorCooperativeLaunchTooLarge;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k, kBlock, 0);
    if (e != hipSuccess)
        return e;
    *block = kBlock;
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
