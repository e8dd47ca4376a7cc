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
// The per-workgroup accumulators then meet at a grid barrier: every workgroup publishes its partial,
// workgroup 0 gathers all of them and adds them in a fixed order (so the sum is reproducible run to run)
// and publishes the new S to the others.  One read and one write of the state per iteration is the minimum:
// S depends on every amplitude, so no amplitude can be updated twice before all have been read once.
//
// A prologue pass computes S of the incoming state with the same per-thread order as the fused
// accumulation, which makes iterate(a); iterate(b) equal iterate(a + b) bit for bit.
//
// Template parameters: T = storage type (F64Real, C64, C128, CBF16), A = accumulator of the sum (AccF64,
// AccF32, AccF32Kahan; the grid tree runs in A's precision), CHECK = a second symbol of the same code for the
// residency check at context creation, NT = nontemporal accesses beyond the part of the state kept in the
// memory-side cache (kTemporalBytes), U32 = the update in binary32 from 2S/N rounded to binary32 (complex64
// storage with binary64 sums only; otherwise the update is binary64, rounded once to the storage type).
#include "internal.h"

namespace grover {
namespace {

// Tiles of 4096 16-byte vectors (64 KiB), moved by one persistent workgroup per CU in one of two shapes.
// 512 threads of 8 vectors each (two waves per SIMD, so a thread may hold up to 256 VGPRs): on MI355X this
// shape streamed a 2 GiB in-place pass at 5.77 TB/s against 5.66 for 1024 threads of 4 vectors (global
// instructions; 5.82 against 5.76 with the buffer instructions used now), and its registers hold 4 tiles
// where the 1024-thread shape (128 VGPRs a thread) holds one; n = 28 complex64, 27 complex128 and 27
// binary64 searches ran 4.3-4.8 % faster with it.  Complex bfloat16, whose conversions make it the most
// arithmetic per byte, keeps 1024 threads (the 512-thread shape, with three register tiles, ran 1-8 %
// slower at n = 25-27 and 0.6 % faster at n = 28).
constexpr int kTile = 4096;
constexpr int kMaxBlock = 1024;

template <class T>
struct Shape {
    static constexpr int block = T::EPV == 4 ? 1024 : 512;  // threads per workgroup
    static constexpr int unroll = kTile / block;             // 16-byte vectors per thread per tile
    static constexpr int reg_tiles = T::EPV == 4 ? 1 : 4;    // held tiles in registers (4 VGPRs per vector)
    // Nontemporal stores: nt sc1 streamed binary64 and complex128 states 1.6-1.9 % faster than nt alone on
    // MI355X (n = 26, 27), nt alone complex64 and complex bfloat16 states 0.4-1.6 % faster (n = 26-28).
    static constexpr int store_nt = T::kBytes == 16 || !T::kComplex ? kBufNTDevice : kBufNT;
};

struct FusedArgs {
    void *state;
    uint64_t nvec;  // N / EPV
    double N;
    const uint64_t *marks;
    uint64_t m;
    uint64_t *partials;  // slots [2][grid][4], then the published sum [2][4] (tagged words)
    GridSync *sync;
    uint64_t iters;
    uint64_t gen0;
    uint64_t timeout_ticks;
    uint64_t temporal_tiles;  // nontemporal kernels: leading tiles of each share streamed with ordinary accesses
};

template <class V>
struct Shared {
    V red[2 * (kMaxBlock / kWave)];
    V sum[2];
    int abort;
};

// A binary64 value published as two self-validating 64-bit words: each carries 32 bits of the value in its
// high half and the barrier generation (mod 2^32) in its low half.  Each word is one atomic access, so a
// reader that sees the current generation in both words has both halves of this generation's value, and
// the barrier needs no memory fence (on this GPU a release writes back, and an acquire invalidates, a whole
// L2; the workgroups share nothing but these values within a launch).  The host keeps generations below
// 2^32 by clearing the slots before they would wrap.
__device__ inline void put_tagged(uint64_t *w, double x, uint32_t tag)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    __hip_atomic_store(w, (b & 0xFFFFFFFF00000000ull) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(w + 1, (b << 32) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait until the two values at w[0 .. 3] carry generation `tag`; gives up when the error word is
// set or the wall-clock limit passes (then setting the error word).
__device__ inline bool wait_pair(const uint64_t *w, uint32_t tag, const FusedArgs &a, double &x, double &y)
{
    const uint64_t t0 = wall_clock64();
    for (;;) {
        const uint64_t h0 = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t l0 = __hip_atomic_load(w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t h1 = __hip_atomic_load(w + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t l1 = __hip_atomic_load(w + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (uint32_t(h0) == tag && uint32_t(l0) == tag && uint32_t(h1) == tag && uint32_t(l1) == tag) {
            x = __longlong_as_double((long long)((h0 & 0xFFFFFFFF00000000ull) | (l0 >> 32)));
            y = __longlong_as_double((long long)((h1 & 0xFFFFFFFF00000000ull) | (l1 >> 32)));
            return true;
        }
        if (__hip_atomic_load(&a.sync->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
            return false;
        if (uint64_t(wall_clock64()) - t0 > a.timeout_ticks) {
            __hip_atomic_store(&a.sync->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Bounded wait until the pairs of up to four slots, w[i * stride .. i * stride + 3] for i < cnt, carry
// generation `tag`: the loads of every slot not yet seen are issued together, so that the wait costs about
// one memory round trip instead of one per slot.  Gives up as wait_pair does.
__device__ inline bool wait_pairs4(const uint64_t *w, uint64_t stride, unsigned cnt, uint32_t tag,
                                   const FusedArgs &a, double (&x)[4], double (&y)[4])
{
    const uint64_t t0 = wall_clock64();
    const unsigned all = (1u << cnt) - 1u;
    unsigned done = 0u;  // bit i: slot i seen
    for (;;) {
#pragma unroll
        for (unsigned i = 0; i < 4u; ++i) {
            if (i < cnt && ((done >> i) & 1u) == 0u) {
                const uint64_t *s = w + uint64_t(i) * stride;
                const uint64_t h0 = __hip_atomic_load(s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t l0 = __hip_atomic_load(s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t h1 = __hip_atomic_load(s + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t l1 = __hip_atomic_load(s + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (uint32_t(h0) == tag && uint32_t(l0) == tag && uint32_t(h1) == tag && uint32_t(l1) == tag) {
                    x[i] = __longlong_as_double((long long)((h0 & 0xFFFFFFFF00000000ull) | (l0 >> 32)));
                    y[i] = __longlong_as_double((long long)((h1 & 0xFFFFFFFF00000000ull) | (l1 >> 32)));
                    done |= 1u << i;
                }
            }
        }
        if (done == all)
            return true;
        if (__hip_atomic_load(&a.sync->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
            return false;
        if (uint64_t(wall_clock64()) - t0 > a.timeout_ticks) {
            __hip_atomic_store(&a.sync->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Grid-wide sum of (xr, xi) at generation `gen`: every workgroup publishes its partial as tagged words in
// its slot of the generation's parity; wave 0 gathers them (lane l waits for the slots of workgroups l,
// l + 64, ..., four of them at a time together, and adds them in that order; the lanes' values are then
// added by wave_total), so the sum is reproducible run to run.  ALL: every workgroup gathers, and all of them compute the same bits in one
// memory round trip.  Otherwise workgroup 0 gathers and publishes the sum as tagged words, which the other
// workgroups poll: two round trips, but far fewer polls while other workgroups still stream (the form
// for states too large for the memory-side cache).  A slot of parity p is rewritten two generations later:
// its owner's next partial needs this generation's sum, and the one after that needs every workgroup's
// next partial, which each publishes only after its reads here; the published sum is double-buffered the
// same way.  Two workgroup barriers: one before thread 0 adds the wave partials, one before every thread
// reads the sum.  The LDS words are written again only after the first barrier of the next call, which
// every thread reaches after its reads here, so no barrier is needed behind them.  Returns false when a
// wait gave up.
template <class V, bool ALL, int B>
__device__ __forceinline__ bool grid_sum(V &xr, V &xi, const FusedArgs &a, uint64_t gen, Shared<V> &sh)
{
    const uint32_t tag = uint32_t(gen);
    const unsigned p = unsigned(gen & 1u);
    const unsigned lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    uint64_t *slots = a.partials + uint64_t(p) * gridDim.x * 4u;
    uint64_t *bcast = a.partials + uint64_t(2) * gridDim.x * 4u + uint64_t(p) * 4u;
    xr = wave_total(xr);
    xi = wave_total(xi);
    if (lane == 0) {
        sh.red[2 * wave] = xr;
        sh.red[2 * wave + 1] = xi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        V sr = V(0), si = V(0);
        for (unsigned w = 0; w < B / kWave; ++w) {
            sr += sh.red[2 * w];
            si += sh.red[2 * w + 1];
        }
        uint64_t *slot = slots + uint64_t(blockIdx.x) * 4u;
        put_tagged(slot, double(sr), tag);
        put_tagged(slot + 2, double(si), tag);
    }
    if (ALL || blockIdx.x == 0) {
        if (wave == 0) {
            V pr = V(0), pi = V(0);
            bool ok = true;
            for (unsigned g0 = 0; g0 < gridDim.x && ok; g0 += 4u * kWave) {
                const unsigned first = g0 + lane;
                const unsigned left = first < gridDim.x ? (gridDim.x - first + kWave - 1u) / kWave : 0u;
                const unsigned cnt = left < 4u ? left : 4u;
                double x[4], y[4];
                ok = wait_pairs4(slots + uint64_t(first) * 4u, uint64_t(kWave) * 4u, cnt, tag, a, x, y);
                for (unsigned i = 0; i < cnt && ok; ++i) {
                    pr += V(x[i]);
                    pi += V(y[i]);
                }
            }
            pr = wave_total(pr);
            pi = wave_total(pi);
            const bool failed = __any(!ok);
            if (lane == 0) {
                sh.abort = failed;
                if (!failed) {
                    if (!ALL) {
                        put_tagged(bcast, double(pr), tag);
                        put_tagged(bcast + 2, double(pi), tag);
                    }
                    sh.sum[0] = pr;
                    sh.sum[1] = pi;
                }
            }
        }
    } else if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
        const bool ok = wait_pair(bcast, tag, a, x, y);
        sh.abort = !ok;
        sh.sum[0] = V(x);
        sh.sum[1] = V(y);
    }
    __syncthreads();
    xr = sh.sum[0];
    xi = sh.sum[1];
    return sh.abort == 0;
}

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
// amplitudes; without a table every tile is checked against the marked list.  NT: loads and stores carry the
// nontemporal hint (+6 % measured on MI355X at n = 28), except in the first a.temporal_tiles unmarked tiles
// of the share, whose ordinary accesses leave them in the memory-side cache for the next pass; without NT
// (a state that fits that cache) every access is ordinary.  See kTemporalBytes.
// A workgroup keeps the last held_tiles<T>() tiles of its share on chip for the whole launch: the last
// reg_tiles<T>() in registers (rt[r][u], U vectors per thread each, always indexed by compile-time r and u
// so that they stay in registers), the kLdsTiles before them in LDS (each thread its own slots,
// held[(h * U + u) * B + tid], so no barrier guards them).  The launch's first pass loads them
// while it sums them, every iteration then updates them in place, and the end of the launch writes them
// back.  They are the last tiles each pass visits, so the additions happen in the same order as when they
// stream and the results are identical; an iteration's memory traffic drops by held_tiles<T>() of the
// workgroup's tiles (6/128 of it at n = 28, complex64, on 256 workgroups; 3/64 for complex bfloat16).
constexpr int kLdsTiles = 2;
template <class T>
constexpr int reg_tiles() { return Shape<T>::reg_tiles; }
template <class T>
constexpr int held_tiles() { return kLdsTiles + reg_tiles<T>(); }

// First held tile (local index) of this workgroup's share of cnt tiles, and the first held in registers.
template <class T>
__device__ inline uint64_t held_start(uint64_t cnt)
{
    return cnt > uint64_t(held_tiles<T>()) ? cnt - held_tiles<T>() : 0;
}
template <class T>
__device__ inline uint64_t reg_start(uint64_t cnt)
{
    return cnt > uint64_t(reg_tiles<T>()) ? cnt - reg_tiles<T>() : 0;
}

// The update of one vector in the kernel's update precision: U32, binary32 from 2S/N rounded to binary32
// (complex64 storage only); otherwise binary64, rounded once to the storage type.
template <class T, bool U32, class A>
__device__ __forceinline__ void update_one(typename T::vec &v, double mr, double mi, float mr32, float mi32,
                                           unsigned bits, A &acc)
{
    if constexpr (U32)
        update_vec_f32(v, mr32, mi32, bits, acc);
    else
        update_vec<T>(v, mr, mi, bits, acc);
}

// The state is accessed through one buffer resource per tile: vectors [v0, v0 + kTile) cut at nvec, each
// thread's u-th vector at byte offset (u B + tid) 16, the same for every tile.  NT: loads nt, stores
// Shape<T>::store_nt; otherwise ordinary.  (One resource over the whole state, with the tile's byte offset
// added to every lane's, made the kernel 0.2-2.3 % slower on MI355X at n = 26-28.)
template <class V>
__device__ inline __amdgpu_buffer_rsrc_t tile_rsrc(void *state, uint64_t nvec, uint64_t v0)
{
    const uint64_t n = nvec - v0 < uint64_t(kTile) ? nvec - v0 : uint64_t(kTile);
    return buffer_rsrc(static_cast<V *>(state) + v0, uint32_t(n * 16u));
}
template <int B>
__device__ inline uint32_t lane_off(int u, unsigned tid)
{
    return (uint32_t(u) * uint32_t(B) + tid) * 16u;
}
template <bool NT>
constexpr int load_policy() { return NT ? kBufNT : kBufPlain; }
template <class T, bool NT>
constexpr int store_policy() { return NT ? Shape<T>::store_nt : kBufPlain; }

// A full tile without marked amplitudes: every sign is +1.  NT selects the nontemporal loads and stores.
template <class T, class A, bool UPDATE, bool NT, bool U32>
__device__ __forceinline__ void plain_tile(void *state, uint64_t nvec, uint64_t v0, unsigned tid, double mr,
                                           double mi, float mr32, float mi32, A &acc)
{
    constexpr int B = Shape<T>::block, U = Shape<T>::unroll;
    using V = typename T::vec;
    const auto rs = tile_rsrc<V>(state, nvec, v0);
    V x[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
        x[u] = bload16<load_policy<NT>(), V>(rs, lane_off<B>(u, tid));
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (UPDATE) {
            update_one<T, U32>(x[u], mr, mi, mr32, mi32, 0u, acc);
            bstore16<store_policy<T, NT>()>(x[u], rs, lane_off<B>(u, tid));
        } else {
            accum_vec<T>(x[u], 0u, acc);
        }
    }
}

// One held tile in registers (local index j of the share), updated in place or, in the first pass, loaded
// and summed; mp is the running position in the marked list, as in the streamed tiles.
template <class T, class A, bool UPDATE, bool U32>
__device__ __forceinline__ void reg_tile(const FusedArgs &a, const uint32_t *slow_tiles, bool table, double mr,
                                         double mi, float mr32, float mi32, A &acc, uint64_t j, uint64_t &mp,
                                         typename T::vec (&r)[Shape<T>::unroll])
{
    constexpr int B = Shape<T>::block, U = Shape<T>::unroll;
    using V = typename T::vec;
    const unsigned tid = threadIdx.x;
    const uint64_t t = blockIdx.x + j * gridDim.x;
    const uint64_t v0 = t * kTile;
    const bool full = v0 + kTile <= a.nvec;
    const bool marked = table ? ((slow_tiles[j >> 5] >> (j & 31)) & 1u) != 0u : a.m > 0;
    uint64_t mq = mp;
    bool in_regs = true;
    uint64_t mk[kTileMarks];
    if (!full || marked) {
        mp = gallop_lower_bound(a.marks, mp, a.m, v0 * T::EPV);
        mq = gallop_lower_bound(a.marks, mp, a.m, (v0 + kTile) * T::EPV);
        in_regs = mq - mp <= uint64_t(kTileMarks);
#pragma unroll
        for (int q = 0; q < kTileMarks; ++q)
            mk[q] = in_regs && mp + q < mq ? a.marks[mp + q] : ~uint64_t(0);
    }
    if (!UPDATE) {
        const auto rs = tile_rsrc<V>(a.state, a.nvec, v0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t v = v0 + u * B + tid;
            if (v < a.nvec)
                r[u] = bload16<kBufNT, V>(rs, lane_off<B>(u, tid));
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint64_t v = v0 + u * B + tid;
        if (v < a.nvec) {
            unsigned bits = 0u;
            if (!full || marked)
                bits = in_regs ? bits_from_regs<T::EPV>(mk, v * T::EPV) : marked_bits<T::EPV>(a.marks, mp, mq, v * T::EPV);
            if (UPDATE)
                update_one<T, U32>(r[u], mr, mi, mr32, mi32, bits, acc);
            else
                accum_vec<T>(r[u], bits, acc);
        }
    }
    if (!full || marked)
        mp = mq;
}

template <class T, class A, bool UPDATE, bool NT, bool U32>
__device__ __forceinline__ void chunk_pass(const FusedArgs &a, const uint32_t *slow_tiles, bool table, double mr, double mi,
                                  A &acc, typename T::vec *held, typename T::vec (&rt)[reg_tiles<T>()][Shape<T>::unroll])
{
    constexpr int B = Shape<T>::block, U = Shape<T>::unroll;
    using V = typename T::vec;
    const float mr32 = float(mr), mi32 = float(mi);  // the binary32 update's 2S/N (rounded to nearest even)
    const unsigned tid = threadIdx.x;
    const uint64_t ntiles = (a.nvec + kTile - 1) / kTile;
    const uint64_t cnt = blockIdx.x < ntiles ? (ntiles - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
    const uint64_t hstart = held_start<T>(cnt);
    uint64_t mp = 0;  // marked entries before this position lie in tiles already visited
    for (uint64_t j = 0; j < hstart; ++j) {
        const uint64_t t = blockIdx.x + j * gridDim.x;
        const uint64_t v0 = t * kTile;
        const bool full = v0 + kTile <= a.nvec;
        const bool marked = table ? ((slow_tiles[j >> 5] >> (j & 31)) & 1u) != 0u : a.m > 0;
        if (full && !marked && (!NT || j < a.temporal_tiles)) {
            plain_tile<T, A, UPDATE, false, U32>(a.state, a.nvec, v0, tid, mr, mi, mr32, mi32, acc);
        } else if (full && !marked) {
            plain_tile<T, A, UPDATE, true, U32>(a.state, a.nvec, v0, tid, mr, mi, mr32, mi32, acc);
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
            const auto rs = tile_rsrc<V>(a.state, a.nvec, v0);
            V x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t v = v0 + u * B + tid;
                if (v < a.nvec)
                    x[u] = bload16<load_policy<NT>(), V>(rs, lane_off<B>(u, tid));
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t v = v0 + u * B + tid;
                if (v < a.nvec) {
                    const unsigned bits = in_regs ? bits_from_regs<T::EPV>(mk, v * T::EPV)
                                                  : marked_bits<T::EPV>(a.marks, mp, mq, v * T::EPV);
                    if (UPDATE) {
                        update_one<T, U32>(x[u], mr, mi, mr32, mi32, bits, acc);
                        bstore16<store_policy<T, NT>()>(x[u], rs, lane_off<B>(u, tid));
                    } else {
                        accum_vec<T>(x[u], bits, acc);
                    }
                }
            }
            mp = mq;
        }
    }
    // the held tiles: the same arithmetic on the thread's LDS slots (loaded from memory by the first pass),
    // then on the last tiles, kept in registers
    const uint64_t rstart = reg_start<T>(cnt);
    for (uint64_t j = hstart; j < rstart; ++j) {
        V *hv = held + (j - hstart) * kTile;
        const uint64_t t = blockIdx.x + j * gridDim.x;
        const uint64_t v0 = t * kTile;
        const bool full = v0 + kTile <= a.nvec;
        const bool marked = table ? ((slow_tiles[j >> 5] >> (j & 31)) & 1u) != 0u : a.m > 0;
        uint64_t mq = mp;
        bool in_regs = true;
        uint64_t mk[kTileMarks];
        if (!full || marked) {
            mp = gallop_lower_bound(a.marks, mp, a.m, v0 * T::EPV);
            mq = gallop_lower_bound(a.marks, mp, a.m, (v0 + kTile) * T::EPV);
            in_regs = mq - mp <= uint64_t(kTileMarks);
#pragma unroll
            for (int q = 0; q < kTileMarks; ++q)
                mk[q] = in_regs && mp + q < mq ? a.marks[mp + q] : ~uint64_t(0);
        }
        const auto rs = tile_rsrc<V>(a.state, a.nvec, v0);
        V x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t v = v0 + u * B + tid;
            if (v < a.nvec) {
                if (UPDATE) {
                    x[u] = hv[u * B + tid];
                } else {
                    x[u] = bload16<kBufNT, V>(rs, lane_off<B>(u, tid));
                    hv[u * B + tid] = x[u];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t v = v0 + u * B + tid;
            if (v < a.nvec) {
                unsigned bits = 0u;
                if (!full || marked)
                    bits = in_regs ? bits_from_regs<T::EPV>(mk, v * T::EPV)
                                   : marked_bits<T::EPV>(a.marks, mp, mq, v * T::EPV);
                if (UPDATE) {
                    update_one<T, U32>(x[u], mr, mi, mr32, mi32, bits, acc);
                    hv[u * B + tid] = x[u];
                } else {
                    accum_vec<T>(x[u], bits, acc);
                }
            }
        }
        if (!full || marked)
            mp = mq;
    }
#pragma unroll
    for (int r = 0; r < reg_tiles<T>(); ++r)
        if (rstart + uint64_t(r) < cnt)
            reg_tile<T, A, UPDATE, U32>(a, slow_tiles, table, mr, mi, mr32, mi32, acc, rstart + uint64_t(r), mp, rt[r]);
}

// CHECK only names a second, code-identical instantiation used for the residency check at context
// creation, so that profiles list it apart from the iteration launches.
template <class T, class A, bool CHECK, bool NT, bool U32>
__global__ __launch_bounds__(Shape<T>::block) void fused_iterate_kernel(FusedArgs a)
{
    constexpr int B = Shape<T>::block, U = Shape<T>::unroll;
    using Val = typename A::value;
    __shared__ Shared<Val> sh;
    __shared__ uint32_t slow_tiles[kMarkWords];
    __shared__ typename T::vec held[kLdsTiles * kTile];  // held tiles in LDS
    typename T::vec rt[reg_tiles<T>()][U];               // the last held tiles, in registers
    // A launch enqueued behind a failure (a wait that gave up, or input rejected on the device) leaves the
    // state as it is; the error word is cleared before the next launch that should run.  Thread 0 decides
    // for the whole workgroup (the word may change while its threads read it); grid_sum writes sh.abort
    // again only after its first workgroup barrier, which every thread reaches after reading it here.
    if (threadIdx.x == 0)
        sh.abort = __hip_atomic_load(&a.sync->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    __syncthreads();
    if (sh.abort)
        return;
    // Table of this workgroup's tiles that hold marked amplitudes, built once per launch.
    const uint64_t ntiles = (a.nvec + kTile - 1) / kTile;
    const uint64_t cnt = blockIdx.x < ntiles ? (ntiles - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
    const bool table = cnt <= uint64_t(kMarkWords) * 32u && a.m <= uint64_t(64) * B;
    if (table) {
        for (unsigned w = threadIdx.x; w < kMarkWords; w += B)
            slow_tiles[w] = 0u;
        __syncthreads();
        for (uint64_t q = threadIdx.x; q < a.m; q += B) {
            const uint64_t t = a.marks[q] / T::EPV / kTile;
            if (t < ntiles && t % gridDim.x == blockIdx.x) {
                const uint64_t j = t / gridDim.x;
                atomicOr(&slow_tiles[j >> 5], 1u << (j & 31));
            }
        }
        __syncthreads();
    }
    A acc0;
    chunk_pass<T, A, false, NT, U32>(a, slow_tiles, table, 0.0, 0.0, acc0, held, rt);
    Val sr = acc0.res_r(), si = acc0.res_i();
    if (!grid_sum<Val, !NT, B>(sr, si, a, a.gen0 + 1u, sh))
        return;
    for (uint64_t it = 0; it < a.iters; ++it) {
        const double mr = (double(sr) * 2.0) / a.N, mi = (double(si) * 2.0) / a.N;
        A acc;
        chunk_pass<T, A, true, NT, U32>(a, slow_tiles, table, mr, mi, acc, held, rt);
        sr = acc.res_r();
        si = acc.res_i();
        if (!grid_sum<Val, !NT, B>(sr, si, a, a.gen0 + 2u + it, sh))
            return;
    }
    if (a.iters > 0) {  // the held tiles go back to memory
        using V = typename T::vec;
        for (uint64_t j = held_start<T>(cnt); j < reg_start<T>(cnt); ++j) {
            const V *hv = held + (j - held_start<T>(cnt)) * kTile;
            const uint64_t v0 = (blockIdx.x + j * gridDim.x) * kTile;
            const auto rs = tile_rsrc<V>(a.state, a.nvec, v0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t v = v0 + u * B + threadIdx.x;
                if (v < a.nvec)
                    bstore16<Shape<T>::store_nt>(hv[u * B + threadIdx.x], rs, lane_off<B>(u, threadIdx.x));
            }
        }
#pragma unroll
        for (int r = 0; r < reg_tiles<T>(); ++r) {
            const uint64_t j = reg_start<T>(cnt) + uint64_t(r);
            if (j < cnt) {
                const uint64_t v0 = (blockIdx.x + j * gridDim.x) * kTile;
                const auto rs = tile_rsrc<V>(a.state, a.nvec, v0);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint64_t v = v0 + u * B + threadIdx.x;
                    if (v < a.nvec)
                        bstore16<Shape<T>::store_nt>(rt[r][u], rs, lane_off<B>(u, threadIdx.x));
                }
            }
        }
    }
}

template <class A, bool CHECK, bool NT>
const void *pick_storage(uint32_t dtype)
{
    switch (dtype) {
    case GROVER_F64_REAL: return reinterpret_cast<const void *>(&fused_iterate_kernel<F64Real, A, CHECK, NT, false>);
    case GROVER_C64: return reinterpret_cast<const void *>(&fused_iterate_kernel<C64, A, CHECK, NT, false>);
    case GROVER_C128: return reinterpret_cast<const void *>(&fused_iterate_kernel<C128, A, CHECK, NT, false>);
    case GROVER_CBF16: return reinterpret_cast<const void *>(&fused_iterate_kernel<CBF16, A, CHECK, NT, false>);
    default: return nullptr;
    }
}

template <bool CHECK, bool NT>
const void *kernel_for_access(uint32_t dtype, uint32_t accum, uint32_t update)
{
    if (update == GROVER_UPDATE_F32)  // complex64 storage with binary64 sums only
        return dtype == GROVER_C64 && accum == GROVER_ACC_F64
                   ? reinterpret_cast<const void *>(&fused_iterate_kernel<C64, AccF64, CHECK, NT, true>)
                   : nullptr;
    switch (accum) {
    case GROVER_ACC_F64: return pick_storage<AccF64, CHECK, NT>(dtype);
    case GROVER_ACC_F32: return pick_storage<AccF32, CHECK, NT>(dtype);
    case GROVER_ACC_F32_KAHAN: return pick_storage<AccF32Kahan, CHECK, NT>(dtype);
    default: return nullptr;
    }
}

template <bool CHECK>
const void *kernel_for(uint32_t dtype, uint32_t accum, bool temporal, uint32_t update = GROVER_UPDATE_F64)
{
    return temporal ? kernel_for_access<CHECK, false>(dtype, accum, update)
                    : kernel_for_access<CHECK, true>(dtype, accum, update);
}

// Bytes of the state per pass streamed with ordinary (temporal) loads and stores, so that the next pass
// finds them in MI355X's 256 MB memory-side cache; the rest streams with nontemporal accesses, which keep it
// from evicting them.  A state no larger streams entirely with ordinary accesses: one optimal search at
// n = 23, 24, 25 (complex64: 64, 128, 256 MiB) took 10 %, 7 % and 16 % less time than with nontemporal
// ones.  At n = 28 the first 17 tiles of each workgroup's share (272 MiB on 256 workgroups) cut the time per
// iteration the most: on one box 17 tiles 292.3-293.3 ms per 400 iterations, 16 295.4, 18 294.4, 19 296.3;
// on another 16 tiles -1.2 % and 18 -1.9 % against none, 20 tiles nothing, all tiles +6 %.  17 keeps a
// margin below the size where the gain vanishes.
constexpr uint64_t kTemporalBytes = uint64_t(272) << 20;

// Threads per workgroup of the fused kernel for a storage type.
int fused_block(uint32_t dtype)
{
    return dtype == GROVER_CBF16 ? Shape<CBF16>::block : Shape<C64>::block;
}

}  // namespace

hipError_t fused_configure(grover_ctx *c, int *per_cu, int *block, int64_t *forced_grid)
{
    const uint64_t state_bytes = c->N * elem_bytes(c->dtype);
    uint64_t budget = kTemporalBytes;
    if (const char *env = getenv("GROVER_FUSED_TEMPORAL")) {
        if (env[0] == '0')
            budget = 0;  // every access nontemporal
        else if (env[0] == '1')
            budget = state_bytes;  // every access ordinary
    }
    const bool temporal = state_bytes <= budget;
    const void *k = kernel_for<false>(c->dtype, c->accum, temporal, c->update);
    if (!k)
        return hipErrorInvalidValue;
    c->fused_kernel = k;
    c->fused_check_kernel = kernel_for<true>(c->dtype, c->accum, temporal, c->update);
    c->fused_temporal_bytes = temporal ? state_bytes : budget;
    c->fused_tile = kTile;
    int coop = 0;
    hipError_t e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c->device);
    if (e != hipSuccess)
        return e;
    if (!coop)
        return hipErrorCooperativeLaunchTooLarge;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k, fused_block(c->dtype), 0);
    if (e != hipSuccess)
        return e;
    *block = fused_block(c->dtype);
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

uint64_t fused_tiles_of(uint32_t dtype, uint64_t N)
{
    const uint64_t nvec = N / elems_per_vec(dtype);
    return (nvec + kTile - 1) / kTile;
}

hipError_t launch_fused_external(const FusedExternal &x)
{
    const uint64_t state_bytes = x.N * elem_bytes(x.dtype);
    const bool temporal = state_bytes <= kTemporalBytes;
    const void *fn = kernel_for<false>(x.dtype, GROVER_ACC_F64, temporal);
    if (!fn || x.grid < 1)
        return hipErrorInvalidValue;
    FusedArgs a;
    a.state = x.state;
    a.nvec = x.N / elems_per_vec(x.dtype);
    a.N = double(x.N);
    a.marks = x.marks;
    a.m = x.m;
    a.partials = x.slots;
    a.sync = x.sync;
    a.iters = x.k;
    a.gen0 = 0;
    a.timeout_ticks = x.timeout_ticks;
    a.temporal_tiles = kTemporalBytes / (uint64_t(x.grid) * kTile * 16u);
    void *args[] = {&a};
    return hipLaunchCooperativeKernel(fn, dim3(x.grid), dim3(fused_block(x.dtype)), args, 0, x.stream);
}

uint64_t fused_tiles(const grover_ctx *c)
{
    const uint64_t nvec = c->N / elems_per_vec(c->dtype);
    return (nvec + c->fused_tile - 1) / c->fused_tile;
}

uint64_t fused_temporal_tiles(const grover_ctx *c)
{
    const uint64_t share = uint64_t(c->grid > 0 ? c->grid : 1) * kTile * 16u;  // bytes of one tile per workgroup
    return c->fused_temporal_bytes / share;
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
    a.temporal_tiles = fused_temporal_tiles(c);
    void *args[] = {&a};
    const void *fn = check ? c->fused_check_kernel : c->fused_kernel;
    const hipError_t e = hipLaunchCooperativeKernel(fn, dim3(c->grid), dim3(c->block), args, 0, c->stream);
    if (e == hipSuccess)
        c->generation += k + 1u;
    return e;
}

}  // namespace grover
