// Device code shared by the batched and the phase kernels: the team barrier that also reduces the
// iteration's sum, the marked-tile table, and one streaming pass of a team's share of a state.  A "team"
// is T workgroups of one launch (rank 0 .. T-1) that iterate one state together.  The single-state fused
// kernel keeps its own copy of the same pass and barrier specialised to the whole grid: written against
// these generic helpers (team rank and size as run-time values) the compiler scheduled the tile loop's
// loads less well and the n = 28 iteration ran 4 % slower on MI355X.
#pragma once

#include "internal.h"

namespace grover {

constexpr int kStreamBlock = 1024;  // one workgroup per CU: fewest barrier participants, 16 waves per CU
constexpr int kStreamUnroll = 4;    // 16-byte vectors per thread per tile
constexpr int kStreamTile = kStreamBlock * kStreamUnroll;
constexpr int kMarkWords = 1024;    // LDS bitmap of a workgroup's tiles that hold marked amplitudes
constexpr int kTileMarks = 8;       // marks of one tile held in registers

template <class V>
struct TeamShared {
    V red[2][2 * (kStreamBlock / kWave)];  // per-wave partials, double-buffered (see block_allsum)
    V sum[2];
    int failed;
};

// The 16 wave values of a 1024-thread workgroup, (re, im) interleaved in red[0 .. 32), added as a balanced
// tree (four levels of dependent additions instead of fifteen).
template <class V>
__device__ inline void add_wave_values(const V *red, V &sr, V &si)
{
    V r[kStreamBlock / kWave], i[kStreamBlock / kWave];
#pragma unroll
    for (unsigned w = 0; w < kStreamBlock / kWave; ++w) {
        r[w] = red[2 * w];
        i[w] = red[2 * w + 1];
    }
#pragma unroll
    for (unsigned h = 1; h < kStreamBlock / kWave; h *= 2) {
#pragma unroll
        for (unsigned w = 0; w < kStreamBlock / kWave; w += 2 * h) {
            r[w] += r[w + h];
            i[w] += i[w + h];
        }
    }
    sr = r[0];
    si = i[0];
}

// Where a team's barrier lives: its error word (GridSync), its member slots [2][T][4] (the member's partial
// sum as tagged words, see put_tagged; double-buffered by the generation's parity), the number of
// workgroups T, this workgroup's rank, and the wait limit.
struct Team {
    GridSync *sync;
    uint64_t *partials;
    unsigned size;
    unsigned rank;
    uint64_t timeout_ticks;
};

__device__ inline uint64_t load_bits(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void store_bits(uint64_t *p, double x)
{
    __hip_atomic_store(p, (uint64_t)__double_as_longlong(x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A binary64 value published as two self-validating 64-bit words: each carries 32 bits of the value in its
// high half and the barrier generation (mod 2^32) in its low half.  Each word is stored and loaded as one
// atomic access, so a reader that sees the current tag in both words has both halves of this generation's
// value, and no memory fence (which on this GPU writes back or invalidates a whole L2) is needed to order
// the value against a separate flag.  Slots are zeroed before a launch and generations start at 1.
__device__ inline void put_tagged(uint64_t *w, double x, uint32_t tag)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    __hip_atomic_store(w, (b & 0xFFFFFFFF00000000ull) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(w + 1, (b << 32) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline bool tagged_ready(const uint64_t *w, uint32_t tag, uint64_t &hi, uint64_t &lo)
{
    hi = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    lo = __hip_atomic_load(w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return uint32_t(hi) == tag && uint32_t(lo) == tag;
}

__device__ inline double tagged_value(uint64_t hi, uint64_t lo)
{
    return __longlong_as_double((long long)((hi & 0xFFFFFFFF00000000ull) | (lo >> 32)));
}

// Bounded wait for the two values (tagged words w[0..3]) of generation `tag`, giving up when the team's
// error word is set or the wall-clock limit passes (then setting the error word).
__device__ inline bool wait_pair(const uint64_t *w, uint32_t tag, const Team &tm, double &a, double &b)
{
    const uint64_t t0 = wall_clock64();
    uint64_t h0, l0, h1, l1;
    for (;;) {
        const bool ra = tagged_ready(w, tag, h0, l0);
        const bool rb = tagged_ready(w + 2, tag, h1, l1);
        if (ra && rb)
            break;
        if (__hip_atomic_load(&tm.sync->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
            return false;
        if (uint64_t(wall_clock64()) - t0 > tm.timeout_ticks) {
            __hip_atomic_store(&tm.sync->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    a = tagged_value(h0, l0);
    b = tagged_value(h1, l1);
    return true;
}

// Bounded wait for the value pairs of up to four slots w + 4 kWave i (i < cnt, slot i of a lane that gathers
// members lane + kWave i), polled together so that the wait ends one memory round trip after the last of
// them is published instead of one round trip per slot; same limits as wait_pair.
__device__ inline bool wait_pairs4(const uint64_t *w, unsigned cnt, uint32_t tag, const Team &tm, double (&a)[4],
                                   double (&b)[4])
{
    const uint64_t t0 = wall_clock64();
    const unsigned all = (1u << cnt) - 1u;
    unsigned done = 0u;  // bit i: slot i read
    for (;;) {
#pragma unroll
        for (unsigned i = 0; i < 4u; ++i) {
            if (i < cnt && ((done >> i) & 1u) == 0u) {
                const uint64_t *slot = w + uint64_t(i) * kWave * 4u;
                uint64_t h0, l0, h1, l1;
                const bool ra = tagged_ready(slot, tag, h0, l0);
                const bool rb = tagged_ready(slot + 2, tag, h1, l1);
                if (ra && rb) {
                    a[i] = tagged_value(h0, l0);
                    b[i] = tagged_value(h1, l1);
                    done |= 1u << i;
                }
            }
        }
        if (done == all)
            return true;
        if (__hip_atomic_load(&tm.sync->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
            return false;
        if (uint64_t(wall_clock64()) - t0 > tm.timeout_ticks) {
            __hip_atomic_store(&tm.sync->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Team-wide sum of (xr, xi) at barrier generation `gen` (1, 2, ... per barrier object; slots zeroed before
// the launch), in the arithmetic of V (binary64 or binary32; partials travel as binary64, which holds a
// binary32 exactly).  Returns false when the wait gave up (time limit, or another workgroup gave up); every
// thread of the workgroup gets the same answer and the sum in (xr, xi).
//
// An all-gather: every member publishes its partial in its own slot of the generation's parity as tagged
// words; then, in every member, wave 0 waits for the members' words of this generation (lane l for members
// l, l + 64, ...; in teams of more than 256 one thread per member) and the partials are added in a fixed
// order, so every member computes the same sum bit for bit after one memory round trip.  A member rewrites a slot of parity p only at generation g + 2:
// its partial for g + 1 depends on the sum of g, so its reads of generation g have returned before it
// publishes g + 1, and g + 2 follows only after every member's g + 1 has been seen.  (Arrivals counted
// with one atomic per member serialise at the counter's address, and a gather to one member followed by a
// broadcast costs two round trips.)  The team's workgroups share no other memory within a launch, so the
// barrier orders nothing but these values.
template <class V, bool kTogether = false>
__device__ bool team_sum(V &xr, V &xi, const Team &tm, uint64_t gen, TeamShared<V> &sh)
{
    const uint32_t tag = uint32_t(gen);
    uint64_t *slots = tm.partials + uint64_t(gen & 1u) * tm.size * 4u;
    const unsigned lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    // this member's partial: wave totals, then thread 0 adds the wave values by a fixed tree and publishes
    // it.  sh.red[0] is read by thread 0 only before the workgroup barrier below; a wave writes it again
    // only in the next call, after that barrier, so no barrier is needed behind the read.
    xr = wave_total(xr);
    xi = wave_total(xi);
    if (lane == 0) {
        sh.red[0][2 * wave] = xr;
        sh.red[0][2 * wave + 1] = xi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        V sr, si;
        add_wave_values(sh.red[0], sr, si);
        uint64_t *slot = slots + uint64_t(tm.rank) * 4u;
        put_tagged(slot, double(sr), tag);
        put_tagged(slot + 2, double(si), tag);
    }
    if (tm.size <= 4u * kWave) {
        // wave 0 gathers the members' partials (lane l waits for members l, l + 64, ... and adds them in that
        // order) and adds the lanes' values with wave_total, which leaves the same bits in every lane and in
        // every member; one workgroup barrier hands the sum on.  sh.sum and sh.failed are written again only
        // after the first barrier of the next call, which every thread reaches after reading them here.
        if (wave == 0) {
            V ar = V(0), ai = V(0);
            bool ok = true;
            if (kTogether && tm.size > kWave) {
                // 2 to 4 members per lane, waited for together and added in member order
                const unsigned cnt = lane < tm.size ? (tm.size - lane + kWave - 1u) / kWave : 0u;
                double a[4], b[4];
                ok = wait_pairs4(slots + uint64_t(lane) * 4u, cnt, tag, tm, a, b);
                for (unsigned i = 0; i < cnt && ok; ++i) {
                    ar += V(a[i]);
                    ai += V(b[i]);
                }
            } else {
                for (unsigned w = lane; w < tm.size && ok; w += kWave) {
                    double a = 0.0, b = 0.0;
                    ok = wait_pair(slots + uint64_t(w) * 4u, tag, tm, a, b);
                    ar += V(a);
                    ai += V(b);
                }
            }
            const V pr = wave_total(ar), pi = wave_total(ai);
            const bool failed = __any(!ok);
            if (lane == 0) {
                sh.sum[0] = pr;
                sh.sum[1] = pi;
                sh.failed = failed;
            }
        }
        __syncthreads();
        xr = sh.sum[0];
        xi = sh.sum[1];
        return !sh.failed;
    }
    V pr = V(0), pi = V(0);
    bool ok = true;
    for (unsigned w = threadIdx.x; w < tm.size; w += kStreamBlock) {
        double a = 0.0, b = 0.0;
        ok = ok && wait_pair(slots + uint64_t(w) * 4u, tag, tm, a, b);
        pr += V(a);
        pi += V(b);
    }
    const bool failed = __syncthreads_or(!ok) != 0;
    block_sum2(pr, pi, sh.red[1]);
    if (threadIdx.x == 0) {
        sh.sum[0] = pr;
        sh.sum[1] = pi;
    }
    __syncthreads();
    xr = sh.sum[0];
    xi = sh.sum[1];
    __syncthreads();  // sh.sum is rewritten by the next call before its first barrier on this path
    return !failed;
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

// Marked bits of the EPV amplitudes starting at element i, from up to kTileMarks marks held in registers
// (padded with ~0, which never equals an amplitude index).
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

// One team member's view of a state: its tiles are t = rank + j * size, j = 0, 1, ... (tiles of
// kStreamTile 16-byte vectors).  At any moment the team streams one contiguous window of the state, spread
// over all HBM channels, while each tile stays with the same workgroup (hence XCD) in every iteration.
template <class T>
struct Share {
    typename T::vec *st;
    uint64_t nvec;
    const uint64_t *marks;  // the state's sorted marked list
    uint64_t m;
    uint64_t rank;
    uint64_t size;
    __device__ uint64_t ntiles() const { return (nvec + kStreamTile - 1) / kStreamTile; }
    __device__ uint64_t count() const { return rank < ntiles() ? (ntiles() - rank + size - 1) / size : 0; }
};

// Table of this workgroup's tiles that hold marked amplitudes (bit j = tile rank + j * size), built by the
// whole workgroup.  Returns false when it cannot be used (too many tiles, or a marked list so long that
// scanning it per workgroup costs more than checking every tile); every tile then takes the checked path.
template <class T>
__device__ bool build_mark_table(const Share<T> &sh, uint32_t *table)
{
    const bool use = sh.count() <= uint64_t(kMarkWords) * 32u && sh.m <= uint64_t(64) * kStreamBlock;
    if (use) {
        for (unsigned w = threadIdx.x; w < kMarkWords; w += kStreamBlock)
            table[w] = 0u;
        __syncthreads();
        for (uint64_t q = threadIdx.x; q < sh.m; q += kStreamBlock) {
            const uint64_t t = sh.marks[q] / T::EPV / kStreamTile;
            if (t % sh.size == sh.rank) {
                const uint64_t j = t / sh.size;
                atomicOr(&table[j >> 5], 1u << (j & 31));
            }
        }
    }
    __syncthreads();
    return use;
}

enum PassMode { kAccumulate, kUpdate, kFill };

// One pass over the workgroup's tiles.  kUpdate: c' = 2S/N - s c written back (nontemporal) and s c' added
// to the accumulator; kAccumulate: s c added; kFill: `fill` written everywhere and s * fill added.  The
// per-thread order of the sum is identical in all modes, so a fresh sum of a stored state equals, bit for
// bit, the sum the pass that wrote it produced.  U32: the update in binary32 from 2S/N rounded to binary32
// (complex64 storage only); otherwise in binary64.
template <class T, class A, PassMode MODE, bool U32 = false>
__device__ inline void stream_pass(const Share<T> &sh, const uint32_t *table, bool use_table, double mr, double mi,
                                   const typename T::vec &fill, A &acc)
{
    using V = typename T::vec;
    const float mr32 = float(mr), mi32 = float(mi);
    auto update = [&](V &v, unsigned bits) {
        if constexpr (U32)
            update_vec_f32(v, mr32, mi32, bits, acc);
        else
            update_vec<T>(v, mr, mi, bits, acc);
    };
    const unsigned tid = threadIdx.x;
    const uint64_t cnt = sh.count();
    uint64_t mp = 0;  // marked entries before this position lie in tiles already visited
    for (uint64_t j = 0; j < cnt; ++j) {
        const uint64_t t = sh.rank + j * sh.size;
        const uint64_t v0 = t * kStreamTile;
        const bool full = v0 + kStreamTile <= sh.nvec;
        const bool marked = use_table ? ((table[j >> 5] >> (j & 31)) & 1u) != 0u : sh.m > 0;
        if (full && !marked) {
            V x[kStreamUnroll];
            if (MODE != kFill) {
#pragma unroll
                for (int u = 0; u < kStreamUnroll; ++u)
                    x[u] = load16<true>(sh.st + v0 + u * kStreamBlock + tid);
            }
#pragma unroll
            for (int u = 0; u < kStreamUnroll; ++u) {
                if (MODE == kUpdate) {
                    update(x[u], 0u);
                    store16<true>(x[u], sh.st + v0 + u * kStreamBlock + tid);
                } else if (MODE == kFill) {
                    store16<true>(fill, sh.st + v0 + u * kStreamBlock + tid);
                    accum_vec<T>(fill, 0u, acc);
                } else {
                    accum_vec<T>(x[u], 0u, acc);
                }
            }
        } else {
            // Ragged tail of the state, or a tile that may hold marked amplitudes: each amplitude's sign
            // comes from the tile's slice [mp, mq) of the sorted marked list.
            mp = gallop_lower_bound(sh.marks, mp, sh.m, v0 * T::EPV);
            const uint64_t mq = gallop_lower_bound(sh.marks, mp, sh.m, (v0 + kStreamTile) * T::EPV);
            const bool in_regs = mq - mp <= uint64_t(kTileMarks);
            uint64_t mk[kTileMarks];
#pragma unroll
            for (int q = 0; q < kTileMarks; ++q)
                mk[q] = in_regs && mp + q < mq ? sh.marks[mp + q] : ~uint64_t(0);
            V x[kStreamUnroll];
#pragma unroll
            for (int u = 0; u < kStreamUnroll; ++u) {
                const uint64_t v = v0 + u * kStreamBlock + tid;
                if (v < sh.nvec)
                    x[u] = MODE == kFill ? fill : load16<true>(sh.st + v);
            }
#pragma unroll
            for (int u = 0; u < kStreamUnroll; ++u) {
                const uint64_t v = v0 + u * kStreamBlock + tid;
                if (v < sh.nvec) {
                    const unsigned bits = in_regs ? bits_from_regs<T::EPV>(mk, v * T::EPV)
                                                  : marked_bits<T::EPV>(sh.marks, mp, mq, v * T::EPV);
                    if (MODE == kUpdate) {
                        update(x[u], bits);
                        store16<true>(x[u], sh.st + v);
                    } else {
                        if (MODE == kFill)
                            store16<true>(x[u], sh.st + v);
                        accum_vec<T>(x[u], bits, acc);
                    }
                }
            }
            mp = mq;
        }
    }
}

}  // namespace grover
