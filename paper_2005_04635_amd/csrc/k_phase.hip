// Generalized iteration with per-iteration phases, and its adjoint (reverse sweep) for the gradient.
//
// Iteration j (1 .. K) of schedule b applies O(phi_j) then D(theta_j), with
//   O(phi):   c_i <- e^{i phi} c_i on the marked indices (Algorithm 3 is phi = pi),
//   D(theta): c_i <- (1 - e^{i theta}) S / N - c_i with S the sum of the state (Eq. 2 is theta = pi),
// from the uniform superposition; the loss is L = 1 - sum over marked i of |c_i|^2.
//
// Forward: one pass per iteration, fused as in the plain kernel: the pass that writes c' = alpha - O c also
// accumulates the sum T of c' and the sum Mk of its marked entries, so the next iteration's
// S = sum O(phi') c' = T + (e^{i phi'} - 1) Mk needs no extra pass.  Every `every`-th state is also written
// to a checkpoint buffer.
//
// Adjoint: lambda = dL/d(conj c) starts as -g c on the marked entries (g = upstream gradient of L) and is
// carried back through the inverses of the unitary steps, D(theta)^-1 = D(-theta) and O(phi)^-1 = O(-phi),
// while the state is rebuilt backwards with the same inverses.  Step j needs the sums of c_j and
// lambda_j and yields, with y = O(phi_j) c_{j-1} = D(-theta_j) c_j and nu = D(-theta_j) lambda_j,
//   dL/dtheta_j = -2 Im( conj(sum lambda_j) * sum c_j ) / N,
//   dL/dphi_j   = -2 Im( sum over marked of conj(nu) * y ),
//   c_{j-1} = O(-phi_j) y,  lambda_{j-1} = O(-phi_j) nu,
// all in one pass that also accumulates the sums for step j - 1.  Where j - 1 is a checkpoint the state is
// re-read from it (the uniform state for j - 1 = 0) instead of being rebuilt, which bounds the drift of the
// rebuilt state to `every` steps.
//
// Storage is complex64 (float re, im); phases, sums and the element arithmetic are binary64.  A team of
// `team_size` workgroups iterates one schedule at a time, with one team barrier per iteration that also
// reduces six binary64 values; teams take schedules b = team, team + teams, ...
#include "phase.h"
#include "stream.h"

namespace grover {
namespace {

constexpr int kPV = 6;  // values a barrier reduces

struct C2 {
    double re, im;
};

__device__ inline C2 cmul(C2 a, C2 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

struct PhaseShared {
    double red[kPV * (kStreamBlock / kWave)];
    double sum[kPV];
    int failed;
};

struct PhaseTeam {
    PhaseSync *sync;
    uint64_t *partials;  // [2][size][16]: kPV values as tagged word pairs
    unsigned size;
    unsigned rank;
    uint64_t timeout_ticks;
};

// Workgroup sum of v[0 .. kPV): wave butterflies, then thread 0 adds the wave values in wave order.
__device__ inline void block_sum_n(double (&v)[kPV], PhaseShared &sh)
{
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
    for (int q = 0; q < kPV; ++q)
        v[q] = wave_total(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < kPV; ++q)
            sh.red[q * (kStreamBlock / kWave) + wave] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < kPV; ++q) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w)
                s += sh.red[q * (kStreamBlock / kWave) + w];
            v[q] = s;
        }
    }
    __syncthreads();
}

// Bounded wait until the first NV values of one member's slot carry generation `tag`, then adds them to w.
// False when the wait gave up (time limit, or another workgroup gave up).
template <int NV>
__device__ inline bool wait_slot_n(const uint64_t *slot, uint32_t tag, const PhaseTeam &tm, double (&w)[kPV])
{
    const uint64_t t0 = wall_clock64();
    uint64_t hi[NV], lo[NV];
    for (;;) {
        bool ready = true;
#pragma unroll
        for (int q = 0; q < NV; ++q)
            ready = tagged_ready(slot + 2 * q, tag, hi[q], lo[q]) && ready;
        if (ready)
            break;
        if (__hip_atomic_load(&tm.sync->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
            return false;
        if (uint64_t(wall_clock64()) - t0 > tm.timeout_ticks) {
            __hip_atomic_store(&tm.sync->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
#pragma unroll
    for (int q = 0; q < NV; ++q)
        w[q] += tagged_value(hi[q], lo[q]);
    return true;
}

// Team-wide sum of v[0 .. NV) (the other entries are left as they are), an all-gather as in the batched
// kernels' barrier: every member publishes its partials in its slot of the generation's parity as tagged
// words (two per value, each carrying the generation; see put_tagged); in every member the slots are
// awaited in parallel, one member per thread, until all of a member's words carry this generation, and the
// partials are added by a fixed tree, so all members compute identical sums.  Slots are double-buffered by
// parity (a slot is rewritten two generations later, after every member has read it).  Every thread gets
// the sums; false when the wait gave up.  Each value costs two more words to publish and to poll, so
// callers pass only the values the next step needs.  A member's partial: wave totals, then lane q of wave 0
// adds value q's 16 wave values by a tree and publishes it (the values in parallel).  For T <= 256 the
// gather is done by wave 0 alone (lane l adds members l, l + 64, ... in order) and the lanes' sums are added
// by wave totals (the same bits in every lane and member), so the barrier costs two workgroup barriers;
// LDS words are written again only after the first barrier of the next call, which every thread reaches
// after reading them.
template <int NV = kPV>
__device__ bool team_sum_n(double (&v)[kPV], const PhaseTeam &tm, uint64_t gen, PhaseShared &sh)
{
    static_assert(NV >= 1 && NV <= kPV, "values per barrier");
    constexpr unsigned kW = kStreamBlock / kWave;
    const uint32_t tag = uint32_t(gen);
    uint64_t *slots = tm.partials + uint64_t(gen & 1u) * tm.size * 16u;
    const unsigned lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < NV; ++q)
        v[q] = wave_total(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q)
            sh.red[q * kW + wave] = v[q];
    }
    __syncthreads();
    if (wave == 0 && lane < unsigned(NV)) {
        double r[kW];
#pragma unroll
        for (unsigned w = 0; w < kW; ++w)
            r[w] = sh.red[lane * kW + w];
#pragma unroll
        for (unsigned h = 1; h < kW; h *= 2)
#pragma unroll
            for (unsigned w = 0; w < kW; w += 2 * h)
                r[w] += r[w + h];
        put_tagged(slots + uint64_t(tm.rank) * 16u + 2 * lane, r[0], tag);
    }
    if (tm.size <= 4u * kWave) {
        if (wave == 0) {
            double w[kPV] = {};
            bool ok = true;
            for (unsigned r = lane; r < tm.size && ok; r += kWave)  // members lane, lane + 64, ... in order
                ok = wait_slot_n<NV>(slots + uint64_t(r) * 16u, tag, tm, w);
#pragma unroll
            for (int q = 0; q < NV; ++q)
                w[q] = wave_total(w[q]);
            const bool failed = __any(!ok);
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < NV; ++q)
                    sh.sum[q] = w[q];
                sh.failed = failed;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NV; ++q)
            v[q] = sh.sum[q];
        return sh.failed == 0;
    }
    double w[kPV] = {};
    bool ok = true;
    for (unsigned r = threadIdx.x; r < tm.size && ok; r += kStreamBlock)
        ok = wait_slot_n<NV>(slots + uint64_t(r) * 16u, tag, tm, w);
    const bool failed = __syncthreads_or(!ok) != 0;
    block_sum_n(w, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q)
            sh.sum[q] = w[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q)
        v[q] = sh.sum[q];
    __syncthreads();  // sh.sum is rewritten by the next call before its first barrier on this path
    return !failed;
}

struct PhaseArgs {
    float4 *state;   // [B][nvec]
    float4 *lambda;  // [B][nvec]
    float4 *ckpt;    // [B][nck][nvec]
    const uint64_t *marks;
    uint64_t m;
    uint64_t nvec;
    double N;
    float amp;  // uniform amplitude rounded to binary32
    uint32_t B, K, every, nck;
    const double *phi, *theta;  // [B][K]
    double *loss;               // [B]
    double *aux;                // [B][2] sum of the final state (forward -> adjoint)
    const double *dloss;        // [B]
    double *dphi, *dtheta;      // [B][K]
    PhaseSync *sync;            // one per team
    uint64_t *partials;         // [teams][2][T][8]
    uint32_t team_size;
    uint32_t probe;  // 1: only meet once at a barrier of the whole grid (residency check)
    uint64_t timeout_ticks;
};

// Marked entries of one tile: the slice [mp, mq) of the sorted list, held in registers when short.
struct TileMarks {
    uint64_t mp, mq;
    bool in_regs;
    uint64_t mk[kTileMarks];
    __device__ void load(const uint64_t *marks, uint64_t m, uint64_t v0)
    {
        mp = gallop_lower_bound(marks, mp, m, v0 * 2u);
        mq = gallop_lower_bound(marks, mp, m, (v0 + kStreamTile) * 2u);
        in_regs = mq - mp <= uint64_t(kTileMarks);
#pragma unroll
        for (int q = 0; q < kTileMarks; ++q)
            mk[q] = in_regs && mp + q < mq ? marks[mp + q] : ~uint64_t(0);
    }
    __device__ unsigned bits(const uint64_t *marks, uint64_t v) const
    {
        return in_regs ? bits_from_regs<2>(mk, v * 2u) : marked_bits<2>(marks, mp, mq, v * 2u);
    }
};

__device__ inline C2 lo(const float4 &x) { return {double(x.x), double(x.y)}; }
__device__ inline C2 hi(const float4 &x) { return {double(x.z), double(x.w)}; }
__device__ inline float4 pack(C2 a, C2 b) { return make_float4(float(a.re), float(a.im), float(b.re), float(b.im)); }

// The team-rank-th share of one state: tiles t = rank + j * size (kStreamTile vectors each).
__device__ inline uint64_t share_tiles(uint64_t nvec, unsigned rank, unsigned size)
{
    const uint64_t nt = (nvec + kStreamTile - 1) / kStreamTile;
    return rank < nt ? (nt - rank + size - 1) / size : 0;
}

// Does local tile j of this workgroup's share hold a marked amplitude?  From the LDS table when it could be
// built, otherwise assume it may (the tile then finds its marks by search).
__device__ inline bool tile_marked(const PhaseArgs &a, const uint32_t *table, bool use_table, uint64_t j)
{
    return use_table ? ((table[j >> 5] >> (j & 31)) & 1u) != 0u : a.m > 0;
}

// The table of this workgroup's tiles that hold marked amplitudes; every schedule shares the marked set and
// the tile assignment, so it is built once per launch.
__device__ inline bool build_phase_table(const PhaseArgs &a, const PhaseTeam &tm, uint32_t *table)
{
    const Share<C64> share{nullptr, a.nvec, a.marks, a.m, tm.rank, tm.size};
    return build_mark_table(share, table);
}

// Forward pass over a team's share.  mode 0: write the uniform state; mode 1: c' = alpha - O(phi) c.
// Accumulates v = {sum re, sum im, marked sum re, marked sum im, marked |c|^2, 0} of the values stored.
__device__ void forward_pass(const PhaseArgs &a, float4 *st, float4 *ck, const PhaseTeam &tm, const uint32_t *table,
                             bool use_table, int mode, C2 alpha, C2 ephi, double (&v)[kPV])
{
    const unsigned tid = threadIdx.x;
    const uint64_t cnt = share_tiles(a.nvec, tm.rank, tm.size);
    TileMarks tmk;
    tmk.mp = 0;
    for (uint64_t j = 0; j < cnt; ++j) {
        const uint64_t v0 = (tm.rank + j * tm.size) * uint64_t(kStreamTile);
        const bool fast = !tile_marked(a, table, use_table, j) && v0 + kStreamTile <= a.nvec;
        if (!fast)
            tmk.load(a.marks, a.m, v0);
        float4 x[kStreamUnroll];
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) {
            const uint64_t vi = v0 + u * kStreamBlock + tid;
            if (fast || vi < a.nvec)
                x[u] = mode == 0 ? make_float4(a.amp, 0.0f, a.amp, 0.0f) : load16<true>(st + vi);
        }
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) {
            const uint64_t vi = v0 + u * kStreamBlock + tid;
            if (!fast && vi >= a.nvec)
                continue;
            const unsigned bits = fast ? 0u : tmk.bits(a.marks, vi);
            float4 out;
            if (mode == 0) {
                out = x[u];
            } else {
                C2 c0 = lo(x[u]), c1 = hi(x[u]);
                if (bits & 1u)
                    c0 = cmul(ephi, c0);
                if (bits & 2u)
                    c1 = cmul(ephi, c1);
                out = pack({alpha.re - c0.re, alpha.im - c0.im}, {alpha.re - c1.re, alpha.im - c1.im});
            }
            store16<true>(out, st + vi);
            if (ck)
                store16<true>(out, ck + vi);
            const C2 r0 = lo(out), r1 = hi(out);
            v[0] += r0.re + r1.re;
            v[1] += r0.im + r1.im;
            if (bits & 1u) {
                v[2] += r0.re;
                v[3] += r0.im;
                v[4] += r0.re * r0.re + r0.im * r0.im;
            }
            if (bits & 2u) {
                v[2] += r1.re;
                v[3] += r1.im;
                v[4] += r1.re * r1.re + r1.im * r1.im;
            }
        }
        if (!fast)
            tmk.mp = tmk.mq;
    }
}

__global__ __launch_bounds__(kStreamBlock) void phase_forward_kernel(PhaseArgs a)
{
    __shared__ PhaseShared sh;
    __shared__ uint32_t table[kMarkWords];
    const unsigned T = a.team_size, teams = gridDim.x / T, team_id = blockIdx.x / T;
    if (team_id >= teams)
        return;
    const PhaseTeam tm{a.sync + team_id, a.partials + uint64_t(team_id) * 32u * T, T, blockIdx.x % T,
                       a.timeout_ticks};
    uint64_t gen = 0;
    if (a.probe) {
        double v[kPV] = {};
        (void)team_sum_n(v, tm, ++gen, sh);
        return;
    }
    const bool use_table = build_phase_table(a, tm, table);
    for (uint32_t b = team_id; b < a.B; b += teams) {
        float4 *st = a.state + uint64_t(b) * a.nvec;
        double v[kPV] = {};
        forward_pass(a, st, nullptr, tm, table, use_table, 0, {0.0, 0.0}, {1.0, 0.0}, v);
        if (!team_sum_n(v, tm, ++gen, sh))
            return;
        for (uint32_t k = 1; k <= a.K; ++k) {
            const double ph = a.phi[uint64_t(b) * a.K + k - 1], th = a.theta[uint64_t(b) * a.K + k - 1];
            const C2 ephi{cos(ph), sin(ph)}, eth{cos(th), sin(th)};
            // S = sum of O(phi) c = T + (e^{i phi} - 1) Mk;  alpha = (1 - e^{i theta}) S / N
            const C2 S = {v[0] + (ephi.re - 1.0) * v[2] - ephi.im * v[3], v[1] + (ephi.re - 1.0) * v[3] + ephi.im * v[2]};
            const C2 f = cmul({1.0 - eth.re, -eth.im}, S);
            const C2 alpha{f.re / a.N, f.im / a.N};
            float4 *ck = (k % a.every == 0 && k < a.K)
                             ? a.ckpt + (uint64_t(b) * a.nck + (k / a.every - 1u)) * a.nvec
                             : nullptr;
            double w[kPV] = {};
            forward_pass(a, st, ck, tm, table, use_table, 1, alpha, ephi, w);
            if (!team_sum_n(w, tm, ++gen, sh))
                return;
#pragma unroll
            for (int q = 0; q < kPV; ++q)
                v[q] = w[q];
        }
        if (tm.rank == 0 && threadIdx.x == 0) {
            a.loss[b] = 1.0 - v[4];
            a.aux[2u * b] = v[0];
            a.aux[2u * b + 1u] = v[1];
        }
    }
}

// Adjoint seed: lambda = -g c on the marked entries, 0 elsewhere; accumulates its sum into v[2], v[3].
__device__ void lambda_seed_pass(const PhaseArgs &a, const float4 *st, float4 *lam, const PhaseTeam &tm,
                                 const uint32_t *table, bool use_table, double g, double (&v)[kPV])
{
    const unsigned tid = threadIdx.x;
    const uint64_t cnt = share_tiles(a.nvec, tm.rank, tm.size);
    TileMarks tmk;
    tmk.mp = 0;
    for (uint64_t j = 0; j < cnt; ++j) {
        const uint64_t v0 = (tm.rank + j * tm.size) * uint64_t(kStreamTile);
        const bool marked = tile_marked(a, table, use_table, j);
        if (marked)
            tmk.load(a.marks, a.m, v0);
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) {
            const uint64_t vi = v0 + u * kStreamBlock + tid;
            if (vi >= a.nvec)
                continue;
            const unsigned bits = !marked || tmk.mq == tmk.mp ? 0u : tmk.bits(a.marks, vi);
            float4 out = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (bits) {
                const float4 x = st[vi];
                const C2 c0 = lo(x), c1 = hi(x);
                const C2 l0 = (bits & 1u) ? C2{-g * c0.re, -g * c0.im} : C2{0.0, 0.0};
                const C2 l1 = (bits & 2u) ? C2{-g * c1.re, -g * c1.im} : C2{0.0, 0.0};
                out = pack(l0, l1);
                const C2 r0 = lo(out), r1 = hi(out);
                v[2] += r0.re + r1.re;
                v[3] += r0.im + r1.im;
            }
            store16<true>(out, lam + vi);
        }
        if (marked)
            tmk.mp = tmk.mq;
    }
}

// One reverse step over a team's share (see the file comment).  src: the checkpoint to re-read c_{j-1}
// from, or null with anchor set for the uniform state, or anchor clear to rebuild from the state.
// Accumulates v = {sum c_{j-1}, sum lambda_{j-1}, sum over marked of conj(nu) y}.
__device__ void reverse_pass(const PhaseArgs &a, float4 *st, float4 *lam, const float4 *src, bool anchor,
                             const PhaseTeam &tm, const uint32_t *table, bool use_table, C2 beta_c, C2 beta_l,
                             C2 ephi, double (&v)[kPV])
{
    const unsigned tid = threadIdx.x;
    const uint64_t cnt = share_tiles(a.nvec, tm.rank, tm.size);
    const C2 emphi{ephi.re, -ephi.im};
    TileMarks tmk;
    tmk.mp = 0;
    for (uint64_t j = 0; j < cnt; ++j) {
        const uint64_t v0 = (tm.rank + j * tm.size) * uint64_t(kStreamTile);
        const bool fast = !tile_marked(a, table, use_table, j) && v0 + kStreamTile <= a.nvec;
        if (!fast)
            tmk.load(a.marks, a.m, v0);
        float4 xc[kStreamUnroll], xl[kStreamUnroll];
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) {
            const uint64_t vi = v0 + u * kStreamBlock + tid;
            if (fast || vi < a.nvec) {
                if (!anchor)
                    xc[u] = load16<true>(st + vi);
                else
                    xc[u] = src ? load16<true>(src + vi) : make_float4(a.amp, 0.0f, a.amp, 0.0f);
                xl[u] = load16<true>(lam + vi);
            }
        }
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) {
            const uint64_t vi = v0 + u * kStreamBlock + tid;
            if (!fast && vi >= a.nvec)
                continue;
            const unsigned bits = fast ? 0u : tmk.bits(a.marks, vi);
            C2 cp[2], lp[2];
            const C2 cin[2] = {lo(xc[u]), hi(xc[u])}, lin[2] = {lo(xl[u]), hi(xl[u])};
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const bool mk = (bits >> e) & 1u;
                C2 y;
                if (anchor) {
                    cp[e] = cin[e];
                    y = mk ? cmul(ephi, cin[e]) : cin[e];
                } else {
                    y = {beta_c.re - cin[e].re, beta_c.im - cin[e].im};
                    cp[e] = mk ? cmul(emphi, y) : y;
                }
                const C2 nu{beta_l.re - lin[e].re, beta_l.im - lin[e].im};
                lp[e] = mk ? cmul(emphi, nu) : nu;
                if (mk) {
                    // conj(nu) * y
                    v[4] += nu.re * y.re + nu.im * y.im;
                    v[5] += nu.re * y.im - nu.im * y.re;
                }
            }
            const float4 oc = pack(cp[0], cp[1]), ol = pack(lp[0], lp[1]);
            store16<true>(oc, st + vi);
            store16<true>(ol, lam + vi);
            v[0] += double(oc.x) + double(oc.z);
            v[1] += double(oc.y) + double(oc.w);
            v[2] += double(ol.x) + double(ol.z);
            v[3] += double(ol.y) + double(ol.w);
        }
        if (!fast)
            tmk.mp = tmk.mq;
    }
}

__global__ __launch_bounds__(kStreamBlock) void phase_adjoint_kernel(PhaseArgs a)
{
    __shared__ PhaseShared sh;
    __shared__ uint32_t table[kMarkWords];
    const unsigned T = a.team_size, teams = gridDim.x / T, team_id = blockIdx.x / T;
    if (team_id >= teams)
        return;
    const PhaseTeam tm{a.sync + team_id, a.partials + uint64_t(team_id) * 32u * T, T, blockIdx.x % T,
                       a.timeout_ticks};
    uint64_t gen = 0;
    if (a.probe) {
        double v[kPV] = {};
        (void)team_sum_n(v, tm, ++gen, sh);
        return;
    }
    const bool leader = tm.rank == 0 && threadIdx.x == 0;
    const bool use_table = build_phase_table(a, tm, table);
    for (uint32_t b = team_id; b < a.B; b += teams) {
        float4 *st = a.state + uint64_t(b) * a.nvec;
        float4 *lam = a.lambda + uint64_t(b) * a.nvec;
        double v[kPV] = {};
        lambda_seed_pass(a, st, lam, tm, table, use_table, a.dloss[b], v);
        if (!team_sum_n(v, tm, ++gen, sh))
            return;
        C2 sc{a.aux[2u * b], a.aux[2u * b + 1u]}, sl{v[2], v[3]};
        for (uint32_t k = a.K; k >= 1; --k) {
            const uint64_t pk = uint64_t(b) * a.K + k - 1;
            const double ph = a.phi[pk], th = a.theta[pk];
            if (leader)  // -2 Im(conj(sum lambda) * sum c) / N
                a.dtheta[pk] = -2.0 * (sl.re * sc.im - sl.im * sc.re) / a.N;
            const C2 emth{cos(th), -sin(th)};
            const C2 om{1.0 - emth.re, -emth.im};
            const C2 fc = cmul(om, sc), fl = cmul(om, sl);
            const C2 beta_c{fc.re / a.N, fc.im / a.N}, beta_l{fl.re / a.N, fl.im / a.N};
            const bool anchor = (k - 1u) % a.every == 0u;
            const float4 *src = (anchor && k - 1u > 0u)
                                    ? a.ckpt + (uint64_t(b) * a.nck + ((k - 1u) / a.every - 1u)) * a.nvec
                                    : nullptr;
            double w[kPV] = {};
            reverse_pass(a, st, lam, src, anchor, tm, table, use_table, beta_c, beta_l, {cos(ph), sin(ph)}, w);
            if (!team_sum_n(w, tm, ++gen, sh))
                return;
            if (leader)  // -2 Im(sum over marked of conj(nu) y)
                a.dphi[pk] = -2.0 * w[5];
            sc = {w[0], w[1]};
            sl = {w[2], w[3]};
        }
    }
}

// ------------------------------------------------------------------------------ on-chip form
// For states small enough to stay on chip the same iteration and reverse sweep run with each state held in
// its team's registers and LDS for all K steps, so that the only memory traffic is the checkpoints, the
// final state and the reads of the checkpoints in the reverse sweep.  Team size T (a power of two, set by
// the host from the state size): member `rank` owns the contiguous vectors [rank * per, (rank + 1) * per),
// per = nvec / T, and thread tid the vectors rank * per + e * 1024 + tid, e < ne = per / 1024 (or, when
// per < 1024, the one vector tid < per).  Forward: up to 16 vectors per thread, 8 in registers and 8 in
// its own LDS slots.  Adjoint: up to 8 vectors of the state in registers and 8 of the adjoint state in LDS.
// The marked set is the same for every schedule and step, so each thread finds the marked bits of its
// vectors once per launch (two per vector, packed); threads without marks take a shorter update.
constexpr int kHeldReg = 8;
constexpr int kHeldLds = 8;

struct HeldShare {
    uint64_t base, per;
    unsigned ne;
    bool active;
};

__device__ inline HeldShare held_share(uint64_t nvec, const PhaseTeam &tm)
{
    HeldShare h;
    h.per = nvec / tm.size;
    h.base = uint64_t(tm.rank) * h.per;
    h.ne = h.per >= kStreamBlock ? unsigned(h.per / kStreamBlock) : 1u;
    h.active = threadIdx.x < h.per;
    return h;
}

__device__ inline uint32_t held_mask(const PhaseArgs &a, const HeldShare &h)
{
    uint32_t mask = 0u;
    if (h.active && a.m > 0)
        for (unsigned e = 0; e < h.ne; ++e) {
            const uint64_t v = h.base + uint64_t(e) * kStreamBlock + threadIdx.x;
            mask |= uint32_t(marked_bits<2>(a.marks, 0, a.m, v * 2u)) << (2 * e);
        }
    return mask;
}

// e^{i phi_k} and e^{i theta_k} of one schedule for a chunk of kTrigChunk steps, computed once by the
// workgroup's threads (step k0 + i by thread i) into LDS instead of at every step by every thread: on chip a
// step costs a few microseconds, and binary64 sine and cosine plus the loads of the phases would be a large
// part of that.  Entry i holds {cos phi, sin phi, cos theta, sin theta} of step k0 + i (0-based).  Called by
// every thread at the same step; the barrier at its end publishes the table, and the table is rewritten
// only after the next team barrier, which every thread reaches after its last read of the old entries.
constexpr uint32_t kTrigChunk = 512;

struct TrigTable {
    double v[4][kTrigChunk];
};

__device__ inline void fill_trig(const PhaseArgs &a, uint32_t b, uint32_t k0, TrigTable &t)
{
    for (uint32_t i = threadIdx.x; i < kTrigChunk && k0 + i < a.K; i += kStreamBlock) {
        const uint64_t pk = uint64_t(b) * a.K + k0 + i;
        double sp, cp, sth, cth;
        sincos(a.phi[pk], &sp, &cp);
        sincos(a.theta[pk], &sth, &cth);
        t.v[0][i] = cp;
        t.v[1][i] = sp;
        t.v[2][i] = cth;
        t.v[3][i] = sth;
    }
    __syncthreads();
}

// One forward step of one held vector: c' = alpha - O(phi) c; the stored values' sums go to w
// ({sum, marked sum, marked |c|^2}, as forward_pass).  kMarks = false: the vector holds no marked amplitude.
template <bool kMarks>
__device__ inline void held_forward_vec(float4 &x, unsigned bits, C2 alpha, C2 ephi, double (&w)[kPV])
{
    if (!kMarks || bits == 0u) {
        x.x = float(alpha.re - double(x.x));
        x.y = float(alpha.im - double(x.y));
        x.z = float(alpha.re - double(x.z));
        x.w = float(alpha.im - double(x.w));
        w[0] += double(x.x) + double(x.z);
        w[1] += double(x.y) + double(x.w);
        return;
    }
    C2 c0 = lo(x), c1 = hi(x);
    if (bits & 1u)
        c0 = cmul(ephi, c0);
    if (bits & 2u)
        c1 = cmul(ephi, c1);
    x = pack({alpha.re - c0.re, alpha.im - c0.im}, {alpha.re - c1.re, alpha.im - c1.im});
    const C2 r0 = lo(x), r1 = hi(x);
    w[0] += r0.re + r1.re;
    w[1] += r0.im + r1.im;
    if (bits & 1u) {
        w[2] += r0.re;
        w[3] += r0.im;
        w[4] += r0.re * r0.re + r0.im * r0.im;
    }
    if (bits & 2u) {
        w[2] += r1.re;
        w[3] += r1.im;
        w[4] += r1.re * r1.re + r1.im * r1.im;
    }
}

// One forward step over a thread's held vectors (registers, then LDS), each also written to the checkpoint
// `ck` (this member's part of it) when one is due.
template <bool kMarks>
__device__ inline void held_forward_sweep(float4 (&x)[kHeldReg], float4 *held, const HeldShare &h, uint32_t mask,
                                          C2 alpha, C2 ephi, float4 *ck, double (&w)[kPV])
{
    const unsigned tid = threadIdx.x;
#pragma unroll
    for (int e = 0; e < kHeldReg; ++e)
        if (unsigned(e) < h.ne) {
            held_forward_vec<kMarks>(x[e], (mask >> (2 * e)) & 3u, alpha, ephi, w);
            if (ck)
                store16<true>(x[e], ck + uint64_t(e) * kStreamBlock + tid);
        }
    if (h.ne > unsigned(kHeldReg)) {
#pragma unroll
        for (int e = 0; e < kHeldLds; ++e) {
            float4 y = held[e * kStreamBlock + tid];
            held_forward_vec<kMarks>(y, (mask >> (2 * (kHeldReg + e))) & 3u, alpha, ephi, w);
            held[e * kStreamBlock + tid] = y;
            if (ck)
                store16<true>(y, ck + uint64_t(kHeldReg + e) * kStreamBlock + tid);
        }
    }
}

__global__ __launch_bounds__(kStreamBlock) void phase_forward_held_kernel(PhaseArgs a)
{
    __shared__ PhaseShared sh;
    __shared__ float4 held[kHeldLds * kStreamBlock];
    __shared__ TrigTable trig;
    const unsigned T = a.team_size, teams = gridDim.x / T, team_id = blockIdx.x / T;
    if (team_id >= teams)
        return;
    const PhaseTeam tm{a.sync + team_id, a.partials + uint64_t(team_id) * 32u * T, T, blockIdx.x % T,
                       a.timeout_ticks};
    uint64_t gen = 0;
    if (a.probe) {
        double v[kPV] = {};
        (void)team_sum_n(v, tm, ++gen, sh);
        return;
    }
    const unsigned tid = threadIdx.x;
    const HeldShare h = held_share(a.nvec, tm);
    const uint32_t mask = held_mask(a, h);
    const double inv_n = 1.0 / a.N;  // N is a power of two: x * (1/N) rounds as x / N
    const float4 fill = make_float4(a.amp, 0.0f, a.amp, 0.0f);
    for (uint32_t b = team_id; b < a.B; b += teams) {
        float4 *st = a.state + uint64_t(b) * a.nvec + h.base;
        float4 x[kHeldReg];
        double v[kPV] = {};
        if (h.active) {
#pragma unroll
            for (int e = 0; e < kHeldReg; ++e)
                x[e] = fill;
            if (h.ne > unsigned(kHeldReg))
#pragma unroll
                for (int e = 0; e < kHeldLds; ++e)
                    held[e * kStreamBlock + tid] = fill;
            // the sums of the uniform state, as the first pass of the streamed form computes them
            for (unsigned e = 0; e < h.ne; ++e) {
                const unsigned bits = (mask >> (2 * e)) & 3u;
                const C2 r{double(a.amp), 0.0};
                v[0] += r.re + r.re;
                v[1] += r.im + r.im;
                for (unsigned q = 0; q < 2; ++q)
                    if ((bits >> q) & 1u) {
                        v[2] += r.re;
                        v[3] += r.im;
                        v[4] += r.re * r.re + r.im * r.im;
                    }
            }
        }
        // the next step needs the total and the marked sum (4 values); the last one also the marked |c|^2
        if (!team_sum_n<4>(v, tm, ++gen, sh))
            return;
        for (uint32_t k = 1; k <= a.K; ++k) {
            const uint32_t i = (k - 1u) % kTrigChunk;
            if (i == 0u)
                fill_trig(a, b, k - 1u, trig);
            const C2 ephi{trig.v[0][i], trig.v[1][i]}, eth{trig.v[2][i], trig.v[3][i]};
            const C2 S = {v[0] + (ephi.re - 1.0) * v[2] - ephi.im * v[3], v[1] + (ephi.re - 1.0) * v[3] + ephi.im * v[2]};
            const C2 f = cmul({1.0 - eth.re, -eth.im}, S);
            const C2 alpha{f.re * inv_n, f.im * inv_n};
            float4 *ck = (k % a.every == 0 && k < a.K)
                             ? a.ckpt + (uint64_t(b) * a.nck + (k / a.every - 1u)) * a.nvec + h.base
                             : nullptr;
            double w[kPV] = {};
            if (h.active) {
                if (mask == 0u)
                    held_forward_sweep<false>(x, held, h, mask, alpha, ephi, ck, w);
                else
                    held_forward_sweep<true>(x, held, h, mask, alpha, ephi, ck, w);
            }
            if (!(k == a.K ? team_sum_n<5>(w, tm, ++gen, sh) : team_sum_n<4>(w, tm, ++gen, sh)))
                return;
#pragma unroll
            for (int q = 0; q < kPV; ++q)
                v[q] = w[q];
        }
        // the final state goes to memory: the adjoint starts from it, and it is the result
        if (h.active) {
#pragma unroll
            for (int e = 0; e < kHeldReg; ++e)
                if (unsigned(e) < h.ne)
                    store16<true>(x[e], st + uint64_t(e) * kStreamBlock + tid);
            if (h.ne > unsigned(kHeldReg))
#pragma unroll
                for (int e = 0; e < kHeldLds; ++e)
                    store16<true>(held[e * kStreamBlock + tid], st + uint64_t(kHeldReg + e) * kStreamBlock + tid);
        }
        if (tm.rank == 0 && tid == 0) {
            a.loss[b] = 1.0 - v[4];
            a.aux[2u * b] = v[0];
            a.aux[2u * b + 1u] = v[1];
        }
    }
}

// One reverse step of one held pair (state vector xc, adjoint vector xl), as reverse_pass: with anchor set
// the state c_{j-1} is given (cin: a checkpoint or the uniform state) instead of being rebuilt.
template <bool kMarks>
__device__ inline void held_reverse_vec(float4 &xc, float4 &xl, const float4 &cin, bool anchor, unsigned bits,
                                        C2 beta_c, C2 beta_l, C2 ephi, double (&w)[kPV])
{
    if (!kMarks || bits == 0u) {
        if (anchor) {
            xc = cin;
        } else {
            xc.x = float(beta_c.re - double(xc.x));
            xc.y = float(beta_c.im - double(xc.y));
            xc.z = float(beta_c.re - double(xc.z));
            xc.w = float(beta_c.im - double(xc.w));
        }
        xl.x = float(beta_l.re - double(xl.x));
        xl.y = float(beta_l.im - double(xl.y));
        xl.z = float(beta_l.re - double(xl.z));
        xl.w = float(beta_l.im - double(xl.w));
    } else {
        const C2 emphi{ephi.re, -ephi.im};
        C2 cp[2], lp[2];
        const C2 cs[2] = {lo(anchor ? cin : xc), hi(anchor ? cin : xc)}, ls[2] = {lo(xl), hi(xl)};
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const bool mk = (bits >> e) & 1u;
            C2 y;
            if (anchor) {
                cp[e] = cs[e];
                y = mk ? cmul(ephi, cs[e]) : cs[e];
            } else {
                y = {beta_c.re - cs[e].re, beta_c.im - cs[e].im};
                cp[e] = mk ? cmul(emphi, y) : y;
            }
            const C2 nu{beta_l.re - ls[e].re, beta_l.im - ls[e].im};
            lp[e] = mk ? cmul(emphi, nu) : nu;
            if (mk)  // Im(conj(nu) y), the only part the gradient uses
                w[4] += nu.re * y.im - nu.im * y.re;
        }
        xc = pack(cp[0], cp[1]);
        xl = pack(lp[0], lp[1]);
    }
    w[0] += double(xc.x) + double(xc.z);
    w[1] += double(xc.y) + double(xc.w);
    w[2] += double(xl.x) + double(xl.z);
    w[3] += double(xl.y) + double(xl.w);
}

template <bool kMarks>
__device__ inline void held_reverse_sweep(float4 (&xc)[kHeldReg], float4 *held, const HeldShare &h, uint32_t mask,
                                          const float4 *src, bool anchor, float amp, C2 beta_c, C2 beta_l, C2 ephi,
                                          double (&w)[kPV])
{
    const unsigned tid = threadIdx.x;
    const float4 uniform = make_float4(amp, 0.0f, amp, 0.0f);
#pragma unroll
    for (int e = 0; e < kHeldReg; ++e)
        if (unsigned(e) < h.ne) {
            const float4 cin = anchor && src ? load16<true>(src + uint64_t(e) * kStreamBlock + tid) : uniform;
            float4 xl = held[e * kStreamBlock + tid];
            held_reverse_vec<kMarks>(xc[e], xl, cin, anchor, (mask >> (2 * e)) & 3u, beta_c, beta_l, ephi, w);
            held[e * kStreamBlock + tid] = xl;
        }
}

__global__ __launch_bounds__(kStreamBlock) void phase_adjoint_held_kernel(PhaseArgs a)
{
    __shared__ PhaseShared sh;
    __shared__ float4 held[kHeldLds * kStreamBlock];  // the adjoint state
    __shared__ TrigTable trig;
    const unsigned T = a.team_size, teams = gridDim.x / T, team_id = blockIdx.x / T;
    if (team_id >= teams)
        return;
    const PhaseTeam tm{a.sync + team_id, a.partials + uint64_t(team_id) * 32u * T, T, blockIdx.x % T,
                       a.timeout_ticks};
    uint64_t gen = 0;
    if (a.probe) {
        double v[kPV] = {};
        (void)team_sum_n(v, tm, ++gen, sh);
        return;
    }
    const unsigned tid = threadIdx.x;
    const bool leader = tm.rank == 0 && tid == 0;
    const HeldShare h = held_share(a.nvec, tm);
    const uint32_t mask = held_mask(a, h);
    const double inv_n = 1.0 / a.N;
    for (uint32_t b = team_id; b < a.B; b += teams) {
        float4 *st = a.state + uint64_t(b) * a.nvec + h.base;
        const double g = a.dloss[b];
        float4 xc[kHeldReg];
        double v[kPV] = {};
        // the final state of the forward run, and the seed lambda = -g c on the marked entries
        if (h.active) {
#pragma unroll
            for (int e = 0; e < kHeldReg; ++e)
                if (unsigned(e) < h.ne) {
                    xc[e] = load16<true>(st + uint64_t(e) * kStreamBlock + tid);
                    const unsigned bits = (mask >> (2 * e)) & 3u;
                    float4 out = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    if (bits) {
                        const C2 c0 = lo(xc[e]), c1 = hi(xc[e]);
                        const C2 l0 = (bits & 1u) ? C2{-g * c0.re, -g * c0.im} : C2{0.0, 0.0};
                        const C2 l1 = (bits & 2u) ? C2{-g * c1.re, -g * c1.im} : C2{0.0, 0.0};
                        out = pack(l0, l1);
                        const C2 r0 = lo(out), r1 = hi(out);
                        v[2] += r0.re + r1.re;
                        v[3] += r0.im + r1.im;
                    }
                    held[e * kStreamBlock + tid] = out;
                }
        }
        if (!team_sum_n<4>(v, tm, ++gen, sh))  // the seed's sum, in v[2], v[3]
            return;
        C2 sc{a.aux[2u * b], a.aux[2u * b + 1u]}, sl{v[2], v[3]};
        for (uint32_t k = a.K; k >= 1; --k) {
            const uint64_t pk = uint64_t(b) * a.K + k - 1;
            // the table covers the chunk of step k - 1 (0-based); refilled on entering a chunk from above
            const uint32_t i = (k - 1u) % kTrigChunk;
            if (k == a.K || i == kTrigChunk - 1u)
                fill_trig(a, b, k - 1u - i, trig);
            if (leader)  // -2 Im(conj(sum lambda) * sum c) / N
                a.dtheta[pk] = -2.0 * (sl.re * sc.im - sl.im * sc.re) / a.N;
            const C2 emth{trig.v[2][i], -trig.v[3][i]};
            const C2 om{1.0 - emth.re, -emth.im};
            const C2 fc = cmul(om, sc), fl = cmul(om, sl);
            const C2 beta_c{fc.re * inv_n, fc.im * inv_n}, beta_l{fl.re * inv_n, fl.im * inv_n};
            const bool anchor = (k - 1u) % a.every == 0u;
            const float4 *src = (anchor && k - 1u > 0u)
                                    ? a.ckpt + (uint64_t(b) * a.nck + ((k - 1u) / a.every - 1u)) * a.nvec + h.base
                                    : nullptr;
            double w[kPV] = {};
            if (h.active) {
                const C2 ephi{trig.v[0][i], trig.v[1][i]};
                if (mask == 0u)
                    held_reverse_sweep<false>(xc, held, h, mask, src, anchor, a.amp, beta_c, beta_l, ephi, w);
                else
                    held_reverse_sweep<true>(xc, held, h, mask, src, anchor, a.amp, beta_c, beta_l, ephi, w);
            }
            // sum c, sum lambda and Im(sum over marked of conj(nu) y): 5 values
            if (!team_sum_n<5>(w, tm, ++gen, sh))
                return;
            if (leader)  // -2 Im(sum over marked of conj(nu) y)
                a.dphi[pk] = -2.0 * w[4];
            sc = {w[0], w[1]};
            sl = {w[2], w[3]};
        }
        // back at the uniform state: written out, as the streamed form leaves it
        if (h.active)
#pragma unroll
            for (int e = 0; e < kHeldReg; ++e)
                if (unsigned(e) < h.ne)
                    store16<true>(xc[e], st + uint64_t(e) * kStreamBlock + tid);
    }
}

// Zeroes the team barriers and the member slots (whose generation tags the barriers compare against)
// before a launch — a kernel, so that launches can be captured and replayed.
__global__ void phase_reset_kernel(uint64_t *words, uint64_t nwords, uint64_t *slots, uint64_t nslots)
{
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t w = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; w < nwords; w += stride)
        words[w] = 0u;
    for (uint64_t w = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; w < nslots; w += stride)
        slots[w] = 0u;
}

}  // namespace

const void *phase_kernel_fn(bool adjoint, bool held)
{
    if (held)
        return adjoint ? reinterpret_cast<const void *>(&phase_adjoint_held_kernel)
                       : reinterpret_cast<const void *>(&phase_forward_held_kernel);
    return adjoint ? reinterpret_cast<const void *>(&phase_adjoint_kernel)
                   : reinterpret_cast<const void *>(&phase_forward_kernel);
}

hipError_t launch_phase(const PhaseLaunch &L, bool adjoint)
{
    PhaseArgs a;
    a.state = static_cast<float4 *>(L.state);
    a.lambda = static_cast<float4 *>(L.lambda);
    a.ckpt = static_cast<float4 *>(L.ckpt);
    a.marks = L.marks;
    a.m = L.m;
    a.nvec = L.nvec;
    a.N = L.N;
    a.amp = L.amp;
    a.B = L.B;
    a.K = L.K;
    a.every = L.every;
    a.nck = L.nck;
    a.phi = L.phi;
    a.theta = L.theta;
    a.loss = L.loss;
    a.aux = L.aux;
    a.dloss = L.dloss;
    a.dphi = L.dphi;
    a.dtheta = L.dtheta;
    a.sync = L.sync;
    a.partials = L.partials;
    a.team_size = L.team_size;
    a.probe = L.probe;
    a.timeout_ticks = L.timeout_ticks;
    uint64_t *words = reinterpret_cast<uint64_t *>(L.sync);
    uint64_t nwords = uint64_t(L.teams_alloc) * sizeof(PhaseSync) / sizeof(uint64_t);
    uint64_t *slots = L.partials;
    uint64_t nslots = uint64_t(L.grid) * 32u;
    void *ra[] = {&words, &nwords, &slots, &nslots};
    hipError_t e = hipLaunchKernel(reinterpret_cast<const void *>(&phase_reset_kernel), dim3(64), dim3(256), ra, 0,
                                   L.stream);
    if (e != hipSuccess)
        return e;
    void *args[] = {&a};
    return hipLaunchCooperativeKernel(phase_kernel_fn(adjoint, L.held != 0u), dim3(L.grid), dim3(kStreamBlock), args,
                                      0, L.stream);
}

}  // namespace grover
