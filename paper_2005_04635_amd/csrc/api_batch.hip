// C ABI of batched searches (grover_batch_* in grover.h): validation, the batch buffers, the work queues of
// a tiling, the autotuner that picks the tiling by timing the batch itself, and the graph capture of a
// run.  The device work is one persistent launch (k_batch.hip) preceded by a small reset kernel.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>

#include "batch.h"

using namespace grover;

struct grover_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    int cu_count = 0;
    uint64_t count = 0;
    std::vector<uint32_t> n;
    std::vector<uint64_t> m, iters, nvec, state_off, marks_off;
    std::vector<uint64_t> marks;  // concatenated, each instance's list sorted
    uint64_t total_vecs = 0;
    double total_updates = 0.0;
    void *state = nullptr;
    uint64_t *marks_dev = nullptr;
    BatchInstance *inst_dev = nullptr;
    uint32_t *queue = nullptr;
    unsigned long long *heads = nullptr;
    GridSync *team_sync = nullptr;
    uint64_t *team_partials = nullptr;
    int grid = 0;
    uint32_t split_n = 0, team_size = 1, resident = 0;
    uint64_t n_team = 0;  // instances in multi-workgroup phases
    uint32_t nphases = 0;
    uint64_t qoff[kBatchMaxPhases + 1] = {};
    uint32_t phase_team[kBatchMaxPhases] = {}, phase_resident[kBatchMaxPhases] = {};
    uint32_t streams = 1;  // 0 when the tiling holds every state on chip
    uint32_t update = 0;   // grover_update of the element update
    uint64_t timeout_ticks = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string last_error;
};

namespace {

constexpr uint32_t kBatchMaxQubits = 24;  // a batch instance holds at most 2^24 amplitudes (128 MiB)

int bfail(grover_batch *b, int status, const std::string &msg)
{
    if (b)
        b->last_error = msg;
    return status;
}

int bhip(grover_batch *b, hipError_t e, const char *what)
{
    (void)hipGetLastError();
    int status = GROVER_E_HIP;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        status = GROVER_E_NOMEM;
    else if (e == hipErrorCooperativeLaunchTooLarge)
        status = GROVER_E_COOP;
    return bfail(b, status, std::string(what) + ": " + hipGetErrorString(e));
}

#define BATCH_HIP(b, expr, what)              \
    do {                                      \
        const hipError_t e_ = (expr);         \
        if (e_ != hipSuccess)                 \
            return bhip((b), e_, (what));     \
    } while (0)

template <class P>
hipError_t balloc(P **p, size_t bytes)
{
    void *v = nullptr;
    const hipError_t e = hipMalloc(&v, bytes > 0 ? bytes : 16);
    *p = static_cast<P *>(v);
    return e;
}

void release(grover_batch *b)
{
    if (!b)
        return;
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    for (void *p : {b->state, (void *)b->marks_dev, (void *)b->inst_dev, (void *)b->queue, (void *)b->heads,
                    (void *)b->team_sync, (void *)b->team_partials})
        if (p)
            (void)hipFree(p);
    delete b;
}

BatchLaunch launch_of(const grover_batch *b, uint64_t timeout_ticks)
{
    BatchLaunch L{};
    L.state = b->state;
    L.marks = b->marks_dev;
    L.inst = b->inst_dev;
    L.queue = b->queue;
    for (int p = 0; p <= kBatchMaxPhases; ++p)
        L.qoff[p] = b->qoff[p];
    for (int p = 0; p < kBatchMaxPhases; ++p) {
        L.team[p] = b->phase_team[p];
        L.resident[p] = b->phase_resident[p];
    }
    L.nphases = b->nphases;
    L.streams = b->streams;
    L.update = b->update;
    L.heads = b->heads;
    L.sync = b->team_sync;
    L.partials = b->team_partials;
    L.grid = b->grid;
    L.timeout_ticks = timeout_ticks;
    L.stream = b->stream;
    return L;
}

// Any team barrier that gave up during the last run?  (Synchronises.)
int check_barriers(grover_batch *b)
{
    BATCH_HIP(b, hipStreamSynchronize(b->stream), "stream synchronise");
    std::vector<GridSync> gs(size_t(b->grid) * kBatchMaxPhases);
    BATCH_HIP(b, hipMemcpy(gs.data(), b->team_sync, gs.size() * sizeof(GridSync), hipMemcpyDeviceToHost),
              "barrier status download");
    for (const GridSync &g : gs)
        if (g.error)
            return bfail(b, GROVER_E_TIMEOUT, "a team barrier wait exceeded its limit; batch results undefined");
    return GROVER_OK;
}

uint32_t next_pow2(uint64_t x)
{
    uint32_t p = 1;
    while (p < x)
        p <<= 1;
    return p;
}

// Phases of a tiling.  With resident vectors r > 0, an instance whose state fits on chip in a team of
// T = the power of two >= nvec / (r * 1024) workgroups (T no larger than the largest power of two <= grid)
// runs in the resident phase of that T; states of <= 16384 vectors (n <= 15) run alone on chip.
// Every other instance streams: with n >= split_n and team > 1 in a streamed phase of teams of `team`
// workgroups, else alone.  Phases are ordered by decreasing team size (streamed before resident at equal
// size), each queue by decreasing work N * k (ties by index, for a reproducible order).
int apply_tiling(grover_batch *b, uint32_t split_n, uint32_t team_size, uint32_t resident)
{
    if (team_size < 1 || team_size > uint32_t(b->grid))
        return bfail(b, GROVER_E_INVAL, "team size must lie in [1, grid size]");
    if (resident > uint32_t(kBatchHoldE) || (resident & (resident - 1u)) != 0u)
        return bfail(b, GROVER_E_INVAL, "resident vectors per thread must be 0, 1, 2, 4, 8 or 16");
    const uint32_t max_team = next_pow2(uint64_t(b->grid) + 1) / 2;  // largest power of two <= grid
    std::vector<uint32_t> order(b->count);
    std::iota(order.begin(), order.end(), 0u);
    auto work = [&](uint32_t i) { return double(b->nvec[i]) * double(b->iters[i] + 1); };
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return work(x) > work(y); });
    // phase key: team size, and streamed (1) before resident (0) at equal size
    std::vector<std::pair<std::pair<uint32_t, uint32_t>, std::vector<uint32_t>>> phases;
    auto phase_of = [&](uint32_t t, uint32_t streamed) -> std::vector<uint32_t> & {
        for (auto &ph : phases)
            if (ph.first == std::make_pair(t, streamed))
                return ph.second;
        phases.push_back({{t, streamed}, {}});
        return phases.back().second;
    };
    uint64_t n_team = 0;
    for (uint32_t i : order) {
        const uint64_t nvec = b->nvec[i];
        if (nvec <= uint64_t(kBatchHoldE) * 1024u) {
            phase_of(1, 0).push_back(i);
            continue;
        }
        if (resident > 0) {
            const uint32_t t = next_pow2((nvec + uint64_t(resident) * 1024u - 1) / (uint64_t(resident) * 1024u));
            if (t <= max_team) {
                phase_of(t, 0).push_back(i);
                ++n_team;
                continue;
            }
        }
        if (team_size > 1 && b->n[i] >= split_n) {
            phase_of(team_size, 1).push_back(i);
            ++n_team;
        } else {
            phase_of(1, 0).push_back(i);
        }
    }
    std::stable_sort(phases.begin(), phases.end(), [](const auto &x, const auto &y) {
        return x.first.first != y.first.first ? x.first.first > y.first.first : x.first.second > y.first.second;
    });
    // each team size must divide the previous one (all are powers of two except a streamed `team`)
    for (size_t p = 1; p < phases.size(); ++p)
        if (phases[p - 1].first.first % phases[p].first.first != 0u)
            return bfail(b, GROVER_E_UNSUPPORTED,
                         "the streamed team size must be a power of two when resident teams are used");
    if (phases.size() > size_t(kBatchMaxPhases))
        return bfail(b, GROVER_E_UNSUPPORTED, "too many phases");
    std::vector<uint32_t> q;
    q.reserve(b->count);
    b->nphases = uint32_t(phases.size());
    for (int p = 0; p <= kBatchMaxPhases; ++p)
        b->qoff[p] = 0;
    for (size_t p = 0; p < phases.size(); ++p) {
        b->qoff[p] = q.size();
        b->phase_team[p] = phases[p].first.first;
        b->phase_resident[p] = phases[p].first.second ? 0u : (phases[p].first.first > 1 ? resident : 1u);
        q.insert(q.end(), phases[p].second.begin(), phases[p].second.end());
    }
    for (size_t p = phases.size(); p <= size_t(kBatchMaxPhases); ++p)
        b->qoff[p] = q.size();
    BATCH_HIP(b, hipMemcpy(b->queue, q.data(), q.size() * 4, hipMemcpyHostToDevice), "queue upload");
    // the kernel without the streamed paths serves tilings whose phases all hold their states on chip
    uint32_t streams = 0;
    for (size_t p = 0; p < phases.size(); ++p) {
        if (phases[p].first.second)
            streams = 1;
        if (phases[p].first.first == 1)
            for (uint32_t i : phases[p].second)
                if (b->nvec[i] > uint64_t(kBatchHoldE) * 1024u)
                    streams = 1;
    }
    b->streams = streams;
    b->n_team = n_team;
    b->split_n = split_n;
    b->team_size = team_size;
    b->resident = resident;
    if (b->exec) {  // a captured graph holds the old tiling's arguments
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
    }
    return GROVER_OK;
}

// The grid of the batch kernel must be co-resident (teams wait on each other).  As for the fused kernel,
// the runtime's occupancy figure is confirmed on the device: one team spanning the whole grid meets once at
// a barrier under a short wait limit (both queues empty); on a time-out the grid shrinks.
int select_grid(grover_batch *b, int clock_khz)
{
    int per_cu = 0;
    int per_cu_held = 0;
    const bool u32 = b->update == GROVER_UPDATE_F32;
    BATCH_HIP(b, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel_fn(true, u32), 1024, 0),
              "occupancy");
    BATCH_HIP(b, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_held, batch_kernel_fn(false, u32), 1024, 0),
              "occupancy");
    per_cu = std::min(per_cu, per_cu_held);
    const int max_grid = std::max(1, per_cu) * b->cu_count;
    BATCH_HIP(b, balloc(&b->team_sync, size_t(max_grid) * kBatchMaxPhases * sizeof(GridSync)), "batch allocation");
    BATCH_HIP(b, balloc(&b->team_partials, size_t(max_grid) * kBatchMaxPhases * 8 * sizeof(uint64_t)),
              "batch allocation");
    // work still running on other (non-blocking) streams could hold CUs and starve the check
    BATCH_HIP(b, hipDeviceSynchronize(), "device synchronise before the grid check");
    const uint64_t probe_ticks = uint64_t(clock_khz > 0 ? clock_khz : 100000) * 250;  // 0.25 s
    for (int pc = per_cu > 1 ? per_cu - 1 : 1; pc >= 1; --pc) {
        b->grid = pc * b->cu_count;
        // both instantiations of the kernel (with and without the streamed paths) must fit this grid
        bool fits = true;
        for (uint32_t streams : {1u, 0u}) {
            BatchLaunch L = launch_of(b, probe_ticks);
            L.probe = 1;
            L.streams = streams;
            BATCH_HIP(b, launch_batch(L), "batch grid check");
            BATCH_HIP(b, hipStreamSynchronize(b->stream), "batch grid check");
            if (check_barriers(b) != GROVER_OK) {
                fits = false;
                break;
            }
        }
        if (fits)
            return GROVER_OK;
    }
    return bfail(b, GROVER_E_COOP, "no co-resident grid of the batch kernel on this device");
}

// The persistent kernel node of a captured run must keep the cooperative launch's co-residency
// guarantee: find it and make sure its cooperative attribute is set.
hipError_t make_node_cooperative(hipGraph_t g)
{
    size_t count = 0;
    hipError_t e = hipGraphGetNodes(g, nullptr, &count);
    if (e != hipSuccess)
        return e;
    std::vector<hipGraphNode_t> nodes(count);
    e = hipGraphGetNodes(g, nodes.data(), &count);
    if (e != hipSuccess)
        return e;
    int found = 0;
    for (hipGraphNode_t node : nodes) {
        hipGraphNodeType type;
        e = hipGraphNodeGetType(node, &type);
        if (e != hipSuccess)
            return e;
        if (type != hipGraphNodeTypeKernel)
            continue;
        hipKernelNodeParams kp{};
        e = hipGraphKernelNodeGetParams(node, &kp);
        if (e != hipSuccess)
            return e;
        bool batch_node = false;
        for (bool streams : {true, false})
            for (bool u32 : {true, false})
                batch_node = batch_node || kp.func == batch_kernel_fn(streams, u32);
        if (!batch_node)
            continue;
        ++found;
        hipKernelNodeAttrValue v{};
        e = hipGraphKernelNodeGetAttribute(node, hipKernelNodeAttributeCooperative, &v);
        if (e != hipSuccess)
            return e;
        if (!v.cooperative) {
            v.cooperative = 1;
            e = hipGraphKernelNodeSetAttribute(node, hipKernelNodeAttributeCooperative, &v);
            if (e != hipSuccess)
                return e;
        }
    }
    return found == 1 ? hipSuccess : hipErrorInvalidValue;
}

}  // namespace

extern "C" {

int grover_batch_init(grover_batch **out, const grover_batch_config *cfg, void *hip_stream)
{
    if (!out)
        return GROVER_E_INVAL;
    *out = nullptr;
    if (!cfg || cfg->count == 0 || !cfg->n || !cfg->m || cfg->flags != 0 || cfg->reserved != 0 ||
        cfg->update > GROVER_UPDATE_F32)
        return GROVER_E_INVAL;
    if (cfg->dtype != GROVER_C64)
        return GROVER_E_UNSUPPORTED;
    grover_batch *b = new (std::nothrow) grover_batch;
    if (!b)
        return GROVER_E_NOMEM;
    int status = GROVER_OK;
    try {
        b->count = cfg->count;
        b->update = cfg->update;
        b->stream = static_cast<hipStream_t>(hip_stream);
        uint64_t total_m = 0;
        for (uint64_t i = 0; i < cfg->count; ++i) {
            if (cfg->n[i] < 1 || cfg->n[i] > kBatchMaxQubits || cfg->m[i] > (uint64_t(1) << cfg->n[i])) {
                release(b);
                return GROVER_E_INVAL;
            }
            total_m += cfg->m[i];
        }
        if (total_m > 0 && !cfg->marked) {
            release(b);
            return GROVER_E_INVAL;
        }
        b->n.assign(cfg->n, cfg->n + cfg->count);
        b->m.assign(cfg->m, cfg->m + cfg->count);
        b->marks.assign(cfg->marked, cfg->marked + total_m);
        b->iters.resize(b->count);
        b->nvec.resize(b->count);
        b->state_off.resize(b->count);
        b->marks_off.resize(b->count);
        std::vector<BatchInstance> inst(b->count);
        uint64_t moff = 0, soff = 0;
        for (uint64_t i = 0; i < b->count; ++i) {
            const uint64_t N = uint64_t(1) << b->n[i];
            auto first = b->marks.begin() + int64_t(moff), last = first + int64_t(b->m[i]);
            std::sort(first, last);
            for (auto it = first; it != last; ++it)
                if (*it >= N || (it != first && *it == *(it - 1))) {
                    release(b);
                    return GROVER_E_INVAL;
                }
            b->iters[i] = cfg->iterations ? cfg->iterations[i] : grover_optimal_iterations(b->n[i], b->m[i]);
            b->nvec[i] = N / 2;  // n >= 1: two complex64 amplitudes per 16-byte vector
            b->state_off[i] = soff;
            b->marks_off[i] = moff;
            const int n = int(b->n[i]);
            inst[i].state_off = soff;
            inst[i].nvec = b->nvec[i];
            inst[i].marks_off = moff;
            inst[i].m = b->m[i];
            inst[i].iters = b->iters[i];
            inst[i].N = double(N);
            inst[i].amp = (n % 2 == 0) ? std::ldexp(1.0, -n / 2) : std::ldexp(std::sqrt(2.0), -(n + 1) / 2);
            soff += (b->nvec[i] + 15) / 16 * 16;  // 256-byte aligned instances
            moff += b->m[i];
            b->total_updates += double(N) * double(b->iters[i]);
        }
        b->total_vecs = soff;
        hipError_t e = hipGetDevice(&b->device);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&b->cu_count, hipDeviceAttributeMultiprocessorCount, b->device);
        int clock_khz = 0;
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, b->device);
        int coop = 0;
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, b->device);
        if (e != hipSuccess) {
            status = bhip(b, e, "device query");
            throw status;
        }
        if (!coop) {
            status = bfail(b, GROVER_E_COOP, "device without cooperative launch");
            throw status;
        }
        uint64_t timeout_ms = 10000;
        if (const char *env = getenv("GROVER_BARRIER_TIMEOUT_MS"))
            timeout_ms = strtoull(env, nullptr, 10);
        b->timeout_ticks = uint64_t(clock_khz > 0 ? clock_khz : 100000) * timeout_ms;
        e = balloc(&b->state, size_t(b->total_vecs) * 16);
        if (e == hipSuccess)
            e = balloc(&b->marks_dev, std::max<size_t>(1, total_m) * sizeof(uint64_t));
        if (e == hipSuccess)
            e = balloc(&b->inst_dev, b->count * sizeof(BatchInstance));
        if (e == hipSuccess)
            e = balloc(&b->queue, b->count * 4);
        if (e == hipSuccess)
            e = balloc(&b->heads, kBatchMaxPhases * sizeof(unsigned long long));
        if (e == hipSuccess && total_m > 0)
            e = hipMemcpy(b->marks_dev, b->marks.data(), total_m * sizeof(uint64_t), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(b->inst_dev, inst.data(), inst.size() * sizeof(BatchInstance), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            status = bhip(b, e, "batch allocation");
            throw status;
        }
        status = select_grid(b, clock_khz);
        if (status != GROVER_OK)
            throw status;
        // default tiling until tuned: states held on chip by teams sized for 16 vectors per thread (8 in
        // registers, 8 in LDS); states too large for that stream with teams of 2
        status = apply_tiling(b, 19, b->grid >= 2 ? 2u : 1u, uint32_t(kBatchHoldE));
        if (status != GROVER_OK)
            throw status;
    } catch (int) {
        release(b);
        return status;
    } catch (...) {
        release(b);
        return GROVER_E_NOMEM;
    }
    *out = b;
    return GROVER_OK;
}

int grover_batch_set_tiling(grover_batch *b, uint32_t split_n, uint32_t team_size, uint32_t resident)
{
    if (!b)
        return GROVER_E_INVAL;
    return apply_tiling(b, split_n, team_size, resident);
}

int grover_batch_run(grover_batch *b)
{
    if (!b)
        return GROVER_E_INVAL;
    if (b->exec) {
        BATCH_HIP(b, hipGraphLaunch(b->exec, b->stream), "graph launch");
        return GROVER_OK;
    }
    BATCH_HIP(b, launch_batch(launch_of(b, b->timeout_ticks)), "batch launch");
    return GROVER_OK;
}

int grover_batch_sync(grover_batch *b)
{
    if (!b)
        return GROVER_E_INVAL;
    return check_barriers(b);
}

int grover_batch_tune(grover_batch *b, uint32_t *split_n, uint32_t *team_size, uint32_t *resident, float *best_ms)
{
    if (!b)
        return GROVER_E_INVAL;
    struct Cand {
        uint32_t split, team, resident;
    };
    std::vector<Cand> cands = {{0, 1, 0}};
    for (uint32_t split : {18u, 19u, 20u})
        for (uint32_t t : {2u, 4u, 8u})
            if (t <= uint32_t(b->grid))
                cands.push_back({split, t, 0});
    for (uint32_t r : {16u, 8u, 4u})
        cands.push_back({19, 2, r});
    hipEvent_t e0, e1;
    BATCH_HIP(b, hipEventCreate(&e0), "event");
    BATCH_HIP(b, hipEventCreate(&e1), "event");
    float best = -1.0f;
    Cand pick = cands[0];
    int status = GROVER_OK;
    for (const Cand &c : cands) {
        status = apply_tiling(b, c.split, c.team, c.resident);
        if (status != GROVER_OK)
            break;
        hipError_t e = hipEventRecord(e0, b->stream);
        if (e == hipSuccess)
            e = launch_batch(launch_of(b, b->timeout_ticks));
        if (e == hipSuccess)
            e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess)
            e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            status = bhip(b, e, "autotuner run");
            break;
        }
        status = check_barriers(b);
        if (status != GROVER_OK)
            break;
        if (best < 0.0f || ms < best) {
            best = ms;
            pick = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != GROVER_OK)
        return status;
    status = apply_tiling(b, pick.split, pick.team, pick.resident);
    if (status != GROVER_OK)
        return status;
    if (split_n)
        *split_n = pick.split;
    if (team_size)
        *team_size = pick.team;
    if (resident)
        *resident = pick.resident;
    if (best_ms)
        *best_ms = best;
    return GROVER_OK;
}

int grover_batch_capture(grover_batch *b)
{
    if (!b)
        return GROVER_E_INVAL;
    if (!b->stream)
        return bfail(b, GROVER_E_UNSUPPORTED, "graph capture needs a non-default stream");
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
    }
    BATCH_HIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    const hipError_t le = launch_batch(launch_of(b, b->timeout_ticks));
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(b->stream, &g);
    if (le != hipSuccess || ce != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return bfail(b, GROVER_E_UNSUPPORTED,
                     std::string("the batch launch could not be captured: ") +
                         hipGetErrorString(le != hipSuccess ? le : ce));
    }
    const hipError_t ne = make_node_cooperative(g);
    if (ne != hipSuccess) {
        (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return bfail(b, GROVER_E_UNSUPPORTED,
                     std::string("captured batch launch is not a cooperative kernel node: ") + hipGetErrorString(ne));
    }
    hipGraphExec_t x = nullptr;
    const hipError_t ie = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(g);
        return bhip(b, ie, "graph instantiate");
    }
    b->graph = g;
    b->exec = x;
    return GROVER_OK;
}

int grover_batch_state(grover_batch *b, uint64_t i, void **dev_ptr, size_t *bytes)
{
    if (!b || !dev_ptr || !bytes || i >= b->count)
        return bfail(b, GROVER_E_INVAL, "bad instance or null argument");
    *dev_ptr = static_cast<char *>(b->state) + b->state_off[i] * 16;
    *bytes = size_t(b->nvec[i]) * 16;
    return GROVER_OK;
}

int grover_batch_read_state(grover_batch *b, uint64_t i, void *host, size_t bytes)
{
    void *p = nullptr;
    size_t want = 0;
    const int st = grover_batch_state(b, i, &p, &want);
    if (st != GROVER_OK)
        return st;
    if (!host || bytes != want)
        return bfail(b, GROVER_E_INVAL, "byte count differs from the instance's state size");
    BATCH_HIP(b, hipMemcpyAsync(host, p, bytes, hipMemcpyDeviceToHost, b->stream), "state download");
    BATCH_HIP(b, hipStreamSynchronize(b->stream), "stream synchronise");
    return GROVER_OK;
}

int grover_batch_query(grover_batch *b, int key, int64_t *value)
{
    if (!b || !value)
        return bfail(b, GROVER_E_INVAL, "null argument");
    switch (key) {
    case 0: *value = int64_t(b->count); break;
    case 1: *value = b->grid; break;
    case 2: *value = b->split_n; break;
    case 3: *value = b->team_size; break;
    case 4: *value = int64_t(b->total_updates); break;
    case 5: *value = b->exec ? 1 : 0; break;
    case 6: *value = int64_t(b->total_vecs * 16); break;
    case 7: *value = int64_t(b->n_team); break;
    case 8: *value = b->resident; break;
    case 9: *value = b->nphases; break;
    case 10: *value = b->streams; break;
    default: return bfail(b, GROVER_E_INVAL, "unknown query key");
    }
    return GROVER_OK;
}

void grover_batch_destroy(grover_batch *b)
{
    if (!b)
        return;
    (void)hipStreamSynchronize(b->stream);
    release(b);
}

const char *grover_batch_last_error(const grover_batch *b) { return b ? b->last_error.c_str() : "no batch"; }

}  // extern "C"
