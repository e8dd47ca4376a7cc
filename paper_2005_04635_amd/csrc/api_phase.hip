// C ABI of the generalized iteration with per-iteration phases and its adjoint (grover_phase_* in
// grover.h): validation, buffers (states, adjoint states, checkpoints), the persistent grid check, and the
// forward / adjoint launches (k_phase.hip).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "phase.h"

using namespace grover;

struct grover_phase {
    int device = 0;
    hipStream_t stream = nullptr;
    int cu_count = 0;
    uint32_t n = 0, B = 0, K = 0, every = 0, nck = 0;
    uint64_t N = 0, nvec = 0;
    float amp = 0.0f;
    std::vector<uint64_t> marks;
    uint64_t *marks_dev = nullptr;
    void *state = nullptr, *lambda = nullptr, *ckpt = nullptr;
    double *params = nullptr;  // [2][B][K]: the phases of the last forward run (phi, then theta)
    double *aux = nullptr;     // [B][2]
    PhaseSync *sync = nullptr;
    uint64_t *partials = nullptr;
    int grid = 0;
    uint32_t team = 1;                           // workgroups per schedule, streamed form
    uint32_t form = GROVER_PHASE_FORM_AUTO;      // as chosen by grover_phase_set_form
    uint32_t held_team_f = 0, held_team_a = 0;   // on-chip form: workgroups per schedule (0: does not fit)
    uint64_t timeout_ticks = 0;
    bool forward_done = false;
    size_t device_bytes = 0;
    std::string last_error;
};

namespace {

constexpr uint32_t kPhaseMaxQubits = 30;

int pfail(grover_phase *p, int status, const std::string &msg)
{
    if (p)
        p->last_error = msg;
    return status;
}

int phip(grover_phase *p, hipError_t e, const char *what)
{
    (void)hipGetLastError();
    int status = GROVER_E_HIP;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        status = GROVER_E_NOMEM;
    else if (e == hipErrorCooperativeLaunchTooLarge)
        status = GROVER_E_COOP;
    return pfail(p, status, std::string(what) + ": " + hipGetErrorString(e));
}

#define PHASE_HIP(p, expr, what)              \
    do {                                      \
        const hipError_t e_ = (expr);         \
        if (e_ != hipSuccess)                 \
            return phip((p), e_, (what));     \
    } while (0)

template <class P>
hipError_t palloc(grover_phase *p, P **ptr, size_t bytes)
{
    void *v = nullptr;
    const hipError_t e = hipMalloc(&v, bytes > 0 ? bytes : 16);
    *ptr = static_cast<P *>(v);
    if (e == hipSuccess)
        p->device_bytes += bytes;
    return e;
}

void release(grover_phase *p)
{
    if (!p)
        return;
    for (void *q : {p->state, p->lambda, p->ckpt, (void *)p->marks_dev, (void *)p->params, (void *)p->aux,
                    (void *)p->sync, (void *)p->partials})
        if (q)
            (void)hipFree(q);
    delete p;
}

PhaseLaunch launch_of(const grover_phase *p)
{
    PhaseLaunch L{};
    L.state = p->state;
    L.lambda = p->lambda;
    L.ckpt = p->ckpt;
    L.marks = p->marks_dev;
    L.m = p->marks.size();
    L.nvec = p->nvec;
    L.N = double(p->N);
    L.amp = p->amp;
    L.B = p->B;
    L.K = p->K;
    L.every = p->every;
    L.nck = p->nck;
    L.phi = p->params;
    L.theta = p->params + uint64_t(p->B) * p->K;
    L.aux = p->aux;
    L.sync = p->sync;
    L.partials = p->partials;
    L.team_size = p->team;
    L.held = 0;
    L.teams_alloc = uint32_t(p->grid);
    L.grid = p->grid;
    L.timeout_ticks = p->timeout_ticks;
    L.stream = p->stream;
    return L;
}

int check_barriers(grover_phase *p)
{
    PHASE_HIP(p, hipStreamSynchronize(p->stream), "stream synchronise");
    std::vector<PhaseSync> s(size_t(p->grid));
    PHASE_HIP(p, hipMemcpy(s.data(), p->sync, s.size() * sizeof(PhaseSync), hipMemcpyDeviceToHost),
              "barrier status download");
    for (const PhaseSync &x : s)
        if (x.error)
            return pfail(p, GROVER_E_TIMEOUT, "a team barrier wait exceeded its limit; results undefined");
    return GROVER_OK;
}

// The teams wait on each other, so the grid must be co-resident: confirmed on the device with one barrier
// of the whole grid under a short wait limit (shrinking on a time-out), as for the other persistent kernels.
int select_grid(grover_phase *p, int clock_khz)
{
    int per_cu = 1 << 30;
    for (bool held : {false, true})
        for (bool adjoint : {false, true}) {
            int pc = 0;
            PHASE_HIP(p, hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, phase_kernel_fn(adjoint, held), 1024, 0),
                      "occupancy");
            per_cu = std::min(per_cu, pc);
        }
    per_cu = std::max(1, per_cu);
    const int max_grid = per_cu * p->cu_count;
    PHASE_HIP(p, palloc(p, &p->sync, size_t(max_grid) * sizeof(PhaseSync)), "phase allocation");
    PHASE_HIP(p, palloc(p, &p->partials, size_t(max_grid) * 32 * sizeof(uint64_t)), "phase allocation");
    // work still running on other (non-blocking) streams could hold CUs and starve the check
    PHASE_HIP(p, hipDeviceSynchronize(), "device synchronise before the grid check");
    const uint64_t probe_ticks = uint64_t(clock_khz > 0 ? clock_khz : 100000) * 250;  // 0.25 s
    for (int pc = per_cu > 1 ? per_cu - 1 : 1; pc >= 1; --pc) {
        p->grid = pc * p->cu_count;
        PhaseLaunch L = launch_of(p);
        L.probe = 1;
        L.team_size = uint32_t(p->grid);
        L.timeout_ticks = probe_ticks;
        bool ok = true;
        for (uint32_t held : {0u, 1u})
            for (bool adjoint : {false, true}) {  // each launch zeroes the barriers first: check after each
                L.held = held;
                PHASE_HIP(p, launch_phase(L, adjoint), "phase grid check");
                ok = ok && check_barriers(p) == GROVER_OK;
            }
        if (ok)
            return GROVER_OK;
    }
    return pfail(p, GROVER_E_COOP, "no co-resident grid of the phase kernels on this device");
}

uint32_t pow2_at_least(uint64_t x)
{
    uint32_t t = 1;
    while (t < x)
        t <<= 1;
    return t;
}

// The on-chip form's team sizes: the power of two of workgroups whose threads can hold a state (forward)
// or a state and its adjoint (adjoint); 0 when that exceeds the largest power of two <= grid.
void held_teams(grover_phase *p)
{
    uint32_t max_team = 1;
    while (uint64_t(max_team) * 2 <= uint64_t(p->grid))
        max_team <<= 1;
    const uint32_t tf = pow2_at_least((p->nvec + kPhaseHeldForwardVecs - 1) / kPhaseHeldForwardVecs);
    const uint32_t ta = pow2_at_least((p->nvec + kPhaseHeldAdjointVecs - 1) / kPhaseHeldAdjointVecs);
    const bool fits = tf <= max_team && ta <= max_team;
    p->held_team_f = fits ? tf : 0;
    p->held_team_a = fits ? ta : 0;
}

bool use_held(const grover_phase *p)
{
    return p->form == GROVER_PHASE_FORM_HELD || (p->form == GROVER_PHASE_FORM_AUTO && p->held_team_f > 0);
}

int run(grover_phase *p, bool adjoint, const double *dloss, double *loss, double *dphi, double *dtheta)
{
    PhaseLaunch L = launch_of(p);
    if (use_held(p)) {
        L.held = 1;
        L.team_size = adjoint ? p->held_team_a : p->held_team_f;
    }
    L.loss = loss;
    L.dloss = dloss;
    L.dphi = dphi;
    L.dtheta = dtheta;
    PHASE_HIP(p, launch_phase(L, adjoint), adjoint ? "adjoint launch" : "forward launch");
    return GROVER_OK;
}

}  // namespace

extern "C" {

int grover_phase_init(grover_phase **out, const grover_phase_config *cfg, void *hip_stream)
{
    if (!out)
        return GROVER_E_INVAL;
    *out = nullptr;
    if (!cfg || cfg->n < 1 || cfg->n > kPhaseMaxQubits || cfg->batch < 1 || cfg->iterations < 1 ||
        cfg->flags != 0 || cfg->m > (uint64_t(1) << cfg->n) || (cfg->m > 0 && !cfg->marked))
        return GROVER_E_INVAL;
    if (cfg->dtype != GROVER_C64)
        return GROVER_E_UNSUPPORTED;
    grover_phase *p = new (std::nothrow) grover_phase;
    if (!p)
        return GROVER_E_NOMEM;
    int status = GROVER_OK;
    try {
        p->n = cfg->n;
        p->B = cfg->batch;
        p->K = cfg->iterations;
        p->every = cfg->checkpoint_every
                       ? cfg->checkpoint_every
                       : std::max<uint32_t>(1u, uint32_t(std::lround(std::sqrt(double(cfg->iterations)))));
        p->nck = (p->K - 1u) / p->every;
        p->N = uint64_t(1) << p->n;
        p->nvec = p->N / 2;
        const int n = int(p->n);
        p->amp = float(n % 2 == 0 ? std::ldexp(1.0, -n / 2) : std::ldexp(std::sqrt(2.0), -(n + 1) / 2));
        p->marks.assign(cfg->marked, cfg->marked + cfg->m);
        std::sort(p->marks.begin(), p->marks.end());
        for (size_t i = 0; i < p->marks.size(); ++i)
            if (p->marks[i] >= p->N || (i > 0 && p->marks[i] == p->marks[i - 1])) {
                release(p);
                return GROVER_E_INVAL;
            }
        p->stream = static_cast<hipStream_t>(hip_stream);
        hipError_t e = hipGetDevice(&p->device);
        int clock_khz = 0, coop = 0;
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&p->cu_count, hipDeviceAttributeMultiprocessorCount, p->device);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, p->device);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, p->device);
        if (e != hipSuccess) {
            status = phip(p, e, "device query");
            throw status;
        }
        if (!coop) {
            status = pfail(p, GROVER_E_COOP, "device without cooperative launch");
            throw status;
        }
        uint64_t timeout_ms = 10000;
        if (const char *env = getenv("GROVER_BARRIER_TIMEOUT_MS"))
            timeout_ms = strtoull(env, nullptr, 10);
        p->timeout_ticks = uint64_t(clock_khz > 0 ? clock_khz : 100000) * timeout_ms;
        const size_t sbytes = size_t(p->B) * p->nvec * 16;
        e = palloc(p, &p->state, sbytes);
        if (e == hipSuccess)
            e = palloc(p, &p->lambda, sbytes);
        if (e == hipSuccess)
            e = palloc(p, &p->ckpt, sbytes * p->nck);
        if (e == hipSuccess)
            e = palloc(p, &p->marks_dev, std::max<size_t>(1, p->marks.size()) * sizeof(uint64_t));
        if (e == hipSuccess)
            e = palloc(p, &p->params, size_t(2) * p->B * p->K * sizeof(double));
        if (e == hipSuccess)
            e = palloc(p, &p->aux, size_t(2) * p->B * sizeof(double));
        if (e == hipSuccess && !p->marks.empty())
            e = hipMemcpy(p->marks_dev, p->marks.data(), p->marks.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            status = phip(p, e, "phase allocation");
            throw status;
        }
        status = select_grid(p, clock_khz);
        if (status != GROVER_OK)
            throw status;
        held_teams(p);
        // default team: the grid split evenly over the schedules, no larger than the tiles of one state
        const uint64_t tiles = (p->nvec + 4095) / 4096;
        p->team = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(uint64_t(p->grid) / p->B, tiles)));
    } catch (int) {
        release(p);
        return status;
    } catch (...) {
        release(p);
        return GROVER_E_NOMEM;
    }
    *out = p;
    return GROVER_OK;
}

int grover_phase_set_team(grover_phase *p, uint32_t team)
{
    if (!p)
        return GROVER_E_INVAL;
    if (team < 1 || team > uint32_t(p->grid))
        return pfail(p, GROVER_E_INVAL, "team size must lie in [1, grid size]");
    p->team = team;
    return GROVER_OK;
}

int grover_phase_set_form(grover_phase *p, uint32_t form)
{
    if (!p)
        return GROVER_E_INVAL;
    if (form > GROVER_PHASE_FORM_HELD)
        return pfail(p, GROVER_E_INVAL, "unknown form");
    if (form == GROVER_PHASE_FORM_HELD && p->held_team_f == 0)
        return pfail(p, GROVER_E_UNSUPPORTED, "the states are too large to hold on chip in this grid");
    p->form = form;
    return GROVER_OK;
}

int grover_phase_forward(grover_phase *p, const double *phi, const double *theta, double *loss)
{
    if (!p)
        return GROVER_E_INVAL;
    if (!phi || !theta || !loss)
        return pfail(p, GROVER_E_INVAL, "null device pointer");
    const size_t bytes = size_t(p->B) * p->K * sizeof(double);
    PHASE_HIP(p, hipMemcpyAsync(p->params, phi, bytes, hipMemcpyDeviceToDevice, p->stream), "phase copy");
    PHASE_HIP(p, hipMemcpyAsync(p->params + size_t(p->B) * p->K, theta, bytes, hipMemcpyDeviceToDevice, p->stream),
              "phase copy");
    const int st = run(p, false, nullptr, loss, nullptr, nullptr);
    p->forward_done = st == GROVER_OK;
    return st;
}

int grover_phase_backward(grover_phase *p, const double *dloss, double *dphi, double *dtheta)
{
    if (!p)
        return GROVER_E_INVAL;
    if (!dloss || !dphi || !dtheta)
        return pfail(p, GROVER_E_INVAL, "null device pointer");
    if (!p->forward_done)
        return pfail(p, GROVER_E_INVAL, "the adjoint needs the states of a forward run (one adjoint per forward)");
    p->forward_done = false;  // the adjoint sweep overwrites the states
    return run(p, true, dloss, nullptr, dphi, dtheta);
}

int grover_phase_sync(grover_phase *p)
{
    if (!p)
        return GROVER_E_INVAL;
    return check_barriers(p);
}

int grover_phase_state(grover_phase *p, uint32_t b, void **dev_ptr, size_t *bytes)
{
    if (!p || !dev_ptr || !bytes || b >= p->B)
        return pfail(p, GROVER_E_INVAL, "bad schedule index or null argument");
    *dev_ptr = static_cast<char *>(p->state) + size_t(b) * p->nvec * 16;
    *bytes = size_t(p->nvec) * 16;
    return GROVER_OK;
}

int grover_phase_read_state(grover_phase *p, uint32_t b, void *host, size_t bytes)
{
    void *src = nullptr;
    size_t want = 0;
    const int st = grover_phase_state(p, b, &src, &want);
    if (st != GROVER_OK)
        return st;
    if (!host || bytes != want)
        return pfail(p, GROVER_E_INVAL, "byte count differs from the state size");
    PHASE_HIP(p, hipMemcpyAsync(host, src, bytes, hipMemcpyDeviceToHost, p->stream), "state download");
    PHASE_HIP(p, hipStreamSynchronize(p->stream), "stream synchronise");
    return GROVER_OK;
}

int grover_phase_query(grover_phase *p, int key, int64_t *value)
{
    if (!p || !value)
        return pfail(p, GROVER_E_INVAL, "null argument");
    switch (key) {
    case 0: *value = p->B; break;
    case 1: *value = p->grid; break;
    case 2: *value = p->team; break;
    case 3: *value = p->every; break;
    case 4: *value = p->nck; break;
    case 5: *value = int64_t(p->device_bytes); break;
    case 6: *value = use_held(p) ? GROVER_PHASE_FORM_HELD : GROVER_PHASE_FORM_STREAMED; break;
    case 7: *value = p->held_team_f; break;
    case 8: *value = p->held_team_a; break;
    default: return pfail(p, GROVER_E_INVAL, "unknown query key");
    }
    return GROVER_OK;
}

void grover_phase_destroy(grover_phase *p)
{
    if (!p)
        return;
    (void)hipStreamSynchronize(p->stream);
    release(p);
}

const char *grover_phase_last_error(const grover_phase *p) { return p ? p->last_error.c_str() : "no phase context"; }

}  // extern "C"
