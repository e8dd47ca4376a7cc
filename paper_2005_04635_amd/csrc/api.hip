// C ABI of libgrover (declared and documented in grover.h): validation, context and buffer management,
// error reporting, and the dispatch of each call to the kernel launchers of the other translation units.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "internal.h"
#include "wht.h"

using namespace grover;

namespace {

constexpr uint64_t kDefaultTimeoutMs = 10000;  // grid-barrier wait limit before a kernel gives up

int fail(grover_ctx *c, int status, const std::string &msg)
{
    if (c)
        c->last_error = msg;
    return status;
}

int hip_fail(grover_ctx *c, hipError_t e, const char *what)
{
    (void)hipGetLastError();  // clear the runtime's sticky copy
    int status = GROVER_E_HIP;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        status = GROVER_E_NOMEM;
    else if (e == hipErrorCooperativeLaunchTooLarge)
        status = GROVER_E_COOP;
    return fail(c, status, std::string(what) + ": " + hipGetErrorString(e));
}

#define GROVER_HIP(ctx, expr, what)                 \
    do {                                            \
        const hipError_t e_ = (expr);               \
        if (e_ != hipSuccess)                       \
            return hip_fail((ctx), e_, (what));     \
    } while (0)

template <class P>
hipError_t dev_alloc(P **p, size_t bytes)
{
    void *v = nullptr;
    const hipError_t e = hipMalloc(&v, bytes > 0 ? bytes : 16);
    *p = static_cast<P *>(v);
    return e;
}

void release(grover_ctx *c)
{
    if (!c)
        return;
    if (c->owns_state && c->state)
        (void)hipFree(c->state);
    for (void *p : {(void *)c->marks_dev, (void *)c->partials, (void *)c->sync, (void *)c->red_partials,
                    (void *)c->red_out, (void *)c->cdf, (void *)c->block_sums, (void *)c->shots_buf,
                    (void *)c->u53_buf, (void *)c->flag_dev})
        if (p)
            (void)hipFree(p);
    if (c->host_pinned)
        (void)hipHostFree(c->host_pinned);
    delete c;
}

int check_ctx(const grover_ctx *c) { return c ? GROVER_OK : GROVER_E_INVAL; }

// Bytes of the fused kernel's barrier slots: [2][grid][4] member slots and the [2][4] published sum.
size_t barrier_slot_bytes(int64_t grid) { return size_t(8 * grid + 8) * sizeof(uint64_t); }

// Clear the grid-barrier state (after a wait gave up, the device grid has exited by then; or before the
// generation tags would wrap).  A failure is reported with the name of the call that failed.
int reset_barrier(grover_ctx *c, const char *why)
{
    c->generation = 0;
    const std::string w(why);
    GROVER_HIP(c, hipMemsetAsync(c->sync, 0, sizeof(GridSync), c->stream), (w + ": clearing the barrier words").c_str());
    if (c->partials && c->partials_grid > 0)
        GROVER_HIP(c, hipMemsetAsync(c->partials, 0, barrier_slot_bytes(c->partials_grid), c->stream),
                   (w + ": clearing the barrier slots").c_str());
    GROVER_HIP(c, hipStreamSynchronize(c->stream), (w + ": synchronising the stream").c_str());
    return GROVER_OK;
}

// A residency check must not share the device with work still running on other streams: torch's streams
// are non-blocking, so a persistent kernel launched on one of them (another context's, or a batch's) is not
// ordered before this context's stream and may still hold CUs, and a check grid that cannot become
// resident times out and shrinks.  Waiting for the whole device first makes the check see only itself.
int quiesce_device(grover_ctx *c, const char *what)
{
    GROVER_HIP(c, hipDeviceSynchronize(), what);
    return GROVER_OK;
}

// Persistent grid of the fused form.  Every workgroup of a launch must be resident at once, or the first
// grid barrier can never complete.  The runtime's occupancy figure has proved optimistic (MI355X admits
// fewer workgroups per CU of this kernel than it reports), so the grid is confirmed on the device: the
// fused kernel runs with zero iterations (a read-only sum pass and one barrier) under a short wait limit,
// and on a time-out the grid shrinks by one workgroup per CU.  GROVER_FUSED_GRID forces a grid, which must
// pass the same check.  Allocates the barrier state and the per-workgroup partials.
int select_persistent_grid(grover_ctx *c, int clock_khz)
{
    int per_cu = 0, block = 0;
    int64_t forced = 0;
    GROVER_HIP(c, fused_configure(c, &per_cu, &block, &forced), "persistent grid configuration");
    c->per_cu_reported = per_cu;
    if (per_cu < 1)
        per_cu = 1;  // the runtime may report 0 workgroups per CU; the device check below decides
    const int64_t max_grid = forced > 0 ? forced : int64_t(per_cu) * c->cu_count;
    GROVER_HIP(c, dev_alloc(&c->partials, barrier_slot_bytes(max_grid)), "barrier allocation");
    GROVER_HIP(c, hipMemset(c->partials, 0, barrier_slot_bytes(max_grid)), "barrier allocation");
    c->partials_grid = max_grid;
    GROVER_HIP(c, dev_alloc(&c->sync, sizeof(GridSync)), "barrier allocation");
    if (int st = reset_barrier(c, "barrier reset before the grid check"))
        return st;
    if (int st = quiesce_device(c, "device synchronise before the grid check"))
        return st;
    const uint64_t probe_ticks = uint64_t(clock_khz > 0 ? clock_khz : 100000) * 250;  // 0.25 s
    const uint64_t tiles = fused_tiles(c);
    c->block = block;
    for (int pc = per_cu > 1 ? per_cu - 1 : 1; pc >= 1; --pc) {
        int64_t g = forced > 0 ? forced : int64_t(pc) * c->cu_count;
        if (forced == 0 && uint64_t(g) > tiles)
            g = int64_t(tiles > 0 ? tiles : 1);
        if (g > max_grid)
            return fail(c, GROVER_E_COOP, "persistent grid larger than its barrier allocation");
        c->grid = int(g);
        GROVER_HIP(c, launch_fused_iterate(c, 0, probe_ticks, true), "persistent grid check");
        GROVER_HIP(c, hipStreamSynchronize(c->stream), "persistent grid check");
        GridSync gs;
        GROVER_HIP(c, hipMemcpy(&gs, c->sync, sizeof(gs), hipMemcpyDeviceToHost), "persistent grid check");
        if (!gs.error)
            return GROVER_OK;
        if (int st = reset_barrier(c, "barrier reset after a failed grid check"))
            return st;
        if (forced > 0)
            break;
    }
    return fail(c, GROVER_E_COOP, "no persistent grid of the fused kernel is co-resident on this device");
}

// The held form's team must be co-resident (its members wait on each other): its barrier slots are
// allocated and one team barrier is run under a short wait limit, as the fused form's grid is checked.
int check_held_team(grover_ctx *c, int clock_khz)
{
    const int64_t team = int64_t(c->held_team);
    GROVER_HIP(c, dev_alloc(&c->partials, barrier_slot_bytes(team)), "barrier allocation");
    GROVER_HIP(c, hipMemset(c->partials, 0, barrier_slot_bytes(team)), "barrier allocation");
    c->partials_grid = team;
    GROVER_HIP(c, dev_alloc(&c->sync, sizeof(GridSync)), "barrier allocation");
    if (int st = reset_barrier(c, "barrier reset before the team check"))
        return st;
    if (int st = quiesce_device(c, "device synchronise before the team check"))
        return st;
    const uint64_t probe_ticks = uint64_t(clock_khz > 0 ? clock_khz : 100000) * 250;  // 0.25 s
    GROVER_HIP(c, launch_held_iterate(c, 0, probe_ticks, true), "held team check");
    GROVER_HIP(c, hipStreamSynchronize(c->stream), "held team check");
    GridSync gs;
    GROVER_HIP(c, hipMemcpy(&gs, c->sync, sizeof(gs), hipMemcpyDeviceToHost), "held team check");
    if (gs.error)
        return fail(c, GROVER_E_COOP, "the held form's team is not co-resident on this device");
    return GROVER_OK;
}

int run_iterations(grover_ctx *c, uint64_t k)
{
    if (k == 0)
        return GROVER_OK;
    switch (c->form) {
    case GROVER_FORM_FUSED:
        // barrier generations are tagged modulo 2^32: start again from clear slots before they would wrap
        if (c->generation + k + 2u >= (uint64_t(1) << 32))
            if (int st = reset_barrier(c, "barrier reset before the generation tags wrap"))
                return st;
        GROVER_HIP(c, launch_fused_iterate(c, k, c->timeout_ticks), "fused iterate launch");
        break;
    case GROVER_FORM_RESIDENT: GROVER_HIP(c, launch_resident_iterate(c, k), "resident iterate launch"); break;
    case GROVER_FORM_HELD:
        if (c->generation + k + 2u >= (uint64_t(1) << 32))
            if (int st = reset_barrier(c, "barrier reset before the generation tags wrap"))
                return st;
        GROVER_HIP(c, launch_held_iterate(c, k, c->timeout_ticks), "held iterate launch");
        break;
    case GROVER_FORM_TWO_PASS: GROVER_HIP(c, launch_twopass_iterate(c, k), "two-pass iterate launch"); break;
    default: return fail(c, GROVER_E_INVAL, "context has no iteration form");
    }
    return GROVER_OK;
}

}  // namespace

// The message of the last grover_init (or grover_iterate_static) failure on this thread.
thread_local std::string init_error;

namespace grover {
void set_thread_error(const std::string &msg) { init_error = msg; }
}  // namespace grover

extern "C" {

uint64_t grover_optimal_iterations(uint32_t n, uint64_t m)
{
    if (m == 0 || n > 63 || m > (uint64_t(1) << n))
        return 0;
    const double pi_over_4 = 0.78539816339744830961566084581987572104929234984378;
    return uint64_t(std::floor(pi_over_4 * std::sqrt(std::ldexp(1.0, int(n)) / double(m))));
}

const char *grover_status_str(int status)
{
    switch (status) {
    case GROVER_OK: return "ok";
    case GROVER_E_INVAL: return "invalid argument";
    case GROVER_E_NOMEM: return "out of memory";
    case GROVER_E_HIP: return "HIP runtime error";
    case GROVER_E_COOP: return "persistent grid cannot be co-resident";
    case GROVER_E_UNSUPPORTED: return "unsupported request";
    case GROVER_E_PREDICATE: return "hash predicate hit count differs from m";
    case GROVER_E_TIMEOUT: return "device grid barrier timed out";
    default: return "unknown status";
    }
}


const char *grover_last_error(const grover_ctx *ctx)
{
    if (ctx)
        return ctx->last_error.c_str();
    return init_error.empty() ? "no context" : init_error.c_str();
}

int grover_init(grover_ctx **out, const grover_config *cfg, void *hip_stream, void *state_dev, size_t state_bytes)
{
    if (!out)
        return GROVER_E_INVAL;
    *out = nullptr;
    if (!cfg)
        return GROVER_E_INVAL;
    if (cfg->n < 1 || cfg->n > kMaxQubits || cfg->dtype > GROVER_CBF16 || cfg->oracle_kind > GROVER_ORACLE_HASH ||
        cfg->form > GROVER_FORM_HELD || cfg->flags != 0 || cfg->hash_bits > 64 ||
        cfg->accum > GROVER_ACC_F32_KAHAN || cfg->update > GROVER_UPDATE_F32)
        return GROVER_E_INVAL;
    const uint64_t N = uint64_t(1) << cfg->n;
    if (cfg->m > N)
        return GROVER_E_INVAL;
    // every kernel moves the state in whole 16-byte vectors: a state smaller than one (complex bfloat16 at
    // n = 1, two amplitudes in 8 bytes) would never be written or read
    if (N < elems_per_vec(cfg->dtype))
        return GROVER_E_UNSUPPORTED;
    // bfloat16 storage and binary32 sums exist in the fused form only
    const bool fused_only = cfg->dtype == GROVER_CBF16 || cfg->accum != GROVER_ACC_F64;
    uint32_t form = cfg->form;
    const bool auto_form = form == GROVER_FORM_AUTO;
    // the held form exists for complex64 storage with binary64 sums; AUTO picks it (after the device
    // query, which says whether the state fits on chip) for the sizes above the one-workgroup form, which
    // is faster up to n = 13 and as fast at n = 14 (one optimal search on MI355X, n = 13: 0.145 vs 0.204 ms)
    const bool held_ok = cfg->dtype == GROVER_C64 && cfg->accum == GROVER_ACC_F64;
    if (auto_form)
        form = cfg->n <= kResidentMaxQubits && !fused_only ? GROVER_FORM_RESIDENT : GROVER_FORM_FUSED;
    if (form == GROVER_FORM_RESIDENT && cfg->n > kResidentMaxQubits)
        return GROVER_E_UNSUPPORTED;
    if (form == GROVER_FORM_HELD && !held_ok)
        return GROVER_E_UNSUPPORTED;
    if (fused_only && form != GROVER_FORM_FUSED)
        return GROVER_E_UNSUPPORTED;
    if (cfg->oracle_kind == GROVER_ORACLE_HASH && cfg->m > kHashMarkCap)
        return GROVER_E_UNSUPPORTED;
    // the binary32 update exists for complex64 storage with binary64 sums, in the fused, one-workgroup and
    // held forms (the plain two-pass comparator stays binary64)
    if (cfg->update == GROVER_UPDATE_F32 &&
        (cfg->dtype != GROVER_C64 || cfg->accum != GROVER_ACC_F64 || form == GROVER_FORM_TWO_PASS))
        return GROVER_E_UNSUPPORTED;

    grover_ctx *c = new (std::nothrow) grover_ctx;
    if (!c)
        return GROVER_E_NOMEM;
    int status = GROVER_OK;
    try {
        c->n = cfg->n;
        c->N = N;
        c->dtype = cfg->dtype;
        c->accum = cfg->accum;
        c->update = cfg->update;
        c->form = form;
        c->kind = cfg->oracle_kind;
        c->stream = static_cast<hipStream_t>(hip_stream);
        const size_t eb = elem_bytes(cfg->dtype);
        const size_t need = size_t(N) * eb;

        if (cfg->oracle_kind == GROVER_ORACLE_LIST) {
            if (cfg->m > 0 && !cfg->marked) {
                release(c);
                return GROVER_E_INVAL;
            }
            c->marks.assign(cfg->marked, cfg->marked + cfg->m);
            std::sort(c->marks.begin(), c->marks.end());
            for (size_t i = 0; i < c->marks.size(); ++i) {
                if (c->marks[i] >= N || (i > 0 && c->marks[i] == c->marks[i - 1])) {
                    release(c);
                    return GROVER_E_INVAL;
                }
            }
        }
        if (state_dev) {
            if (state_bytes < need || (reinterpret_cast<uintptr_t>(state_dev) & 15u) != 0) {
                release(c);
                return GROVER_E_INVAL;
            }
            c->state = state_dev;
            c->owns_state = false;
        }

        hipError_t e = hipGetDevice(&c->device);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount, c->device);
        int clock_khz = 0;
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, c->device);
        if (e != hipSuccess) {
            status = hip_fail(c, e, "device query");
            throw status;
        }
        {
            uint32_t max_team = 1;
            while (int64_t(max_team) * 2 <= int64_t(c->cu_count))
                max_team <<= 1;
            const uint32_t team = held_team_size(N / 2, max_team);
            if (auto_form && form == GROVER_FORM_FUSED && held_ok && team > 0)
                form = GROVER_FORM_HELD;
            if (form == GROVER_FORM_HELD) {
                if (team == 0) {
                    status = fail(c, GROVER_E_UNSUPPORTED, "the state is too large for the held form on this device");
                    throw status;
                }
                c->held_team = team;
            }
            c->form = form;
        }
        uint64_t timeout_ms = kDefaultTimeoutMs;
        if (const char *env = getenv("GROVER_BARRIER_TIMEOUT_MS"))
            timeout_ms = strtoull(env, nullptr, 10);
        c->timeout_ticks = uint64_t(clock_khz > 0 ? clock_khz : 100000) * timeout_ms;

        if (!c->state) {
            e = dev_alloc(&c->state, need);
            if (e != hipSuccess) {
                status = hip_fail(c, e, "state allocation");
                throw status;
            }
            c->owns_state = true;
        }
        c->state_bytes = c->owns_state ? need : state_bytes;

        // reduction scratch shared by the two-pass form and the norm
        e = dev_alloc(&c->red_partials, 2 * 2048 * sizeof(double));
        if (e == hipSuccess)
            e = dev_alloc(&c->red_out, 2 * sizeof(double));
        if (e == hipSuccess)
            e = dev_alloc(&c->flag_dev, sizeof(uint32_t));
        if (e == hipSuccess)
            e = hipMemsetAsync(c->flag_dev, 0, sizeof(uint32_t), c->stream);
        if (e == hipSuccess) {
            void *hp = nullptr;
            e = hipHostMalloc(&hp, 4 * sizeof(double), hipHostMallocDefault);
            c->host_pinned = static_cast<double *>(hp);
        }
        if (e != hipSuccess) {
            status = hip_fail(c, e, "scratch allocation");
            throw status;
        }

        if (form == GROVER_FORM_RESIDENT) {
            c->grid = 1;
            c->block = kResidentBlock;
        } else if (form == GROVER_FORM_HELD) {
            c->grid = int(c->held_team);
            c->block = 1024;
        } else {
            c->grid = twopass_blocks(c);
            c->block = 256;
        }

        if (cfg->oracle_kind == GROVER_ORACLE_HASH) {
            // Evaluate the predicate over all N indices, compact the hits, check their number.
            const uint64_t cap = cfg->m + 1;
            uint64_t *list = nullptr;
            unsigned long long *count = nullptr;
            e = dev_alloc(&list, cap * sizeof(uint64_t));
            if (e == hipSuccess)
                e = dev_alloc(&count, sizeof(unsigned long long));
            if (e == hipSuccess)
                e = hipMemsetAsync(count, 0, sizeof(unsigned long long), c->stream);
            if (e == hipSuccess)
                e = launch_hash_marks(c, cfg->hash_seed, cfg->hash_bits, list, cap, count);
            unsigned long long hits = 0;
            if (e == hipSuccess)
                e = hipMemcpyAsync(&hits, count, sizeof(hits), hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess)
                e = hipStreamSynchronize(c->stream);
            if (e == hipSuccess && hits == cfg->m) {
                c->marks.resize(hits);
                if (hits > 0)
                    e = hipMemcpy(c->marks.data(), list, hits * sizeof(uint64_t), hipMemcpyDeviceToHost);
            }
            if (count)
                (void)hipFree(count);
            if (e != hipSuccess) {
                if (list)
                    (void)hipFree(list);
                status = hip_fail(c, e, "hash predicate");
                throw status;
            }
            if (hits != cfg->m) {
                (void)hipFree(list);
                status = fail(c, GROVER_E_PREDICATE, "hash predicate hit count differs from m");
                throw status;
            }
            std::sort(c->marks.begin(), c->marks.end());
            c->marks_dev = list;
        } else if (!c->marks.empty()) {
            e = dev_alloc(&c->marks_dev, c->marks.size() * sizeof(uint64_t));
            if (e != hipSuccess) {
                status = hip_fail(c, e, "marked list allocation");
                throw status;
            }
        }
        if (!c->marks.empty()) {
            e = hipMemcpyAsync(c->marks_dev, c->marks.data(), c->marks.size() * sizeof(uint64_t),
                               hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess)
                e = hipStreamSynchronize(c->stream);  // the host vector must outlive the copy
            if (e != hipSuccess) {
                status = hip_fail(c, e, "marked list upload");
                throw status;
            }
        }
        e = launch_fill_uniform(c);
        if (e != hipSuccess) {
            status = hip_fail(c, e, "initial state");
            throw status;
        }
        if (form == GROVER_FORM_FUSED) {
            // needs the marked list on the device and a written state: it runs the fused kernel
            status = select_persistent_grid(c, clock_khz);
            if (status != GROVER_OK)
                throw status;
        } else if (form == GROVER_FORM_HELD) {
            status = check_held_team(c, clock_khz);
            if (status != GROVER_OK)
                throw status;
        }
    } catch (int) {
        init_error = c->last_error;
        release(c);
        return status;
    } catch (...) {
        init_error = "host allocation failed";
        release(c);
        return GROVER_E_NOMEM;
    }
    *out = c;
    return GROVER_OK;
}

int grover_reset(grover_ctx *ctx)
{
    if (check_ctx(ctx))
        return GROVER_E_INVAL;
    GROVER_HIP(ctx, launch_fill_uniform(ctx), "initial state");
    return GROVER_OK;
}

int grover_iterate(grover_ctx *ctx, uint64_t k)
{
    if (check_ctx(ctx))
        return GROVER_E_INVAL;
    return run_iterations(ctx, k);
}

int grover_gate_iterate(grover_ctx *ctx, uint64_t k)
{
    if (check_ctx(ctx))
        return GROVER_E_INVAL;
    if (ctx->dtype == GROVER_CBF16)
        return fail(ctx, GROVER_E_UNSUPPORTED, "the gate-level path has no bfloat16 form");
    for (uint64_t it = 0; it < k; ++it) {
        GROVER_HIP(ctx, launch_oracle_flip(ctx), "oracle flip");
        GROVER_HIP(ctx, launch_hadamard_all(ctx), "hadamard passes");
        GROVER_HIP(ctx, launch_conditional_phase_shift(ctx), "conditional phase shift");
        GROVER_HIP(ctx, launch_hadamard_all(ctx), "hadamard passes");
    }
    return GROVER_OK;
}

int grover_gate_iterate_blocked(grover_ctx *ctx, uint64_t k)
{
    if (check_ctx(ctx))
        return GROVER_E_INVAL;
    if (ctx->dtype == GROVER_CBF16)
        return fail(ctx, GROVER_E_UNSUPPORTED, "the gate-level path has no bfloat16 form");
    for (uint64_t it = 0; it < k; ++it) {
        GROVER_HIP(ctx, launch_oracle_flip(ctx), "oracle flip");
        GROVER_HIP(ctx, launch_gate_diffusion_blocked(ctx), "blocked Walsh-Hadamard passes");
    }
    return GROVER_OK;
}

int grover_apply_hadamard_all_blocked(grover_ctx *ctx)
{
    if (check_ctx(ctx))
        return GROVER_E_INVAL;
    if (ctx->dtype == GROVER_CBF16)
        return fail(ctx, GROVER_E_UNSUPPORTED, "the gate-level path has no bfloat16 form");
    GROVER_HIP(ctx, launch_hadamard_all_blocked(ctx), "blocked Walsh-Hadamard passes");
    return GROVER_OK;
}

int grover_apply_hadamard_all(grover_ctx *ctx)
{
    if (check_ctx(ctx))
        return GROVER_E_INVAL;
    if (ctx->dtype == GROVER_CBF16)
        return fail(ctx, GROVER_E_UNSUPPORTED, "the gate-level path has no bfloat16 form");
    GROVER_HIP(ctx, launch_hadamard_all(ctx), "hadamard passes");
    return GROVER_OK;
}

static int sample_impl(grover_ctx *c, const uint64_t *u53, int u53_is_device, bool device_uniforms, uint64_t seed,
                       uint64_t shots, uint64_t *out, int out_is_device)
{
    if (shots > 0 && !out)
        return fail(c, GROVER_E_INVAL, "null output");
    if (!device_uniforms && shots > 0 && !u53)
        return fail(c, GROVER_E_INVAL, "null uniforms");
    if (!c->cdf) {
        GROVER_HIP(c, dev_alloc(&c->cdf, size_t(c->N) * sizeof(uint64_t)), "CDF allocation");
        GROVER_HIP(c, dev_alloc(&c->block_sums, sample_block_count(c->N) * sizeof(uint64_t)), "CDF allocation");
    }
    const uint64_t *u_dev = nullptr;
    if (!device_uniforms && shots > 0) {
        if (u53_is_device) {
            u_dev = u53;
        } else {
            if (c->u53_cap < shots) {
                if (c->u53_buf)
                    (void)hipFree(c->u53_buf);
                c->u53_buf = nullptr;
                c->u53_cap = 0;
                GROVER_HIP(c, dev_alloc(&c->u53_buf, shots * sizeof(uint64_t)), "uniform buffer");
                c->u53_cap = shots;
            }
            GROVER_HIP(c, hipMemcpyAsync(c->u53_buf, u53, shots * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream),
                       "uniform upload");
            u_dev = c->u53_buf;
        }
    }
    uint64_t *o_dev = out;
    if (!out_is_device && shots > 0) {
        if (c->shots_cap < shots) {
            if (c->shots_buf)
                (void)hipFree(c->shots_buf);
            c->shots_buf = nullptr;
            c->shots_cap = 0;
            GROVER_HIP(c, dev_alloc(&c->shots_buf, shots * sizeof(uint64_t)), "shot buffer");
            c->shots_cap = shots;
        }
        o_dev = c->shots_buf;
    }
    GROVER_HIP(c, launch_sample(c, u_dev, seed, device_uniforms, shots, o_dev), "sampler launch");
    if (!out_is_device && shots > 0) {
        GROVER_HIP(c, hipMemcpyAsync(out, o_dev, shots * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream),
                   "shot download");
        return grover_sync(c);
    }
    return GROVER_OK;
}

int grover_sample(grover_ctx *ctx, uint64_t shots, uint64_t seed, uint64_t *out, int out_is_device)
{
    if (check_ctx(ctx))
        return GROVER_E_INVAL;
    return sample_impl(ctx, nullptr, 0, true, seed, shots, out, out_is_device);
}

int grover_sample_u53(grover_ctx *ctx, const uint64_t *u53, int u53_is_device, uint64_t shots, uint64_t *out,
                      int out_is_device)
{
    if (check_ctx(ctx))
        return GROVER_E_INVAL;
    return sample_impl(ctx, u53, u53_is_device, false, 0, shots, out, out_is_device);
}

int grover_norm(grover_ctx *ctx, double *out)
{
    if (check_ctx(ctx) || !out)
        return fail(ctx, GROVER_E_INVAL, "null argument");
    GROVER_HIP(ctx, launch_norm(ctx, ctx->red_out), "norm launch");
    GROVER_HIP(ctx, hipMemcpyAsync(ctx->host_pinned, ctx->red_out, sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
               "norm download");
    GROVER_HIP(ctx, hipStreamSynchronize(ctx->stream), "stream synchronise");
    *out = ctx->host_pinned[0];
    return GROVER_OK;
}

int grover_read_state(grover_ctx *ctx, void *host, size_t bytes)
{
    if (check_ctx(ctx) || !host)
        return fail(ctx, GROVER_E_INVAL, "null argument");
    if (bytes != size_t(ctx->N) * elem_bytes(ctx->dtype))
        return fail(ctx, GROVER_E_INVAL, "byte count differs from the state size");
    GROVER_HIP(ctx, hipMemcpyAsync(host, ctx->state, bytes, hipMemcpyDeviceToHost, ctx->stream), "state download");
    GROVER_HIP(ctx, hipStreamSynchronize(ctx->stream), "stream synchronise");
    return GROVER_OK;
}

int grover_write_state(grover_ctx *ctx, const void *host, size_t bytes)
{
    if (check_ctx(ctx) || !host)
        return fail(ctx, GROVER_E_INVAL, "null argument");
    if (bytes != size_t(ctx->N) * elem_bytes(ctx->dtype))
        return fail(ctx, GROVER_E_INVAL, "byte count differs from the state size");
    GROVER_HIP(ctx, hipMemcpyAsync(ctx->state, host, bytes, hipMemcpyHostToDevice, ctx->stream), "state upload");
    GROVER_HIP(ctx, hipStreamSynchronize(ctx->stream), "stream synchronise");
    return GROVER_OK;
}

int grover_state_device(grover_ctx *ctx, void **dev_ptr, size_t *bytes)
{
    if (check_ctx(ctx) || !dev_ptr || !bytes)
        return fail(ctx, GROVER_E_INVAL, "null argument");
    *dev_ptr = ctx->state;
    *bytes = size_t(ctx->N) * elem_bytes(ctx->dtype);
    return GROVER_OK;
}

int grover_marked(grover_ctx *ctx, uint64_t *out, uint64_t cap, uint64_t *count)
{
    if (check_ctx(ctx) || !count || (cap > 0 && !out))
        return fail(ctx, GROVER_E_INVAL, "null argument");
    const uint64_t m = ctx->marks.size();
    const uint64_t w = m < cap ? m : cap;
    if (w > 0)
        memcpy(out, ctx->marks.data(), w * sizeof(uint64_t));
    *count = m;
    return GROVER_OK;
}

int grover_sync(grover_ctx *ctx)
{
    if (check_ctx(ctx))
        return GROVER_E_INVAL;
    GROVER_HIP(ctx, hipStreamSynchronize(ctx->stream), "stream synchronise");
    uint32_t err = 0;
    GROVER_HIP(ctx, hipMemcpy(&err, ctx->flag_dev, sizeof(err), hipMemcpyDeviceToHost), "status download");
    if (err) {
        GROVER_HIP(ctx, hipMemset(ctx->flag_dev, 0, sizeof(uint32_t)), "status reset");
        GROVER_HIP(ctx, hipDeviceSynchronize(), "status reset");
        return fail(ctx, GROVER_E_INVAL, "every outcome probability rounds to zero");
    }
    if (ctx->sync) {
        GridSync gs;
        GROVER_HIP(ctx, hipMemcpy(&gs, ctx->sync, sizeof(gs), hipMemcpyDeviceToHost), "barrier status download");
        if (gs.error) {
            if (int st = reset_barrier(ctx, "barrier reset after a timed-out wait"))
                return st;
            return fail(ctx, GROVER_E_TIMEOUT, "a grid barrier wait exceeded its limit; state undefined");
        }
    }
    return GROVER_OK;
}

int grover_query(grover_ctx *ctx, int key, int64_t *value)
{
    if (check_ctx(ctx) || !value)
        return fail(ctx, GROVER_E_INVAL, "null argument");
    switch (key) {
    case 0: *value = ctx->form; break;
    case 1: *value = ctx->grid; break;
    case 2: *value = ctx->block; break;
    case 3: *value = int64_t(elem_bytes(ctx->dtype)); break;
    case 4: *value = int64_t(ctx->N); break;
    case 5: *value = int64_t(ctx->marks.size()); break;
    case 6: *value = int64_t(ctx->timeout_ticks); break;
    case 7: *value = ctx->per_cu_reported; break;
    case 8: {  // fused form: bytes per pass streamed with ordinary accesses
        const uint64_t state = ctx->N * elem_bytes(ctx->dtype);
        const uint64_t lead = fused_temporal_tiles(ctx) * uint64_t(ctx->grid) * ctx->fused_tile * 16u;
        *value = int64_t(ctx->fused_temporal_bytes >= state ? state : std::min(state, lead));
        break;
    }
    default: return fail(ctx, GROVER_E_INVAL, "unknown query key");
    }
    return GROVER_OK;
}

void grover_destroy(grover_ctx *ctx)
{
    if (!ctx)
        return;
    (void)hipStreamSynchronize(ctx->stream);
    release(ctx);
}

}  // extern "C"
