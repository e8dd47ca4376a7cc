// grover_cli — native driver of libgrover through its C ABI (no Python, no torch), for runs and profiling.
//
//   grover_cli run  --n 28 --dtype c64 --form fused --hash-seed 0x6A09E667F3BCC910 --hash-bits 25 --m 8
//                   [--iters K] [--shots 1000000] [--shot-seed 11] [--steps 1]
//   grover_cli run  --n 10 --dtype f64 --mark 123 ...          (explicit marked indices, repeatable)
//   grover_cli copy --bytes 2147483648 [--reps 1]              (plain copy kernel of known size)
//   grover_cli stream --bytes 2147483648 [--passes 20] [--read-only | --write-only] [--launch-per-pass]
//                   (the bandwidth probe: the fused kernel's access pattern without its arithmetic)
//   grover_cli batch --instances FILE [--split S --team T [--resident V] | --tune] [--graph] [--runs R]
//                   (many searches in one launch; FILE holds one instance per line: n m mark_1 ... mark_m)
//   grover_cli phase --schedules FILE [--every S] [--team T] [--form auto|streamed|held] [--runs R]
//                   (generalized iteration: forward runs and adjoint runs; FILE holds "n m K B", the m marks,
//                    then B rows of K phases phi and B rows of K phases theta)
//   run ... --calibrate-copy B                                  (also copy B bytes once, before the search)
//   run ... --calibrate-stream B                                (and one in-place probe pass over B bytes)
//   run ... --update f32, batch ... --update f32                (the element update in binary32)
//
// `run` creates a context, then per step: writes the uniform state, runs the iterations (timed with HIP
// events on the context's stream), takes the norm and samples the shots with device-generated uniforms.
// It prints one JSON line.  `copy` moves a buffer of known size with a simple streaming kernel; its byte
// counters calibrate hardware-counter traffic measurements of the iteration kernel.
#include <hip/hip_runtime.h>

#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "grover.h"

namespace {

__global__ __launch_bounds__(256) void copy_kernel(const float4 *src, float4 *dst, uint64_t n)
{
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

int usage()
{
    fprintf(stderr,
            "usage: grover_cli run --n N [--dtype f64|c64|c128|cbf16] [--accum f64|f32|f32_kahan]\n"
            "                      [--form auto|fused|resident|two_pass|held]\n"
            "                      [--mark I ... | --hash-seed S --hash-bits B --m M] [--iters K]\n"
            "                      [--shots S] [--shot-seed U] [--steps T] [--calibrate-copy BYTES]\n"
            "                      [--calibrate-stream BYTES] [--update f64|f32]\n"
            "       grover_cli copy --bytes B [--reps R]\n"
            "       grover_cli stream --bytes B [--passes P] [--read-only | --write-only] [--launch-per-pass] [--narrow]\n"
            "       grover_cli batch --instances FILE [--split S --team T [--resident V] | --tune] [--graph] [--runs R]\n"
            "                        [--update f64|f32]\n"
            "       grover_cli phase --schedules FILE [--every S] [--team T] [--form auto|streamed|held] "
            "[--runs R]\n");
    return 2;
}

#define CHECK_HIP(x)                                                                   \
    do {                                                                               \
        const hipError_t e_ = (x);                                                     \
        if (e_ != hipSuccess) {                                                        \
            fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); \
            return 1;                                                                  \
        }                                                                              \
    } while (0)

#define CHECK_GROVER(ctx, x)                                                           \
    do {                                                                               \
        const int s_ = (x);                                                            \
        if (s_ != GROVER_OK) {                                                         \
            fprintf(stderr, "grover error %d (%s): %s\n", s_, grover_status_str(s_),   \
                    grover_last_error(ctx));                                           \
            return 1;                                                                  \
        }                                                                              \
    } while (0)

int run_copy(int argc, char **argv)
{
    uint64_t bytes = uint64_t(1) << 31;
    int reps = 1;
    for (int i = 2; i < argc; ++i) {
        if (!strcmp(argv[i], "--bytes") && i + 1 < argc)
            bytes = strtoull(argv[++i], nullptr, 0);
        else if (!strcmp(argv[i], "--reps") && i + 1 < argc)
            reps = atoi(argv[++i]);
        else
            return usage();
    }
    const uint64_t n = bytes / 16;
    float4 *a = nullptr, *b = nullptr;
    CHECK_HIP(hipMalloc(&a, n * 16));
    CHECK_HIP(hipMalloc(&b, n * 16));
    CHECK_HIP(hipMemset(a, 0, n * 16));
    CHECK_HIP(hipDeviceSynchronize());
    hipEvent_t e0, e1;
    CHECK_HIP(hipEventCreate(&e0));
    CHECK_HIP(hipEventCreate(&e1));
    CHECK_HIP(hipEventRecord(e0));
    for (int r = 0; r < reps; ++r)
        copy_kernel<<<4096, 256>>>(a, b, n);
    CHECK_HIP(hipGetLastError());
    CHECK_HIP(hipEventRecord(e1));
    CHECK_HIP(hipEventSynchronize(e1));
    float ms = 0;
    CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
    printf("{\"mode\": \"copy\", \"bytes_read\": %" PRIu64 ", \"bytes_written\": %" PRIu64
           ", \"reps\": %d, \"ms\": %.4f, \"gbs\": %.1f}\n",
           n * 16, n * 16, reps, ms, 2.0 * n * 16 * reps / (ms / 1e3) / 1e9);
    CHECK_HIP(hipEventDestroy(e0));
    CHECK_HIP(hipEventDestroy(e1));
    CHECK_HIP(hipFree(a));
    CHECK_HIP(hipFree(b));
    return 0;
}

// The bandwidth probe (grover_stream_probe): `passes` in-place nontemporal passes (or read-only) over a
// buffer of `bytes`, in the fused kernel's access pattern.
int run_stream(int argc, char **argv)
{
    uint64_t bytes = uint64_t(1) << 31;
    uint32_t passes = 20;
    int read_only = 0;
    uint32_t mode = 0;
    for (int i = 2; i < argc; ++i) {
        if (!strcmp(argv[i], "--bytes") && i + 1 < argc)
            bytes = strtoull(argv[++i], nullptr, 0);
        else if (!strcmp(argv[i], "--passes") && i + 1 < argc)
            passes = uint32_t(strtoul(argv[++i], nullptr, 0));
        else if (!strcmp(argv[i], "--read-only"))
            read_only = 1;
        else if (!strcmp(argv[i], "--launch-per-pass"))
            mode |= GROVER_PROBE_LAUNCH_PER_PASS;
        else if (!strcmp(argv[i], "--write-only"))
            mode |= GROVER_PROBE_WRITE_ONLY;
        else if (!strcmp(argv[i], "--narrow"))
            mode |= GROVER_PROBE_NARROW;
        else
            return usage();
    }
    if (read_only)
        mode |= GROVER_PROBE_READ_ONLY;
    void *buf = nullptr;
    CHECK_HIP(hipMalloc(&buf, bytes));
    CHECK_HIP(hipMemset(buf, 0, bytes));
    CHECK_HIP(hipDeviceSynchronize());
    float ms = 0.0f;
    CHECK_GROVER(nullptr, grover_stream_probe(nullptr, buf, bytes, 1, mode, &ms));  // warm
    CHECK_GROVER(nullptr, grover_stream_probe(nullptr, buf, bytes, passes, mode, &ms));
    const bool write_only = (mode & GROVER_PROBE_WRITE_ONLY) != 0u;
    const double moved = double(bytes) * passes * (read_only || write_only ? 1.0 : 2.0);
    printf("{\"mode\": \"stream\", \"bytes\": %" PRIu64 ", \"passes\": %u, \"read_only\": %s, \"write_only\": %s"
           ", \"launch_per_pass\": %s, \"ms\": %.4f, \"gbs\": %.1f}\n",
           bytes, passes, read_only ? "true" : "false", write_only ? "true" : "false",
           (mode & GROVER_PROBE_LAUNCH_PER_PASS) ? "true" : "false", ms, moved / (ms / 1e3) / 1e9);
    fflush(stdout);
    CHECK_HIP(hipFree(buf));
    return 0;
}

int run_search(int argc, char **argv)
{
    grover_config cfg;
    memset(&cfg, 0, sizeof(cfg));
    cfg.dtype = GROVER_C64;
    cfg.form = GROVER_FORM_AUTO;
    std::vector<uint64_t> marks;
    uint64_t iters = UINT64_MAX, shots = 0, shot_seed = 1, calib_bytes = 0, stream_bytes = 0;
    int steps = 1;
    bool hash = false;
    for (int i = 2; i < argc; ++i) {
        const std::string k = argv[i];
        const char *v = i + 1 < argc ? argv[i + 1] : nullptr;
        if (!v)
            return usage();
        ++i;
        if (k == "--n")
            cfg.n = uint32_t(atoi(v));
        else if (k == "--dtype")
            cfg.dtype = !strcmp(v, "f64")     ? GROVER_F64_REAL
                        : !strcmp(v, "c128")  ? GROVER_C128
                        : !strcmp(v, "cbf16") ? GROVER_CBF16
                                              : GROVER_C64;
        else if (k == "--accum")
            cfg.accum = !strcmp(v, "f32") ? GROVER_ACC_F32 : !strcmp(v, "f32_kahan") ? GROVER_ACC_F32_KAHAN : GROVER_ACC_F64;
        else if (k == "--form")
            cfg.form = !strcmp(v, "fused")      ? GROVER_FORM_FUSED
                       : !strcmp(v, "resident") ? GROVER_FORM_RESIDENT
                       : !strcmp(v, "two_pass") ? GROVER_FORM_TWO_PASS
                       : !strcmp(v, "held")     ? GROVER_FORM_HELD
                                                : GROVER_FORM_AUTO;
        else if (k == "--mark")
            marks.push_back(strtoull(v, nullptr, 0));
        else if (k == "--hash-seed") {
            cfg.hash_seed = strtoull(v, nullptr, 0);
            hash = true;
        } else if (k == "--hash-bits")
            cfg.hash_bits = uint32_t(atoi(v));
        else if (k == "--m")
            cfg.m = strtoull(v, nullptr, 0);
        else if (k == "--iters")
            iters = strtoull(v, nullptr, 0);
        else if (k == "--shots")
            shots = strtoull(v, nullptr, 0);
        else if (k == "--shot-seed")
            shot_seed = strtoull(v, nullptr, 0);
        else if (k == "--steps")
            steps = atoi(v);
        else if (k == "--calibrate-copy")
            calib_bytes = strtoull(v, nullptr, 0);
        else if (k == "--calibrate-stream")
            stream_bytes = strtoull(v, nullptr, 0);
        else if (k == "--update")
            cfg.update = !strcmp(v, "f32") ? GROVER_UPDATE_F32 : GROVER_UPDATE_F64;
        else
            return usage();
    }
    if (cfg.n == 0)
        return usage();
    if (calib_bytes > 0) {
        // the plain copy kernel of known size, in the same process, for counter calibration
        const uint64_t cn = calib_bytes / 16;
        float4 *ca = nullptr, *cb = nullptr;
        CHECK_HIP(hipMalloc(&ca, cn * 16));
        CHECK_HIP(hipMalloc(&cb, cn * 16));
        CHECK_HIP(hipMemset(ca, 0, cn * 16));
        copy_kernel<<<4096, 256>>>(ca, cb, cn);
        CHECK_HIP(hipGetLastError());
        CHECK_HIP(hipDeviceSynchronize());
        CHECK_HIP(hipFree(ca));
        CHECK_HIP(hipFree(cb));
        fprintf(stderr, "[grover_cli] calibration copy of %" PRIu64 " bytes done\n", cn * 16);
    }
    if (stream_bytes > 0) {
        // one in-place nontemporal pass of the bandwidth probe (the fused kernel's access pattern) over a
        // buffer of known size, in the same process, for counter calibration of nontemporal accesses
        void *buf = nullptr;
        CHECK_HIP(hipMalloc(&buf, stream_bytes));
        CHECK_HIP(hipMemset(buf, 0, stream_bytes));
        CHECK_HIP(hipDeviceSynchronize());
        float pms = 0.0f;
        CHECK_GROVER(nullptr, grover_stream_probe(nullptr, buf, stream_bytes, 1, 0, &pms));
        CHECK_HIP(hipFree(buf));
        fprintf(stderr, "[grover_cli] calibration stream pass over %" PRIu64 " bytes done (%.3f ms)\n",
                stream_bytes, pms);
    }
    if (hash) {
        cfg.oracle_kind = GROVER_ORACLE_HASH;
    } else {
        cfg.oracle_kind = GROVER_ORACLE_LIST;
        cfg.marked = marks.data();
        cfg.m = marks.size();
    }
    if (iters == UINT64_MAX)
        iters = grover_optimal_iterations(cfg.n, cfg.m);

    hipStream_t stream;
    CHECK_HIP(hipStreamCreate(&stream));
    grover_ctx *ctx = nullptr;
    CHECK_GROVER(nullptr, grover_init(&ctx, &cfg, stream, nullptr, 0));
    int64_t grid = 0, block = 0, form = 0;
    CHECK_GROVER(ctx, grover_query(ctx, 1, &grid));
    CHECK_GROVER(ctx, grover_query(ctx, 2, &block));
    CHECK_GROVER(ctx, grover_query(ctx, 0, &form));
    uint64_t *shots_dev = nullptr;
    if (shots > 0)
        CHECK_HIP(hipMalloc(&shots_dev, shots * sizeof(uint64_t)));
    hipEvent_t e0, e1, s0, s1;
    CHECK_HIP(hipEventCreate(&e0));
    CHECK_HIP(hipEventCreate(&e1));
    CHECK_HIP(hipEventCreate(&s0));
    CHECK_HIP(hipEventCreate(&s1));
    double it_ms_sum = 0, step_ms_sum = 0, norm = 0;
    for (int s = 0; s < steps; ++s) {
        CHECK_HIP(hipEventRecord(s0, stream));
        CHECK_GROVER(ctx, grover_reset(ctx));
        CHECK_HIP(hipEventRecord(e0, stream));
        CHECK_GROVER(ctx, grover_iterate(ctx, iters));
        CHECK_HIP(hipEventRecord(e1, stream));
        CHECK_GROVER(ctx, grover_norm(ctx, &norm));
        if (shots > 0)
            CHECK_GROVER(ctx, grover_sample(ctx, shots, shot_seed, shots_dev, 1));
        CHECK_HIP(hipEventRecord(s1, stream));
        CHECK_GROVER(ctx, grover_sync(ctx));
        float it_ms = 0, step_ms = 0;
        CHECK_HIP(hipEventElapsedTime(&it_ms, e0, e1));
        CHECK_HIP(hipEventElapsedTime(&step_ms, s0, s1));
        it_ms_sum += it_ms;
        step_ms_sum += step_ms;
        fprintf(stderr, "[grover_cli] step %d/%d: iterate %.3f ms, step %.3f ms\n", s + 1, steps, it_ms, step_ms);
    }
    CHECK_HIP(hipEventDestroy(e0));
    CHECK_HIP(hipEventDestroy(e1));
    CHECK_HIP(hipEventDestroy(s0));
    CHECK_HIP(hipEventDestroy(s1));
    const double N = double(uint64_t(1) << cfg.n);
    const double it_ms = it_ms_sum / steps;
    printf("{\"mode\": \"run\", \"n\": %u, \"dtype\": %u, \"form\": %" PRId64 ", \"m\": %" PRIu64
           ", \"iterations\": %" PRIu64 ", \"shots\": %" PRIu64 ", \"grid\": %" PRId64 ", \"block\": %" PRId64
           ", \"steps\": %d, \"iterate_ms\": %.4f, \"step_ms\": %.4f, \"updates_per_s\": %.6e, \"norm\": %.12f}\n",
           cfg.n, cfg.dtype, form, cfg.m, iters, shots, grid, block, steps, it_ms, step_ms_sum / steps,
           N * double(iters) / (it_ms / 1e3), norm);
    fflush(stdout);
    if (shots_dev)
        CHECK_HIP(hipFree(shots_dev));
    grover_destroy(ctx);
    CHECK_HIP(hipStreamDestroy(stream));
    return 0;
}

#define CHECK_BATCH(b, x)                                                              \
    do {                                                                               \
        const int s_ = (x);                                                            \
        if (s_ != GROVER_OK) {                                                         \
            fprintf(stderr, "grover batch error %d (%s): %s\n", s_, grover_status_str(s_), \
                    grover_batch_last_error(b));                                       \
            return 1;                                                                  \
        }                                                                              \
    } while (0)

int run_batch(int argc, char **argv)
{
    const char *path = nullptr;
    long split = -1, team = -1, resident = 0;
    int runs = 3;
    bool tune = false, graph = false;
    uint32_t update = GROVER_UPDATE_F64;
    for (int i = 2; i < argc; ++i) {
        if (!strcmp(argv[i], "--instances") && i + 1 < argc)
            path = argv[++i];
        else if (!strcmp(argv[i], "--split") && i + 1 < argc)
            split = strtol(argv[++i], nullptr, 0);
        else if (!strcmp(argv[i], "--team") && i + 1 < argc)
            team = strtol(argv[++i], nullptr, 0);
        else if (!strcmp(argv[i], "--resident") && i + 1 < argc)
            resident = strtol(argv[++i], nullptr, 0);
        else if (!strcmp(argv[i], "--runs") && i + 1 < argc)
            runs = atoi(argv[++i]);
        else if (!strcmp(argv[i], "--tune"))
            tune = true;
        else if (!strcmp(argv[i], "--graph"))
            graph = true;
        else if (!strcmp(argv[i], "--update") && i + 1 < argc)
            update = !strcmp(argv[++i], "f32") ? GROVER_UPDATE_F32 : GROVER_UPDATE_F64;
        else
            return usage();
    }
    if (!path || runs < 1 || (split >= 0) != (team >= 0))
        return usage();
    FILE *f = fopen(path, "r");
    if (!f) {
        fprintf(stderr, "cannot open %s\n", path);
        return 1;
    }
    std::vector<uint32_t> ns;
    std::vector<uint64_t> ms, marks;
    unsigned n = 0;
    unsigned long long m = 0;
    while (fscanf(f, "%u %llu", &n, &m) == 2) {
        ns.push_back(n);
        ms.push_back(m);
        for (unsigned long long j = 0; j < m; ++j) {
            unsigned long long x = 0;
            if (fscanf(f, "%llu", &x) != 1) {
                fclose(f);
                fprintf(stderr, "%s: instance %zu lists fewer than %llu marks\n", path, ns.size() - 1, m);
                return 1;
            }
            marks.push_back(x);
        }
    }
    fclose(f);
    if (ns.empty()) {
        fprintf(stderr, "%s: no instances\n", path);
        return 1;
    }
    grover_batch_config cfg{};
    cfg.count = ns.size();
    cfg.n = ns.data();
    cfg.m = ms.data();
    cfg.marked = marks.empty() ? nullptr : marks.data();
    cfg.dtype = GROVER_C64;
    cfg.update = update;
    hipStream_t stream;
    CHECK_HIP(hipStreamCreate(&stream));
    grover_batch *b = nullptr;
    CHECK_BATCH(nullptr, grover_batch_init(&b, &cfg, stream));
    if (split >= 0)
        CHECK_BATCH(b, grover_batch_set_tiling(b, uint32_t(split), uint32_t(team), uint32_t(resident)));
    if (tune) {
        uint32_t s = 0, t = 0, r = 0;
        float ms_best = 0;
        CHECK_BATCH(b, grover_batch_tune(b, &s, &t, &r, &ms_best));
        fprintf(stderr, "[grover_cli] tuned tiling split=%u team=%u resident=%u (%.3f ms)\n", s, t, r, ms_best);
    }
    if (graph)
        CHECK_BATCH(b, grover_batch_capture(b));
    int64_t updates = 0, grid = 0, sp = 0, tm = 0;
    CHECK_BATCH(b, grover_batch_query(b, 4, &updates));
    CHECK_BATCH(b, grover_batch_query(b, 1, &grid));
    CHECK_BATCH(b, grover_batch_query(b, 2, &sp));
    CHECK_BATCH(b, grover_batch_query(b, 3, &tm));
    hipEvent_t e0, e1;
    CHECK_HIP(hipEventCreate(&e0));
    CHECK_HIP(hipEventCreate(&e1));
    double ms_sum = 0;
    for (int r = 0; r < runs; ++r) {
        CHECK_HIP(hipEventRecord(e0, stream));
        CHECK_BATCH(b, grover_batch_run(b));
        CHECK_HIP(hipEventRecord(e1, stream));
        CHECK_BATCH(b, grover_batch_sync(b));
        float ms = 0;
        CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
        ms_sum += ms;
        fprintf(stderr, "[grover_cli] batch run %d/%d: %.3f ms\n", r + 1, runs, ms);
    }
    CHECK_HIP(hipEventDestroy(e0));
    CHECK_HIP(hipEventDestroy(e1));
    const double run_ms = ms_sum / runs;
    printf("{\"mode\": \"batch\", \"instances\": %zu, \"amplitude_updates\": %" PRId64 ", \"grid\": %" PRId64
           ", \"split_n\": %" PRId64 ", \"team\": %" PRId64 ", \"graph\": %s, \"runs\": %d, \"ms_per_run\": %.4f"
           ", \"updates_per_s\": %.6e}\n",
           ns.size(), updates, grid, sp, tm, graph ? "true" : "false", runs, run_ms,
           double(updates) / (run_ms / 1e3));
    fflush(stdout);
    grover_batch_destroy(b);
    CHECK_HIP(hipStreamDestroy(stream));
    return 0;
}

#define CHECK_PHASE(p, x)                                                              \
    do {                                                                               \
        const int s_ = (x);                                                            \
        if (s_ != GROVER_OK) {                                                         \
            fprintf(stderr, "grover phase error %d (%s): %s\n", s_, grover_status_str(s_), \
                    grover_phase_last_error(p));                                       \
            return 1;                                                                  \
        }                                                                              \
    } while (0)

int run_phase(int argc, char **argv)
{
    const char *path = nullptr;
    unsigned every = 0, team = 0, form = GROVER_PHASE_FORM_AUTO;
    int runs = 3;
    for (int i = 2; i < argc; ++i) {
        if (!strcmp(argv[i], "--schedules") && i + 1 < argc)
            path = argv[++i];
        else if (!strcmp(argv[i], "--form") && i + 1 < argc) {
            const std::string fm = argv[++i];
            if (fm == "auto")
                form = GROVER_PHASE_FORM_AUTO;
            else if (fm == "streamed")
                form = GROVER_PHASE_FORM_STREAMED;
            else if (fm == "held")
                form = GROVER_PHASE_FORM_HELD;
            else
                return usage();
        }
        else if (!strcmp(argv[i], "--every") && i + 1 < argc)
            every = unsigned(atoi(argv[++i]));
        else if (!strcmp(argv[i], "--team") && i + 1 < argc)
            team = unsigned(atoi(argv[++i]));
        else if (!strcmp(argv[i], "--runs") && i + 1 < argc)
            runs = atoi(argv[++i]);
        else
            return usage();
    }
    if (!path || runs < 1)
        return usage();
    FILE *f = fopen(path, "r");
    if (!f) {
        fprintf(stderr, "cannot open %s\n", path);
        return 1;
    }
    unsigned n = 0, K = 0, B = 0;
    unsigned long long m = 0;
    bool ok = fscanf(f, "%u %llu %u %u", &n, &m, &K, &B) == 4 && K > 0 && B > 0 && m < (1ull << 20);
    std::vector<uint64_t> marks(ok ? m : 0);
    for (auto &x : marks) {
        unsigned long long v = 0;
        ok = ok && fscanf(f, "%llu", &v) == 1;
        x = v;
    }
    std::vector<double> params(ok ? size_t(2) * B * K : 0);
    for (auto &x : params)
        ok = ok && fscanf(f, "%lf", &x) == 1;
    fclose(f);
    if (!ok) {
        fprintf(stderr, "%s: malformed schedule file\n", path);
        return 1;
    }
    grover_phase_config cfg{};
    cfg.n = n;
    cfg.batch = B;
    cfg.iterations = K;
    cfg.checkpoint_every = every;
    cfg.marked = marks.empty() ? nullptr : marks.data();
    cfg.m = marks.size();
    cfg.dtype = GROVER_C64;
    hipStream_t stream;
    CHECK_HIP(hipStreamCreate(&stream));
    grover_phase *p = nullptr;
    CHECK_PHASE(nullptr, grover_phase_init(&p, &cfg, stream));
    if (team)
        CHECK_PHASE(p, grover_phase_set_team(p, team));
    CHECK_PHASE(p, grover_phase_set_form(p, form));
    const size_t pb = size_t(B) * K * sizeof(double);
    double *d_par = nullptr, *d_loss = nullptr, *d_dloss = nullptr, *d_grad = nullptr;
    CHECK_HIP(hipMalloc(&d_par, 2 * pb));
    CHECK_HIP(hipMalloc(&d_loss, B * sizeof(double)));
    CHECK_HIP(hipMalloc(&d_dloss, B * sizeof(double)));
    CHECK_HIP(hipMalloc(&d_grad, 2 * pb));
    CHECK_HIP(hipMemcpy(d_par, params.data(), 2 * pb, hipMemcpyHostToDevice));
    std::vector<double> ones(B, 1.0);
    CHECK_HIP(hipMemcpy(d_dloss, ones.data(), B * sizeof(double), hipMemcpyHostToDevice));
    hipEvent_t e0, e1, e2;
    CHECK_HIP(hipEventCreate(&e0));
    CHECK_HIP(hipEventCreate(&e1));
    CHECK_HIP(hipEventCreate(&e2));
    double fsum = 0, bsum = 0;
    for (int r = 0; r < runs; ++r) {
        CHECK_HIP(hipEventRecord(e0, stream));
        CHECK_PHASE(p, grover_phase_forward(p, d_par, d_par + size_t(B) * K, d_loss));
        CHECK_HIP(hipEventRecord(e1, stream));
        CHECK_PHASE(p, grover_phase_backward(p, d_dloss, d_grad, d_grad + size_t(B) * K));
        CHECK_HIP(hipEventRecord(e2, stream));
        CHECK_PHASE(p, grover_phase_sync(p));
        float fm = 0, bm = 0;
        CHECK_HIP(hipEventElapsedTime(&fm, e0, e1));
        CHECK_HIP(hipEventElapsedTime(&bm, e1, e2));
        fsum += fm;
        bsum += bm;
        fprintf(stderr, "[grover_cli] phase run %d/%d: forward %.3f ms, adjoint %.3f ms\n", r + 1, runs, fm, bm);
    }
    double loss0 = 0;
    CHECK_HIP(hipMemcpy(&loss0, d_loss, sizeof(double), hipMemcpyDeviceToHost));
    int64_t grid = 0, tm = 0, ev = 0, fo = 0, tf = 0, ta = 0;
    CHECK_PHASE(p, grover_phase_query(p, 1, &grid));
    CHECK_PHASE(p, grover_phase_query(p, 2, &tm));
    CHECK_PHASE(p, grover_phase_query(p, 3, &ev));
    CHECK_PHASE(p, grover_phase_query(p, 6, &fo));
    CHECK_PHASE(p, grover_phase_query(p, 7, &tf));
    CHECK_PHASE(p, grover_phase_query(p, 8, &ta));
    if (fo == GROVER_PHASE_FORM_HELD)  // the held form sizes its teams from the state
        tm = tf;
    const double upd = double(B) * K * double(uint64_t(1) << n);
    printf("{\"mode\": \"phase\", \"n\": %u, \"m\": %zu, \"K\": %u, \"batch\": %u, \"grid\": %" PRId64
           ", \"team\": %" PRId64 ", \"adjoint_team\": %" PRId64 ", \"form\": \"%s\", \"every\": %" PRId64
           ", \"runs\": %d, \"forward_ms\": %.4f, \"adjoint_ms\": %.4f"
           ", \"forward_updates_per_s\": %.6e, \"loss0\": %.12f}\n",
           n, marks.size(), K, B, grid, tm, fo == GROVER_PHASE_FORM_HELD ? ta : tm,
           fo == GROVER_PHASE_FORM_HELD ? "held" : "streamed", ev, runs, fsum / runs, bsum / runs,
           upd / (fsum / runs / 1e3), loss0);
    fflush(stdout);
    CHECK_HIP(hipEventDestroy(e0));
    CHECK_HIP(hipEventDestroy(e1));
    CHECK_HIP(hipEventDestroy(e2));
    CHECK_HIP(hipFree(d_par));
    CHECK_HIP(hipFree(d_loss));
    CHECK_HIP(hipFree(d_dloss));
    CHECK_HIP(hipFree(d_grad));
    grover_phase_destroy(p);
    CHECK_HIP(hipStreamDestroy(stream));
    return 0;
}

// With GROVER_CLI_MAPS=FILE in the environment, the process's memory map is copied to FILE when main
// returns, so that addresses a crash handler prints after that (in exit-time destructors) can be matched
// to the libraries that hold them.
void save_maps()
{
    const char *path = getenv("GROVER_CLI_MAPS");
    if (!path || !*path)
        return;
    FILE *in = fopen("/proc/self/maps", "r");
    FILE *out = fopen(path, "w");
    if (in && out) {
        char buf[4096];
        size_t n;
        while ((n = fread(buf, 1, sizeof(buf), in)) > 0)
            fwrite(buf, 1, n, out);
    }
    if (in)
        fclose(in);
    if (out)
        fclose(out);
}

int dispatch(int argc, char **argv)
{
    if (argc < 2)
        return usage();
    if (!strcmp(argv[1], "copy"))
        return run_copy(argc, argv);
    if (!strcmp(argv[1], "stream"))
        return run_stream(argc, argv);
    if (!strcmp(argv[1], "run"))
        return run_search(argc, argv);
    if (!strcmp(argv[1], "batch"))
        return run_batch(argc, argv);
    if (!strcmp(argv[1], "phase"))
        return run_phase(argc, argv);
    return usage();
}

}  // namespace

int main(int argc, char **argv)
{
    const int rc = dispatch(argc, argv);
    save_maps();
    return rc;
}
