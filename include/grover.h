/*
 * grover.h — C ABI of libgrover, an MI355X (gfx950) implementation of the fast Grover-search simulation of
 * Chattopadhyay and Menon, "Fast simulation of Grover's quantum search on classical computer"
 * (arXiv:2005.04635).
 *
 * The library keeps an N = 2^n amplitude state vector in device memory and advances it by Grover iterations
 * computed the paper's way: a sign flip of the marked amplitudes (the proposed Oracle, Algorithm 3) followed
 * by inversion about the mean, c_i <- 2*mean - c_i (Eq. 2 and Algorithm 4), repeated as in Algorithm 5.
 * For comparison it also runs the conventional gate-level iteration of Algorithm 2 (H^n built from the
 * 1-qubit unitary of Algorithm 1, the conditional phase shift 2|0><0| - I, H^n again).
 *
 * Conventions shared by every call
 *   - State layout (Background, "Quantum State"): a contiguous array indexed by basis state i, 0 <= i < N;
 *     bit q of i is qubit q.  Element types: GROVER_F64_REAL = one double per amplitude (imaginary part 0);
 *     GROVER_C64 = interleaved float (re, im); GROVER_C128 = interleaved double (re, im).
 *   - Signs: the oracle negates marked amplitudes; the diffusion is 2|psi><psi| - I with |psi> the uniform
 *     superposition, i.e. c_i <- 2*S/N - c_i with S = sum_i c_i (real and imaginary parts, no conjugation)
 *     of the oracle-flipped state.  The conditional phase shift is 2|0><0| - I.
 *   - Every function returns an int status (GROVER_OK = 0, or a negative GROVER_E_* code) and never aborts
 *     or throws.  grover_last_error(ctx) gives a message for the last failure on that context.
 *   - Device work is enqueued on the context's HIP stream and is asynchronous unless stated otherwise.
 *     Calls that deliver results to host memory synchronise that stream before returning.
 *   - A context is not thread-safe; distinct contexts are independent.  All pointers are plain host or
 *     device addresses; no torch or other framework type crosses this boundary.
 */
#ifndef GROVER_H
#define GROVER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------------------------------ status */
#define GROVER_OK 0
#define GROVER_E_INVAL (-1)       /* invalid argument (sizes, pointers, marked list, enum values) */
#define GROVER_E_NOMEM (-2)       /* device or host allocation failed */
#define GROVER_E_HIP (-3)         /* a HIP runtime call failed; message in grover_last_error */
#define GROVER_E_COOP (-4)        /* the persistent grid cannot be made co-resident on this device */
#define GROVER_E_UNSUPPORTED (-5) /* valid request the library does not implement (e.g. form/size mismatch) */
#define GROVER_E_PREDICATE (-6)   /* hash predicate hit count differs from the requested m */
#define GROVER_E_TIMEOUT (-7)     /* a device-side grid barrier exceeded its time limit (reported by grover_sync) */

/* ----------------------------------------------------------------------------------------- enums */
typedef enum grover_dtype {
    GROVER_F64_REAL = 0, /* double per amplitude, imaginary parts identically 0 */
    GROVER_C64 = 1,      /* complex64: float re, float im; update computed in binary64, stored rounded */
    GROVER_C128 = 2,     /* complex128: double re, double im */
    GROVER_CBF16 = 3     /* complex bfloat16: bf16 re, bf16 im (4 bytes); update in binary64, rounded once
                            to nearest even; fused form only */
} grover_dtype;

/* Precision of the sum S = sum_i s_i c_i that the mean is taken from (per-thread accumulation and the
 * reduction tree above it).  The precision of the update c' = 2S/N - s c is grover_update. */
typedef enum grover_accum {
    GROVER_ACC_F64 = 0,       /* binary64 (default) */
    GROVER_ACC_F32 = 1,       /* binary32; fused form only */
    GROVER_ACC_F32_KAHAN = 2  /* binary32 with Kahan-compensated per-thread sums; fused form only */
} grover_accum;

/* Precision of the element update c' = 2S/N - s c (Algorithm 4's second loop). */
typedef enum grover_update {
    GROVER_UPDATE_F64 = 0, /* computed in binary64 from 2S/N and rounded once to the storage type (default) */
    GROVER_UPDATE_F32 = 1  /* complex64 storage with binary64 sums only: 2S/N rounded to binary32, then each
                              part of c' = fl32(2S/N) - s c is one binary32 operation; forms FUSED, RESIDENT,
                              HELD (AUTO picks among them as for GROVER_UPDATE_F64) */
} grover_update;

typedef enum grover_oracle_kind {
    GROVER_ORACLE_LIST = 0, /* marked set given as an explicit list of indices (Algorithm 3's k[]) */
    GROVER_ORACLE_HASH = 1  /* i is marked iff the low hash_bits bits of SplitMix64_i(hash_seed) are 0 */
} grover_oracle_kind;

typedef enum grover_form {
    GROVER_FORM_AUTO = 0,     /* RESIDENT for n <= 14 with f64/c64/c128 storage and binary64 sums; HELD for
                                 larger complex64 states with binary64 sums while they fit on chip; else FUSED */
    GROVER_FORM_FUSED = 1,    /* one persistent cooperative kernel per grover_iterate call, one grid
                                 barrier per iteration, update fused with the next iteration's sum */
    GROVER_FORM_RESIDENT = 2, /* one workgroup holds the whole state on chip (n <= 14) */
    GROVER_FORM_TWO_PASS = 3, /* plain form: per iteration an oracle flip, a sum pass and an update pass,
                                 launched from the host (Algorithms 3 and 4 as separate kernels) */
    GROVER_FORM_HELD = 4      /* complex64 with binary64 sums only: a team of T workgroups (a power of two;
                                 about 2 16-byte vectors per thread up to 64 workgroups, at most 8 per
                                 thread in registers while T <= 128, else 16 with 8 in LDS) loads the state once
                                 per grover_iterate call and keeps it on chip for all k iterations, one team
                                 barrier each; n <= 23 on 256 CUs (GROVER_E_UNSUPPORTED when the state does
                                 not fit) */
} grover_form;

/* ---------------------------------------------------------------------------------------- config */
typedef struct grover_config {
    uint32_t n;              /* qubits, 1 <= n <= 34; N = 2^n amplitudes (GROVER_CBF16: n >= 2, since every
                                kernel moves whole 16-byte vectors; n = 1 is GROVER_E_UNSUPPORTED) */
    uint32_t dtype;          /* grover_dtype */
    uint32_t oracle_kind;    /* grover_oracle_kind */
    uint32_t hash_bits;      /* HASH only: width of the zero test, 0 <= hash_bits <= 64 */
    const uint64_t *marked;  /* LIST only: host array of m distinct indices < N, any order; copied */
    uint64_t m;              /* LIST: length of `marked`; HASH: required number of hits (checked) */
    uint64_t hash_seed;      /* HASH only: SplitMix64 seed of the predicate */
    uint32_t form;           /* grover_form */
    uint32_t flags;          /* reserved, must be 0 */
    uint32_t accum;          /* grover_accum */
    uint32_t update;         /* grover_update */
} grover_config;

typedef struct grover_ctx grover_ctx;

/* grover_init — create a context and prepare the initial state (Algorithm 5: psi = H^n |0>).
 *   out         receives the new context (set to NULL on failure).
 *   cfg         problem description, validated: n range, dtype/form/kind/accum/update values, flags == 0,
 *               the form supports the dtype, accum and update (else GROVER_E_UNSUPPORTED), marked
 *               indices distinct and < N, m <= N; for HASH the predicate is evaluated on the device over
 *               all N indices, its hits compacted into the marked list, and GROVER_E_PREDICATE returned
 *               when their number differs from cfg->m.
 *   hip_stream  hipStream_t to run on (e.g. torch.cuda.current_stream().cuda_stream), NULL = default
 *               stream.  The device is the one current when grover_init is called.
 *   state_dev   optional caller-owned device buffer of at least state_bytes = N * element size bytes,
 *               16-byte aligned; the library uses it as the state and never frees it.  NULL: the context
 *               allocates and owns the state.
 *   state_bytes size of state_dev in bytes (ignored when state_dev is NULL).
 * The state is written as the uniform superposition 2^(-n/2) (correctly rounded to the element type).
 * Synchronises the stream once (HASH: to read back the hit count). */
int grover_init(grover_ctx **out, const grover_config *cfg, void *hip_stream, void *state_dev,
                size_t state_bytes);

/* grover_reset — overwrite the state with the uniform superposition again (marked set unchanged). */
int grover_reset(grover_ctx *ctx);

/* grover_iterate — k Grover iterations of the proposed method (Algorithm 5's loop body: Algorithm 3 then
 * Algorithm 4) in the context's form.  k = 0 is a no-op.  The sum of the current state is recomputed at the
 * start of every call, so edits made through grover_write_state or the device pointer are honoured, and
 * grover_iterate(a) followed by grover_iterate(b) gives bit for bit the state of grover_iterate(a + b).
 * Asynchronous. */
int grover_iterate(grover_ctx *ctx, uint64_t k);

/* grover_gate_iterate — k iterations of the conventional gate-level simulator (Algorithm 2's loop body):
 * oracle sign flip, H^n as n single-qubit passes (Algorithm 1 with U = H), the conditional phase shift
 * 2|0><0| - I, H^n again.  Asynchronous.  GROVER_E_UNSUPPORTED for bfloat16 storage. */
int grover_gate_iterate(grover_ctx *ctx, uint64_t k);

/* grover_apply_hadamard_all — psi <- H^n psi as n single-qubit passes (Algorithm 1).  Asynchronous.
 * GROVER_E_UNSUPPORTED for bfloat16 storage. */
int grover_apply_hadamard_all(grover_ctx *ctx);

/* grover_gate_iterate_blocked / grover_apply_hadamard_all_blocked — the same operators (Algorithm 2's
 * iteration; H^n) with H^n computed as a blocked Walsh-Hadamard transform: qubits are transformed in
 * groups held in LDS (12 or 13 low qubits per pass, then 8 or 9 per pass), with unnormalised butterflies in
 * binary64 and the normalisation applied once (2^(-n/2) for H^n; for the iteration the exact 2^(-n) of
 * both transforms, with the conditional phase shift fused into the first transform's last pass).  At
 * n = 28 an H^n is 3 passes instead of 28.  Results equal the single-qubit path's up to rounding (one
 * rounding to the storage type per pass instead of per qubit).  Asynchronous; GROVER_E_UNSUPPORTED for
 * bfloat16 storage. */
int grover_gate_iterate_blocked(grover_ctx *ctx, uint64_t k);
int grover_apply_hadamard_all_blocked(grover_ctx *ctx);

/* grover_sample — measurement (Background, step 6; the paper gives no procedure, this library defines it):
 *   p_i = re_i^2 + im_i^2 in binary64 (no fused multiply-add), q_i = floor(p_i * 2^62) as uint64,
 *   Q_i = q_0 + ... + q_i (exact integer prefix sum), and for shot j with 53-bit uniform U_j:
 *   t_j = floor(U_j * Q_{N-1} / 2^53), index_j = the smallest i with Q_i > t_j.
 * Because the CDF is an integer prefix sum, the result depends only on the state's bits, not on the order
 * of the device's scan.
 *   shots        number of shots (0 allowed).
 *   seed         U_j = SplitMix64_j(seed) >> 11, generated on the device.
 *   out          shots uint64 indices; a device pointer when out_is_device != 0, else host memory (the call
 *                then synchronises).  Returns GROVER_E_INVAL when every q_i is 0 (reported after a sync).
 * Allocates an N-entry uint64 CDF on first use (kept by the context). */
int grover_sample(grover_ctx *ctx, uint64_t shots, uint64_t seed, uint64_t *out, int out_is_device);

/* grover_sample_u53 — as grover_sample with caller-supplied uniforms u53[0..shots) (host or device memory
 * as u53_is_device says); only their low 53 bits are used. */
int grover_sample_u53(grover_ctx *ctx, const uint64_t *u53, int u53_is_device, uint64_t shots,
                      uint64_t *out, int out_is_device);

/* grover_norm — sum_i |c_i|^2 in binary64 with a fixed summation order (Background: it equals 1).
 * Synchronises; *out receives the value. */
int grover_norm(grover_ctx *ctx, double *out);

/* grover_read_state / grover_write_state — copy the whole state to / from host memory (bytes must equal
 * N * element size).  Synchronous. */
int grover_read_state(grover_ctx *ctx, void *host, size_t bytes);
int grover_write_state(grover_ctx *ctx, const void *host, size_t bytes);

/* grover_state_device — device address and size in bytes of the state. */
int grover_state_device(grover_ctx *ctx, void **dev_ptr, size_t *bytes);

/* grover_marked — the marked list, sorted ascending: writes min(cap, m) entries to host `out` and the total
 * count to *count. */
int grover_marked(grover_ctx *ctx, uint64_t *out, uint64_t cap, uint64_t *count);

/* grover_sync — wait for the context's stream and report device-side failures (GROVER_E_TIMEOUT when a
 * grid barrier gave up; the context is then usable again and the state undefined until reset/written). */
int grover_sync(grover_ctx *ctx);

/* grover_query — launch facts for diagnostics.  key: 0 = resolved form, 1 = persistent grid size
 * (workgroups; the held form's team), 2 = workgroup size, 3 = element size in bytes, 4 = N, 5 = number of marked indices,
 * 6 = grid-barrier wait limit in device wall-clock ticks, 7 = workgroups per CU of the fused kernel as the
 * runtime's occupancy calculator reports them (the grid actually used is confirmed on the device), 8 = bytes
 * of the state per pass that the fused kernel streams with ordinary loads and stores, so that the next pass
 * finds them in the memory-side cache (the whole state up to 272 MiB; above that, the leading tiles of each
 * workgroup's share up to 272 MiB in all, the rest with nontemporal accesses; 0 for the other forms).  The
 * environment variable GROVER_FUSED_TEMPORAL, read at grover_init, forces 0 (all nontemporal) or 1 (all
 * ordinary).  Results are identical either way. */
int grover_query(grover_ctx *ctx, int key, int64_t *value);

/* grover_stream_probe — measurement helper, not a step of the method: the bandwidth ceiling that the fused
 * iteration (Algorithm 5's loop as one streaming pass per iteration) is measured against.  It runs the
 * fused kernel's streaming skeleton without its arithmetic over a caller-owned device buffer: the same
 * persistent grid (one 512-thread workgroup per CU), 64 KiB tiles each owned by one workgroup in every
 * pass, eight nontemporal 16-byte buffer loads and stores per thread and tile (as for a complex64 state).  Each pass negates every 16-byte vector in place (a read and a
 * write of `bytes`), or, with GROVER_PROBE_READ_ONLY in `mode`, only reads it, or, with
 * GROVER_PROBE_WRITE_ONLY, only writes it (the pass number as values; not with READ_ONLY).  The `passes` passes run in
 * one launch (the workgroups move through them freely), or with GROVER_PROBE_LAUNCH_PER_PASS one launch
 * each (a pass starts when the previous one has ended everywhere, as after the fused kernel's grid barrier);
 * GROVER_PROBE_NARROW moves the same 64 KiB tiles with 1024-thread workgroups of 4 vectors per thread;
 * on hip_stream (NULL = default stream), timed there with HIP events; the call synchronises and writes the
 * elapsed milliseconds to *ms_out.
 *   buf_dev  device, 16-byte aligned, bytes >= 16 (a tail shorter than 16 bytes is not touched); its values
 *            are negated `passes` times (the same again after an even number), or overwritten (write-only).
 * GROVER_E_INVAL for bad arguments or unknown mode bits, GROVER_E_HIP when a runtime call fails. */
#define GROVER_PROBE_READ_ONLY 1u
#define GROVER_PROBE_LAUNCH_PER_PASS 2u
#define GROVER_PROBE_WRITE_ONLY 4u
#define GROVER_PROBE_NARROW 8u /* 1024-thread workgroups with 4 vectors per thread per tile (same tiles) */
int grover_stream_probe(void *hip_stream, void *buf_dev, size_t bytes, uint32_t passes, uint32_t mode,
                        float *ms_out);

/* grover_optimal_iterations — floor(pi/4 * sqrt(2^n / m)) (Algorithm 5's iteration count with m
 * solutions; the Fig. 2 example fixes the floor), 0 when m == 0 or m > 2^n or n > 63. */
uint64_t grover_optimal_iterations(uint32_t n, uint64_t m);

/* grover_destroy — release the context and everything it owns (not a caller-provided state buffer).
 * Waits for the stream first.  NULL is ignored. */
void grover_destroy(grover_ctx *ctx);

/* grover_status_str — static text for a status code.  grover_last_error — the last failure message on ctx
 * (empty string when none); with ctx NULL, the message of the last grover_init failure on the calling
 * thread that got past validation (or of the last failed grover_iterate_static call), else a static
 * message. */
const char *grover_status_str(int status);
const char *grover_last_error(const grover_ctx *ctx);

/* grover_iterate_static — for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): k iterations of the proposed method exactly as
 * grover_iterate computes them on a GROVER_FORM_FUSED context with binary64 sums (the same kernel, grid and
 * order of additions, so the same bits), on a state and a marked list the caller holds, with no context.
 * The grid barrier's memory is a fixed array inside the library, 17472 bytes per GPU (barrier slots for a
 * persistent grid of at most 256 workgroups), held until the process ends; nothing is allocated or freed.
 *   hip_stream  stream to enqueue on (NULL = default); the device is the current one.
 *   state_dev   device, 2^n amplitudes of `dtype` (grover_dtype), 16-byte aligned; updated in place.
 *   n           1 .. 34 (GROVER_CBF16: from 2).
 *   marks_dev   device, m strictly increasing indices < 2^n (checked on the device: otherwise the state is
 *               left untouched and the status word reads 2); may be NULL when m = 0.
 *   k           iterations, k < 2^32 - 2 (0: nothing is iterated; the marked list is still checked).
 *   status_dev  optional device uint32, written after the iterations: 0 = done, 1 = a grid-barrier wait
 *               exceeded its 10 s limit (state undefined), 2 = marked list rejected (state untouched).
 * Host-side validation failures return GROVER_E_INVAL / GROVER_E_UNSUPPORTED before any device work, with
 * a message in grover_last_error(NULL).  Asynchronous.  Every call on one GPU shares that GPU's barrier
 * memory and clears it first: calls whose device work overlaps (on different streams) race and must not be
 * made. */
int grover_iterate_static(void *hip_stream, void *state_dev, uint32_t n, uint32_t dtype, const uint64_t *marks_dev,
                          uint64_t m, uint64_t k, uint32_t *status_dev);

/* ------------------------------------------------------------------------------------- batches
 * Many independent searches advanced together (Algorithm 5 per instance, from the uniform superposition of
 * Algorithm 5's first step, with the oracle of Algorithm 3 and the inversion of Eq. 2 / Algorithm 4), in
 * one persistent launch.  Instance states are GROVER_C64 (interleaved float re, im; the sums are computed in
 * binary64 and the update in the precision cfg->update names, as in the single-state GROVER_C64 +
 * GROVER_ACC_F64 context with that update).  Instance i has n[i] qubits (1 <= n[i] <= 24), m[i] marked
 * indices and iterations[i] iterations (k_opt(n[i], m[i]) when `iterations` is NULL).
 *
 * How the device divides the work is the tiling (split_n, team, resident):
 *   - states of 2^n <= 32768 amplitudes are iterated by one workgroup each, held on chip (16 16-byte
 *     vectors per thread: 8 in registers, 8 in LDS);
 *   - with resident = r in {1, 2, 4, 8, 16}, a larger state is held on chip by a team of T workgroups,
 *     T the power of two >= 2^n / (2048 r) (r 16-byte vectors per thread, the first 8 in registers, the
 *     rest in LDS), when T does not exceed the grid: one team barrier per iteration and no memory traffic
 *     until the final write;
 *   - the remaining states stream from memory every iteration: those with n >= split_n by teams of `team`
 *     workgroups each (team = grid size: the whole device per instance), the others one per workgroup.
 * The tiling changes the order of additions in the sums, so results of two tilings agree to rounding, and
 * one tiling's results are reproducible bit for bit.  grover_batch_tune times candidates and keeps the
 * fastest. */
typedef struct grover_batch grover_batch;

typedef struct grover_batch_config {
    uint64_t count;              /* number of instances, >= 1 */
    const uint32_t *n;           /* host, count entries */
    const uint64_t *m;           /* host, count entries; m[i] <= 2^n[i] */
    const uint64_t *marked;      /* host, sum(m) entries: instance 0's list, then instance 1's, ... (any order
                                    within a list, no duplicates, each < 2^n[i]); may be NULL when sum(m) = 0 */
    const uint64_t *iterations;  /* host, count entries, or NULL for k_opt(n[i], m[i]) */
    uint32_t dtype;              /* GROVER_C64 (other types: GROVER_E_UNSUPPORTED) */
    uint32_t flags;              /* must be 0 */
    uint32_t update;             /* grover_update: the element update in binary64 (default) or binary32 */
    uint32_t reserved;           /* must be 0 */
} grover_batch_config;

/* grover_batch_init — validate cfg, copy its arrays, allocate every instance's state (each 256-byte
 * aligned) and the device work queues, and confirm the persistent grid on the device (one short run, as for
 * the fused form).  hip_stream: the hipStream_t all batch work goes to (NULL = default stream; graph capture
 * then unavailable).  Synchronous.  GROVER_E_INVAL for a bad config (before any device work),
 * GROVER_E_UNSUPPORTED for a dtype other than GROVER_C64, GROVER_E_COOP when no grid is co-resident.
 * The initial tiling is split_n = 19, team = 2, resident = 16. */
int grover_batch_init(grover_batch **out, const grover_batch_config *cfg, void *hip_stream);

/* grover_batch_set_tiling — choose the tiling: team in [1, grid size] (team = 1: no streamed teams),
 * resident in {0, 1, 2, 4, 8, 16} (0: no teams that hold a state on chip).  GROVER_E_INVAL outside those ranges,
 * GROVER_E_UNSUPPORTED when a streamed team size does not divide the resident teams' sizes.  Drops a
 * captured graph.  Synchronous. */
int grover_batch_set_tiling(grover_batch *b, uint32_t split_n, uint32_t team, uint32_t resident);

/* grover_batch_tune — run the batch once per candidate tiling (streamed: team = 1, and split_n in
 * {18, 19, 20} x team in {2, 4, 8}; held on chip: resident in {16, 8, 4} with split_n = 19, team = 2),
 * keep the fastest, and report it (any output pointer may be NULL).  Overwrites the states; synchronous;
 * drops a captured graph. */
int grover_batch_tune(grover_batch *b, uint32_t *split_n, uint32_t *team, uint32_t *resident, float *best_ms);

/* grover_batch_capture — record one run (queue reset + the persistent launch) into a HIP graph that later
 * grover_batch_run calls replay.  Needs a non-NULL stream; GROVER_E_UNSUPPORTED when the runtime cannot
 * capture the launch (runs then stay eager). */
int grover_batch_capture(grover_batch *b);

/* grover_batch_run — enqueue one run of the whole batch: every instance restarts from the uniform
 * superposition and performs its iterations.  Asynchronous. */
int grover_batch_run(grover_batch *b);

/* grover_batch_sync — wait for the stream; GROVER_E_TIMEOUT when a team barrier gave up during the last
 * run (results of that run undefined). */
int grover_batch_sync(grover_batch *b);

/* grover_batch_state — device address and size in bytes (2^n[i] * 8) of instance i's state. */
int grover_batch_state(grover_batch *b, uint64_t i, void **dev_ptr, size_t *bytes);

/* grover_batch_read_state — copy instance i's state to host memory; bytes must equal its size.
 * Synchronises the stream. */
int grover_batch_read_state(grover_batch *b, uint64_t i, void *host, size_t bytes);

/* grover_batch_query — key: 0 = count, 1 = persistent grid size, 2 = split_n, 3 = team, 4 = total amplitude
 * updates per run (sum of 2^n[i] * iterations[i]), 5 = 1 when a captured graph is in use, 6 = bytes of all
 * states, 7 = instances iterated by multi-workgroup teams, 8 = resident, 9 = phases of the tiling,
 * 10 = 1 when some state of the tiling streams from memory (0: every state is held on chip, and the run uses
 * the kernel compiled without the streamed paths). */
int grover_batch_query(grover_batch *b, int key, int64_t *value);

/* grover_batch_destroy — wait for the stream and release everything.  NULL is ignored. */
void grover_batch_destroy(grover_batch *b);

/* grover_batch_last_error — message of the last failure on b (a static message when b is NULL). */
const char *grover_batch_last_error(const grover_batch *b);

/* ------------------------------------------------------------ generalized iteration and its adjoint
 * A generalization of Algorithm 5 with a phase per iteration (a convention of this library; at
 * phi = theta = pi it is the paper's iteration): iteration j = 1 .. K applies
 *   O(phi_j):   c_i <- e^{i phi_j} c_i on the marked indices (Algorithm 3 at phi = pi), then
 *   D(theta_j): c_i <- (1 - e^{i theta_j}) S / N - c_i, S = sum_i c_i  (Eq. 2 at theta = pi),
 * from the uniform superposition, and the loss is L = 1 - sum over marked i of |c_i|^2.  A context runs
 * B schedules (phi, theta of shape [B][K]) over the same marked set, each on its own complex64 state
 * (binary64 phases, sums and element arithmetic).
 * The gradient dL/dphi, dL/dtheta comes from a reverse sweep that rebuilds each earlier state with the
 * inverse steps D(-theta), O(-phi) while carrying the adjoint state back, and re-reads the state from a
 * checkpoint every `checkpoint_every` iterations (stored by the forward run), so memory is
 * (2 + floor((K - 1) / checkpoint_every)) states per schedule rather than K + 1. */
typedef struct grover_phase grover_phase;

typedef struct grover_phase_config {
    uint32_t n;                /* qubits, 1 <= n <= 30 */
    uint32_t batch;            /* schedules B >= 1 */
    uint32_t iterations;       /* K >= 1 */
    uint32_t checkpoint_every; /* checkpoint interval s >= 1; 0 = round(sqrt(K)) */
    const uint64_t *marked;    /* host, m distinct indices < 2^n (any order); NULL when m = 0 */
    uint64_t m;
    uint32_t dtype;            /* GROVER_C64 (other types: GROVER_E_UNSUPPORTED) */
    uint32_t flags;            /* must be 0 */
} grover_phase_config;

/* grover_phase_init — validate cfg (GROVER_E_INVAL before any device work), allocate the states, adjoint
 * states and checkpoints, and confirm the persistent grid on the device.  All work goes to hip_stream
 * (NULL = default stream).  Synchronous. */
int grover_phase_init(grover_phase **out, const grover_phase_config *cfg, void *hip_stream);

/* grover_phase_set_team — workgroups per schedule in the streamed form (1 .. grid size; default: grid / B,
 * at most the number of 64 KiB tiles of one state).  Changes the order of additions in the sums, not the
 * results' meaning. */
int grover_phase_set_team(grover_phase *p, uint32_t team);

/* grover_phase_set_form — how the states are kept while they iterate:
 *   GROVER_PHASE_FORM_STREAMED: in memory, read and written by every iteration (any size);
 *   GROVER_PHASE_FORM_HELD: on chip (registers and LDS) for all K iterations, by teams of a power of two of
 *     workgroups sized from the state (forward: 16 16-byte vectors per thread; adjoint: 8 of the state and
 *     8 of the adjoint state); memory holds only the checkpoints and the final state.  Needs both teams to
 *     fit the grid (n <= 22 on a grid of 256): GROVER_E_UNSUPPORTED otherwise;
 *   GROVER_PHASE_FORM_AUTO (default): held when it fits, else streamed.
 * Both forms keep the same checkpoints and final state, so a backward run may use either form whatever the
 * forward run used.  The forms add in different orders, so their results agree to rounding.
 * GROVER_E_INVAL for another value. */
#define GROVER_PHASE_FORM_AUTO 0
#define GROVER_PHASE_FORM_STREAMED 1
#define GROVER_PHASE_FORM_HELD 2
int grover_phase_set_form(grover_phase *p, uint32_t form);

/* grover_phase_forward — run all B schedules.  phi, theta: device, binary64 [B][K] row-major (copied on
 * the stream before the run, so the caller may reuse them afterwards); loss: device, binary64 [B], written.
 * Leaves each schedule's final state in the context (grover_phase_state) with its checkpoints.
 * Asynchronous. */
int grover_phase_forward(grover_phase *p, const double *phi, const double *theta, double *loss);

/* grover_phase_backward — the gradient of sum_b dloss[b] * L_b at the phases of the last forward run:
 * dloss: device binary64 [B]; dphi, dtheta: device binary64 [B][K], written.  Needs a forward run since
 * the last backward (GROVER_E_INVAL otherwise): the sweep overwrites the states, which afterwards hold the
 * uniform superposition.  Asynchronous. */
int grover_phase_backward(grover_phase *p, const double *dloss, double *dphi, double *dtheta);

/* grover_phase_sync — wait for the stream; GROVER_E_TIMEOUT when a team barrier gave up. */
int grover_phase_sync(grover_phase *p);

/* grover_phase_state / grover_phase_read_state — device address and size (2^n * 8 bytes) of schedule
 * b's state; copy it to host memory (synchronises the stream; bytes must equal the size). */
int grover_phase_state(grover_phase *p, uint32_t b, void **dev_ptr, size_t *bytes);
int grover_phase_read_state(grover_phase *p, uint32_t b, void *host, size_t bytes);

/* grover_phase_query — key: 0 = B, 1 = persistent grid size, 2 = workgroups per schedule (streamed form),
 * 3 = checkpoint interval, 4 = stored checkpoints per schedule, 5 = device bytes held, 6 = the form the next
 * run uses (GROVER_PHASE_FORM_STREAMED or _HELD), 7 / 8 = workgroups per schedule of the held form's
 * forward / adjoint run (0 when the states do not fit on chip). */
int grover_phase_query(grover_phase *p, int key, int64_t *value);

/* grover_phase_destroy — wait for the stream and release everything (NULL is ignored);
 * grover_phase_last_error — the last failure message (a static message when p is NULL). */
void grover_phase_destroy(grover_phase *p);
const char *grover_phase_last_error(const grover_phase *p);

#ifdef __cplusplus
}
#endif

#endif /* GROVER_H */
