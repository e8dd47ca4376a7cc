// Internal declarations of libgrover: storage traits, device helpers, the context and the launchers that
// each kernel translation unit exports to the API layer.  Not installed; the public ABI is grover.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "grover.h"

namespace grover {

// ------------------------------------------------------------------------------------------ constants
constexpr int kWave = 64;                 // CDNA wavefront width
constexpr uint32_t kMaxQubits = 34;       // 2^34 complex64 = 128 GiB, half of one MI355X's HBM
constexpr uint32_t kResidentMaxQubits = 14;  // on-chip path: 2^14 amplitudes in one workgroup
constexpr int kResidentBlock = 1024;
constexpr uint64_t kHashMarkCap = uint64_t(1) << 26;  // largest hash-defined marked list kept

// ------------------------------------------------------------------------------------ bfloat16 helpers
// bfloat16 = the top 16 bits of an IEEE binary32.  Rounding from binary64 is done once, correctly: round
// to odd into binary32 (toward zero, then set the last bit when inexact), then round to nearest even into
// bfloat16 — the intermediate has 16 more bits than the target, so no double rounding can occur.  The
// rounding toward zero comes from the hardware's conversion to nearest: when that was inexact and moved
// away from zero, the binary32 one step toward zero (its bit pattern minus one, as the magnitude bits are
// contiguous; from infinity this gives the largest finite value) is the truncation.  About nine
// instructions where the library's round-toward-zero conversion takes some twenty-five.
__device__ __host__ inline float bf16_to_float(uint16_t b)
{
    const uint32_t u = uint32_t(b) << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

__device__ inline uint16_t double_to_bf16(double d)
{
    const float t = float(d);  // nearest
    uint32_t u = __float_as_uint(t);
    const double dt = double(t);
    if (dt != d) {
        if (__builtin_fabs(dt) > __builtin_fabs(d))
            u -= 1u;  // t rounded away from zero: step back to the truncation
        u |= 1u;      // round to odd
    }
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

// ----------------------------------------------------------------------------------- storage traits
// Every kernel streams the state in 16-byte vectors.  A vector holds EPV amplitudes:
//   F64 real: double2 = 2 amplitudes; C64: float4 = 2 amplitudes (re, im, re, im); C128: double2 = 1;
//   CBF16: 8 bfloat16 = 4 amplitudes (re, im, ...).
// re/im read amplitude e as binary64; set writes amplitude e, rounded to the storage type.
struct F64Real {
    using vec = double2;
    static constexpr int EPV = 2;
    static constexpr int kBytes = 8;
    static constexpr bool kComplex = false;
    __device__ static inline double re(const vec &v, int e) { return e == 0 ? v.x : v.y; }
    __device__ static inline double im(const vec &, int) { return 0.0; }
    __device__ static inline void set(vec &v, int e, double r, double)
    {
        if (e == 0)
            v.x = r;
        else
            v.y = r;
    }
};
struct C64 {
    using vec = float4;
    static constexpr int EPV = 2;
    static constexpr int kBytes = 8;
    static constexpr bool kComplex = true;
    __device__ static inline double re(const vec &v, int e) { return e == 0 ? double(v.x) : double(v.z); }
    __device__ static inline double im(const vec &v, int e) { return e == 0 ? double(v.y) : double(v.w); }
    __device__ static inline void set(vec &v, int e, double r, double i)
    {
        if (e == 0) {
            v.x = float(r);
            v.y = float(i);
        } else {
            v.z = float(r);
            v.w = float(i);
        }
    }
};
struct C128 {
    using vec = double2;
    static constexpr int EPV = 1;
    static constexpr int kBytes = 16;
    static constexpr bool kComplex = true;
    __device__ static inline double re(const vec &v, int) { return v.x; }
    __device__ static inline double im(const vec &v, int) { return v.y; }
    __device__ static inline void set(vec &v, int, double r, double i)
    {
        v.x = r;
        v.y = i;
    }
};
struct bf16x8 {
    uint16_t h[8];
};
struct CBF16 {
    using vec = bf16x8;
    static constexpr int EPV = 4;
    static constexpr int kBytes = 4;
    static constexpr bool kComplex = true;
    __device__ static inline double re(const vec &v, int e) { return double(bf16_to_float(v.h[2 * e])); }
    __device__ static inline double im(const vec &v, int e) { return double(bf16_to_float(v.h[2 * e + 1])); }
    __device__ static inline void set(vec &v, int e, double r, double i)
    {
        v.h[2 * e] = double_to_bf16(r);
        v.h[2 * e + 1] = double_to_bf16(i);
    }
};

inline size_t elem_bytes(uint32_t dtype)
{
    return dtype == GROVER_C128 ? 16 : dtype == GROVER_CBF16 ? 4 : 8;
}
inline uint64_t elems_per_vec(uint32_t dtype)
{
    return dtype == GROVER_C128 ? 1 : dtype == GROVER_CBF16 ? 4 : 2;
}

// 16-byte loads and stores of a storage vector; the nontemporal forms mark the lines as streaming so they
// do not displace reused data from the caches.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool NT, class V>
__device__ inline V load16(const V *p)
{
    static_assert(sizeof(V) == 16, "storage vectors are 16 bytes");
    if (NT) {
        const u32x4 r = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
        V v;
        __builtin_memcpy(&v, &r, 16);
        return v;
    }
    return *p;
}

template <bool NT, class V>
__device__ inline void store16(const V &v, V *p)
{
    if (NT) {
        u32x4 r;
        __builtin_memcpy(&r, &v, 16);
        __builtin_nontemporal_store(r, reinterpret_cast<u32x4 *>(p));
    } else {
        *p = v;
    }
}

// 16-byte accesses through a buffer resource: the descriptor holds the base address of a block of vectors
// (a tile) and its byte count, each lane a 32-bit byte offset, so no 64-bit address arithmetic is spent per
// vector, and the cache policy travels as instruction bits (gfx950: 1 = sc0, 2 = nt, 16 = sc1).  A load at
// or beyond the byte count returns zero and a store there writes nothing.  On MI355X an in-place
// nontemporal stream of 2 GiB (512 threads of 8 vectors per 64 KiB tile, one launch per pass) ran at 6.21
// TB/s through buffer instructions against 5.89 TB/s through global ones with the same bits, and at
// 6.26 TB/s with nt sc1 stores.
constexpr int kBufPlain = 0;
constexpr int kBufNT = 2;             // nt: streaming
constexpr int kBufNTDevice = 2 | 16;  // nt sc1: streaming, written through at device scope

__device__ inline __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, uint32_t bytes)
{
    // stride 0 (raw byte offsets); word 3 = 0x00020000, the gfx9-family raw 32-bit data format
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, int(bytes), 0x00020000);
}

template <int AUX, class V>
__device__ inline V bload16(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    static_assert(sizeof(V) == 16, "storage vectors are 16 bytes");
    const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, AUX);
    V v;
    __builtin_memcpy(&v, &x, 16);
    return v;
}

template <int AUX, class V>
__device__ inline void bstore16(const V &v, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    static_assert(sizeof(V) == 16, "storage vectors are 16 bytes");
    u32x4 x;
    __builtin_memcpy(&x, &v, 16);
    __builtin_amdgcn_raw_buffer_store_b128(x, r, off, 0, AUX);
}

// ---------------------------------------------------------------------------------------- accumulators
// Per-thread accumulation of the sum S = sum_i s_i c_i.  add() takes binary64 values of stored amplitudes.
//   AccF64:       binary64 sums (the library's default; the tree above it is binary64 too)
//   AccF32:       plain binary32 sums (tree in binary32)
//   AccF32Kahan:  binary32 sums with Kahan's compensation (tree in binary32)
struct AccF64 {
    using value = double;
    double r = 0.0, i = 0.0;
    __device__ inline void add(double x, double y)
    {
        r += x;
        i += y;
    }
    __device__ inline double res_r() const { return r; }
    __device__ inline double res_i() const { return i; }
};
struct AccF32 {
    using value = float;
    float r = 0.0f, i = 0.0f;
    __device__ inline void add(double x, double y)
    {
        r += float(x);
        i += float(y);
    }
    __device__ inline float res_r() const { return r; }
    __device__ inline float res_i() const { return i; }
};
struct AccF32Kahan {
    using value = float;
    float r = 0.0f, i = 0.0f, cr = 0.0f, ci = 0.0f;  // running sums and their compensations
    __device__ static inline void kahan(float &s, float &c, float x)
    {
        const float y = x - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ inline void add(double x, double y)
    {
        kahan(r, cr, float(x));
        kahan(i, ci, float(y));
    }
    __device__ inline float res_r() const { return r - cr; }
    __device__ inline float res_i() const { return i - ci; }
};

// ------------------------------------------------------------------------------ update of one vector
// Inversion about the mean on the oracle-flipped amplitudes: c' = 2S/N - s*c with s = -1 for marked
// amplitudes (bit e of `marked`), +1 otherwise, computed in binary64 from (mr, mi) = 2S/N and rounded to
// the storage type.  The stored value, times s, is added to the accumulator: that is the next iteration's
// sum.
template <class T, class A>
__device__ inline void update_vec(typename T::vec &v, double mr, double mi, unsigned marked, A &acc)
{
#pragma unroll
    for (int e = 0; e < T::EPV; ++e) {
        const double s = (marked >> e) & 1u ? -1.0 : 1.0;
        T::set(v, e, mr - s * T::re(v, e), mi - s * T::im(v, e));
        acc.add(s * T::re(v, e), s * T::im(v, e));
    }
}

// The same update computed in binary32, for complex64 storage: (mr, mi) = 2S/N already rounded to
// binary32, and each part of c' = mr - s c is one binary32 operation (mr + c for a marked amplitude, the same
// rounding as mr - (-c)).  The stored values, times s, are added to the binary64 accumulator in the order of
// update_vec and accum_vec.
template <class A>
__device__ inline void update_vec_f32(float4 &v, float mr, float mi, unsigned marked, A &acc)
{
    const bool m0 = (marked & 1u) != 0u, m1 = (marked & 2u) != 0u;
    v.x = m0 ? mr + v.x : mr - v.x;
    v.y = m0 ? mi + v.y : mi - v.y;
    v.z = m1 ? mr + v.z : mr - v.z;
    v.w = m1 ? mi + v.w : mi - v.w;
    acc.add(m0 ? -double(v.x) : double(v.x), m0 ? -double(v.y) : double(v.y));
    acc.add(m1 ? -double(v.z) : double(v.z), m1 ? -double(v.w) : double(v.w));
}

// Sum of s*c over one vector, in exactly the order update_vec accumulates (so a fresh sum of a stored
// state equals, bit for bit, the sum the fused update produced while writing it).
template <class T, class A>
__device__ inline void accum_vec(const typename T::vec &v, unsigned marked, A &acc)
{
#pragma unroll
    for (int e = 0; e < T::EPV; ++e) {
        const double s = (marked >> e) & 1u ? -1.0 : 1.0;
        acc.add(s * T::re(v, e), s * T::im(v, e));
    }
}

// --------------------------------------------------------------------------------- device helpers
// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator: output j for `seed`.
__device__ __host__ inline uint64_t splitmix64(uint64_t seed, uint64_t j)
{
    uint64_t z = seed + (j + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// First position in sorted a[lo, hi) whose value is >= x.
__device__ __host__ inline uint64_t lower_bound_u64(const uint64_t *a, uint64_t lo, uint64_t hi, uint64_t x)
{
    while (lo < hi) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Marked bits of the EPV amplitudes starting at element i, against sorted marks[lo, hi).
template <int EPV>
__device__ inline unsigned marked_bits(const uint64_t *marks, uint64_t lo, uint64_t hi, uint64_t i)
{
    unsigned bits = 0;
    uint64_t p = lower_bound_u64(marks, lo, hi, i);
#pragma unroll
    for (int e = 0; e < EPV; ++e) {
        if (p < hi && marks[p] == i + uint64_t(e)) {
            bits |= 1u << e;
            ++p;
        }
    }
    return bits;
}

// Wavefront sum; the butterfly order is fixed and addition is commutative, so every lane ends with the same,
// reproducible value.
template <class V>
__device__ inline V wave_sum(V x)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        x += __shfl_xor(x, off, kWave);
    return x;
}

// Sum over the 64 lanes of a wave, the same bits returned in every lane, without a trip through the LDS
// crossbar: four DPP row shifts (each lane adds the value 1, 2, 4, 8 lanes below it in its row of 16, zero
// past the row's start) leave each row's sum in its last lane; the four row sums are read into scalar
// registers and added as (r0 + r1) + (r2 + r3).  A fixed order, so the result is reproducible.
template <int kCtrl>
__device__ inline double dpp_row_shifted(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, int(b), kCtrl, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), kCtrl, 0xf, 0xf, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

__device__ inline double lane_value(double x, int lane)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane(int(b), lane);
    const int hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

__device__ inline double wave_total(double x)
{
    x += dpp_row_shifted<0x111>(x);  // row_shr:1
    x += dpp_row_shifted<0x112>(x);  // row_shr:2
    x += dpp_row_shifted<0x114>(x);  // row_shr:4
    x += dpp_row_shifted<0x118>(x);  // row_shr:8
    return (lane_value(x, 15) + lane_value(x, 31)) + (lane_value(x, 47) + lane_value(x, 63));
}

__device__ inline float wave_total(float x) { return wave_sum(x); }

// Workgroup sum of (a, b): wave butterflies, then thread 0 adds the per-wave values in wave order.
// `red` must hold 2 * (blockDim / 64) values.  Result valid in thread 0 only.
template <class V>
__device__ inline void block_sum2(V &a, V &b, V *red)
{
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) {
        red[2 * wave] = a;
        red[2 * wave + 1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        V sa = V(0), sb = V(0);
        for (int w = 0; w < nw; ++w) {
            sa += red[2 * w];
            sb += red[2 * w + 1];
        }
        a = sa;
        b = sb;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------- grid barrier state
// One per context, zeroed at creation.  `flag` is a monotonically increasing barrier generation that
// waiting workgroups poll; arrive0/arrive1 count workgroups at a barrier of parity 0/1; sum[p] is that
// barrier's reduced value; `error` is set when a wait gives up.  Polled and atomically updated words sit
// on separate 256-byte lines so that polling does not contend with arrivals.
struct GridSync {
    uint64_t flag;
    uint32_t error;
    uint32_t pad0[61];
    uint32_t arrive0;
    uint32_t pad1[63];
    uint32_t arrive1;
    uint32_t pad2[63];
    uint64_t sum[2][2];  // bit patterns of (re, im) binary64
    uint64_t pad3[28];
};
static_assert(sizeof(GridSync) == 1024, "barrier words on separate lines");

// ------------------------------------------------------------------------------------------ context
}  // namespace grover

struct grover_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t n = 0;
    uint64_t N = 0;
    uint32_t dtype = 0;
    uint32_t accum = 0;
    uint32_t update = 0;  // grover_update: precision of the element update
    uint32_t form = 0;  // resolved (never AUTO)
    uint32_t kind = 0;
    void *state = nullptr;
    size_t state_bytes = 0;
    bool owns_state = false;
    std::vector<uint64_t> marks;  // sorted
    uint64_t *marks_dev = nullptr;
    // fused form
    int grid = 0;
    int block = 0;
    uint64_t *partials = nullptr;  // fused barrier: slots [2][grid][4] and the published sum [2][4]
    int64_t partials_grid = 0;     // the largest grid those slots were allocated for
    int per_cu_reported = 0;       // workgroups per CU of the fused kernel according to the runtime
    grover::GridSync *sync = nullptr;
    const void *fused_kernel = nullptr;        // the fused kernel variant chosen at creation
    const void *fused_check_kernel = nullptr;  // its code-identical twin for the residency check
    uint64_t fused_tile = 0;             // 16-byte vectors per tile of that variant
    uint64_t fused_temporal_bytes = 0;   // bytes per pass streamed with ordinary (not nontemporal) accesses
    uint32_t held_team = 0;              // held form: workgroups holding the state (one launch of that many)
    uint64_t generation = 0;
    uint64_t timeout_ticks = 0;
    // two-pass form and reductions
    double *red_partials = nullptr;  // per-block (re, im)
    int red_blocks = 0;
    double *red_out = nullptr;        // 2 doubles
    double *host_pinned = nullptr;    // 2 doubles, pinned
    // sampler
    uint64_t *cdf = nullptr;
    uint64_t *block_sums = nullptr;
    size_t block_sums_cap = 0;
    uint64_t *shots_buf = nullptr;
    size_t shots_cap = 0;
    uint64_t *u53_buf = nullptr;
    size_t u53_cap = 0;
    uint32_t *flag_dev = nullptr;  // generic device error word for the sampler
    int cu_count = 0;
    std::string last_error;
};

namespace grover {

// ------------------------------------------------------------------------ launchers (one per TU)
// Each returns hipSuccess or the failing HIP error; the API layer maps errors to status codes.
hipError_t launch_fill_uniform(grover_ctx *c);
hipError_t launch_hash_marks(grover_ctx *c, uint64_t seed, uint32_t bits, uint64_t *out, uint64_t cap,
                             unsigned long long *count);

// Occupancy of the fused kernel per CU as the runtime reports it, its workgroup size, and a grid forced by
// GROVER_FUSED_GRID (0 when unset).
hipError_t fused_configure(grover_ctx *c, int *per_cu, int *block, int64_t *forced_grid);
uint64_t fused_tiles(const grover_ctx *c);
// Leading unmarked tiles of each workgroup's share that the fused kernel streams with ordinary accesses.
uint64_t fused_temporal_tiles(const grover_ctx *c);
// `check`: launch the code-identical instantiation reserved for the residency check.
hipError_t launch_fused_iterate(grover_ctx *c, uint64_t k, uint64_t timeout_ticks, bool check = false);
// Tiles of the fused kernel over a state of N amplitudes of the given type.
uint64_t fused_tiles_of(uint32_t dtype, uint64_t N);
// The fused kernel (binary64 sums, the default access split) on barrier memory the caller provides:
// slots [2][grid][4] + [2][4] tagged words and a GridSync, all zero, generations from 1.
struct FusedExternal {
    void *state;
    uint32_t dtype;
    uint64_t N;
    const uint64_t *marks;
    uint64_t m;
    uint64_t k;
    int grid;
    uint64_t *slots;
    GridSync *sync;
    uint64_t timeout_ticks;
    hipStream_t stream;
};
hipError_t launch_fused_external(const FusedExternal &x);
// The message the last failing grover_init or grover_iterate_static left on the calling thread.
void set_thread_error(const std::string &msg);

hipError_t launch_resident_iterate(grover_ctx *c, uint64_t k);

// Held form (complex64, binary64 sums): workgroups that hold a state of nvec vectors, 0 when it does not fit
// a team of at most max_team (a power of two); and the launch (`probe`: one team barrier only).
uint32_t held_team_size(uint64_t nvec, uint32_t max_team);
hipError_t launch_held_iterate(grover_ctx *c, uint64_t k, uint64_t timeout_ticks, bool probe = false);

hipError_t launch_twopass_iterate(grover_ctx *c, uint64_t k);
int twopass_blocks(const grover_ctx *c);

hipError_t launch_norm(grover_ctx *c, double *dev_out);

hipError_t launch_sample(grover_ctx *c, const uint64_t *u53_dev, uint64_t seed, bool device_uniforms,
                         uint64_t shots, uint64_t *out_dev);
size_t sample_block_count(uint64_t N);

hipError_t launch_oracle_flip(grover_ctx *c);
hipError_t launch_hadamard_all(grover_ctx *c);
hipError_t launch_conditional_phase_shift(grover_ctx *c);

}  // namespace grover
