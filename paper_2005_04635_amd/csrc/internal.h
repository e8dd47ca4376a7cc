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

// ----------------------------------------------------------------------------------- storage traits
// Every kernel streams the state in 16-byte vectors.  A vector holds EPV amplitudes:
//   F64 real: double2 = 2 amplitudes; C64: float4 = 2 amplitudes (re, im, re, im); C128: double2 = 1.
struct F64Real {
    using vec = double2;
    static constexpr int EPV = 2;
    static constexpr int kBytes = 8;
    static constexpr bool kComplex = false;
    __device__ static inline double re(const vec &v, int e) { return e == 0 ? v.x : v.y; }
    __device__ static inline double im(const vec &, int) { return 0.0; }
};
struct C64 {
    using vec = float4;
    static constexpr int EPV = 2;
    static constexpr int kBytes = 8;
    static constexpr bool kComplex = true;
    __device__ static inline double re(const vec &v, int e) { return e == 0 ? double(v.x) : double(v.z); }
    __device__ static inline double im(const vec &v, int e) { return e == 0 ? double(v.y) : double(v.w); }
};
struct C128 {
    using vec = double2;
    static constexpr int EPV = 1;
    static constexpr int kBytes = 16;
    static constexpr bool kComplex = true;
    __device__ static inline double re(const vec &v, int) { return v.x; }
    __device__ static inline double im(const vec &v, int) { return v.y; }
};

inline size_t elem_bytes(uint32_t dtype) { return dtype == GROVER_C128 ? 16 : 8; }

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

// ------------------------------------------------------------------------------ update of one vector
// Inversion about the mean on the oracle-flipped amplitudes: c' = 2S/N - s*c with s = -1 for marked
// amplitudes (bit e of `marked`), +1 otherwise.  (mr, mi) = 2S/N in binary64.  The value that is stored
// (rounded to the element type) is also added, times s, to (ar, ai): that is the next iteration's sum.
template <class T>
__device__ inline void update_vec(typename T::vec &v, double mr, double mi, unsigned marked, double &ar,
                                  double &ai);

template <>
__device__ inline void update_vec<C64>(float4 &v, double mr, double mi, unsigned marked, double &ar,
                                       double &ai)
{
    const double s0 = (marked & 1u) ? -1.0 : 1.0, s1 = (marked & 2u) ? -1.0 : 1.0;
    const float r0 = float(mr - s0 * double(v.x)), i0 = float(mi - s0 * double(v.y));
    const float r1 = float(mr - s1 * double(v.z)), i1 = float(mi - s1 * double(v.w));
    v = make_float4(r0, i0, r1, i1);
    ar += s0 * double(r0);
    ai += s0 * double(i0);
    ar += s1 * double(r1);
    ai += s1 * double(i1);
}

template <>
__device__ inline void update_vec<F64Real>(double2 &v, double mr, double, unsigned marked, double &ar,
                                           double &)
{
    const double s0 = (marked & 1u) ? -1.0 : 1.0, s1 = (marked & 2u) ? -1.0 : 1.0;
    const double r0 = mr - s0 * v.x, r1 = mr - s1 * v.y;
    v = make_double2(r0, r1);
    ar += s0 * r0;
    ar += s1 * r1;
}

template <>
__device__ inline void update_vec<C128>(double2 &v, double mr, double mi, unsigned marked, double &ar,
                                        double &ai)
{
    const double s0 = (marked & 1u) ? -1.0 : 1.0;
    const double r0 = mr - s0 * v.x, i0 = mi - s0 * v.y;
    v = make_double2(r0, i0);
    ar += s0 * r0;
    ai += s0 * i0;
}

// Sum of s*c over one vector, in exactly the order update_vec accumulates (so a fresh sum of a stored
// state equals, bit for bit, the sum the fused update produced while writing it).
template <class T>
__device__ inline void accum_vec(const typename T::vec &v, unsigned marked, double &ar, double &ai)
{
#pragma unroll
    for (int e = 0; e < T::EPV; ++e) {
        const double s = (marked >> e) & 1u ? -1.0 : 1.0;
        ar += s * T::re(v, e);
        if (T::kComplex)
            ai += s * T::im(v, e);
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

// Wavefront sum of a double; the butterfly order is fixed, so the result is reproducible.
__device__ inline double wave_sum(double x)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        x += __shfl_xor(x, off, kWave);
    return x;
}

// Workgroup sum of (a, b): wave butterflies, then wave 0 adds the per-wave values in wave order.
// `red` must hold 2 * (blockDim / 64) doubles.  Result valid in thread 0 only.
__device__ inline void block_sum2(double &a, double &b, double *red)
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
        double sa = 0.0, sb = 0.0;
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
    double *partials = nullptr;  // 2 * grid * 2 doubles
    grover::GridSync *sync = nullptr;
    const void *fused_kernel = nullptr;        // the fused kernel variant chosen at creation
    const void *fused_check_kernel = nullptr;  // its code-identical twin for the residency check
    uint64_t fused_tile = 0;             // 16-byte vectors per tile of that variant
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
// `check`: launch the code-identical instantiation reserved for the residency check.
hipError_t launch_fused_iterate(grover_ctx *c, uint64_t k, uint64_t timeout_ticks, bool check = false);

hipError_t launch_resident_iterate(grover_ctx *c, uint64_t k);

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
