// Gate-level comparison path (Background: Algorithms 1 and 2).
//   - one Hadamard pass on qubit q: for every pair (i0, i1 = i0 | 2^q) with bit q of i0 clear,
//     (a, b) -> (h a + h b, h a - h b), h = 1/sqrt(2) — Eq. 1 with U = H, in place per pair;
//   - H^n as n such passes;
//   - the conditional phase shift 2|0><0| - I: every amplitude except index 0 is negated.
// Each pass reads and writes the whole state, so one conventional iteration costs 2n + 1 passes plus the
// oracle flip, against a single pass for the fused proposed iteration.
#include "internal.h"

namespace grover {
namespace {

constexpr int kBlock = 256;
constexpr double kInvSqrt2 = 0.70710678118654752440084436210484903928483593768847;

template <class T>
struct Elem;
template <>
struct Elem<C64> {
    using type = float2;
    __device__ static inline void butterfly(type &a, type &b)
    {
        const double ar = a.x, ai = a.y, br = b.x, bi = b.y;
        a = make_float2(float(kInvSqrt2 * ar + kInvSqrt2 * br), float(kInvSqrt2 * ai + kInvSqrt2 * bi));
        b = make_float2(float(kInvSqrt2 * ar - kInvSqrt2 * br), float(kInvSqrt2 * ai - kInvSqrt2 * bi));
    }
    __device__ static inline type neg(type a) { return make_float2(-a.x, -a.y); }
};
template <>
struct Elem<C128> {
    using type = double2;
    __device__ static inline void butterfly(type &a, type &b)
    {
        const double ar = a.x, ai = a.y, br = b.x, bi = b.y;
        a = make_double2(kInvSqrt2 * ar + kInvSqrt2 * br, kInvSqrt2 * ai + kInvSqrt2 * bi);
        b = make_double2(kInvSqrt2 * ar - kInvSqrt2 * br, kInvSqrt2 * ai - kInvSqrt2 * bi);
    }
    __device__ static inline type neg(type a) { return make_double2(-a.x, -a.y); }
};
template <>
struct Elem<F64Real> {
    using type = double;
    __device__ static inline void butterfly(type &a, type &b)
    {
        const double x = a, y = b;
        a = kInvSqrt2 * x + kInvSqrt2 * y;
        b = kInvSqrt2 * x - kInvSqrt2 * y;
    }
    __device__ static inline type neg(type a) { return -a; }
};

template <class T>
__global__ __launch_bounds__(kBlock) void hadamard_pass_kernel(void *state, uint64_t half, uint32_t q)
{
    using E = typename Elem<T>::type;
    E *st = static_cast<E *>(state);
    const uint64_t low = (uint64_t(1) << q) - 1u;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t j = uint64_t(blockIdx.x) * kBlock + threadIdx.x; j < half; j += stride) {
        const uint64_t i0 = ((j & ~low) << 1) | (j & low);
        const uint64_t i1 = i0 | (uint64_t(1) << q);
        E a = st[i0], b = st[i1];
        Elem<T>::butterfly(a, b);
        st[i0] = a;
        st[i1] = b;
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void phase_shift_kernel(void *state, uint64_t N)
{
    using E = typename Elem<T>::type;
    E *st = static_cast<E *>(state);
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += stride)
        if (i != 0)
            st[i] = Elem<T>::neg(st[i]);
}

unsigned grid_for(uint64_t work, int cu_count)
{
    const uint64_t want = (work + kBlock - 1) / kBlock;
    const uint64_t cap = uint64_t(cu_count > 0 ? cu_count : 256) * 16;
    return unsigned(want < cap ? (want > 0 ? want : 1) : cap);
}

template <class T>
hipError_t hadamard_all(grover_ctx *c)
{
    void *state = c->state;
    uint64_t half = c->N / 2;
    const unsigned grid = grid_for(half, c->cu_count);
    for (uint32_t q = 0; q < c->n; ++q) {
        uint32_t qq = q;
        void *args[] = {&state, &half, &qq};
        const hipError_t e = hipLaunchKernel(reinterpret_cast<const void *>(&hadamard_pass_kernel<T>), dim3(grid),
                                             dim3(kBlock), args, 0, c->stream);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <class T>
hipError_t phase_shift(grover_ctx *c)
{
    void *state = c->state;
    uint64_t N = c->N;
    void *args[] = {&state, &N};
    return hipLaunchKernel(reinterpret_cast<const void *>(&phase_shift_kernel<T>), dim3(grid_for(N, c->cu_count)),
                           dim3(kBlock), args, 0, c->stream);
}

}  // namespace

hipError_t launch_hadamard_all(grover_ctx *c)
{
    switch (c->dtype) {
    case GROVER_F64_REAL: return hadamard_all<F64Real>(c);
    case GROVER_C64: return hadamard_all<C64>(c);
    case GROVER_C128: return hadamard_all<C128>(c);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_conditional_phase_shift(grover_ctx *c)
{
    switch (c->dtype) {
    case GROVER_F64_REAL: return phase_shift<F64Real>(c);
    case GROVER_C64: return phase_shift<C64>(c);
    case GROVER_C128: return phase_shift<C128>(c);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace grover
