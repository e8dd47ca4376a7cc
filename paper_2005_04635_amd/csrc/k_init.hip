// Initial state and marked set (Algorithm 5's preparation; Algorithm 3's solution list k[]).
//   - fill: psi = H^n|0> written directly as the uniform superposition, 2^(-n/2) in every amplitude;
//   - hash predicate: i is marked iff the low `bits` bits of SplitMix64_i(seed) are zero; every index is
//     tested on the device and the hits are compacted into a list (sorted afterwards by the host).
#include <cmath>
#include <cstring>

#include "internal.h"

namespace grover {
namespace {

constexpr int kBlock = 256;

constexpr int kFillBlock = 512;
constexpr int kFillUnroll = 8;  // 16-byte stores per thread per chunk

// Chunks of kFillBlock * kFillUnroll vectors (64 KiB), workgroup b taking chunks b, b + G, ... with one
// workgroup per CU; thread t writes vectors u * kFillBlock + t of a chunk (coalesced rows) with nontemporal
// 16-byte buffer stores through a buffer resource over the chunk (the next pass reads the state from HBM);
// full chunks without bounds checks.  (Two 1024-thread workgroups per CU with global stores wrote 2 GiB
// at 5.39 TB/s; four 256-thread ones at 5.0 TB/s.)
template <class T>
__global__ __launch_bounds__(kFillBlock) void fill_kernel(void *state, uint64_t nvec, typename T::vec value)
{
    using V = typename T::vec;
    constexpr uint64_t chunk = uint64_t(kFillBlock) * kFillUnroll;
    for (uint64_t c0 = uint64_t(blockIdx.x) * chunk; c0 < nvec; c0 += uint64_t(gridDim.x) * chunk) {
        const uint64_t n = nvec - c0 < chunk ? nvec - c0 : chunk;
        const auto rs = buffer_rsrc(static_cast<V *>(state) + c0, uint32_t(n * 16u));
        if (n == chunk) {
#pragma unroll
            for (int u = 0; u < kFillUnroll; ++u)
                bstore16<kBufNT>(value, rs, (uint32_t(u) * kFillBlock + threadIdx.x) * 16u);
        } else {
#pragma unroll
            for (int u = 0; u < kFillUnroll; ++u) {
                const uint32_t w = uint32_t(u) * kFillBlock + threadIdx.x;
                if (w < n)
                    bstore16<kBufNT>(value, rs, w * 16u);
            }
        }
    }
}

unsigned fill_grid(uint64_t nvec, int cu_count)
{
    const uint64_t chunks = (nvec + uint64_t(kFillBlock) * kFillUnroll - 1) / (uint64_t(kFillBlock) * kFillUnroll);
    const uint64_t cap = uint64_t(cu_count > 0 ? cu_count : 256);
    return unsigned(chunks < cap ? (chunks > 0 ? chunks : 1) : cap);
}

__global__ __launch_bounds__(kBlock) void hash_marks_kernel(uint64_t N, uint64_t seed, uint64_t mask,
                                                            uint64_t *out, uint64_t cap,
                                                            unsigned long long *count)
{
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < N; i += stride) {
        if ((splitmix64(seed, i) & mask) == 0) {
            const unsigned long long pos = atomicAdd(count, 1ull);
            if (pos < cap)
                out[pos] = i;
        }
    }
}

// Host twin of double_to_bf16 for the one constant the fill writes: one correct rounding to nearest even
// (round to odd into binary32, then to nearest even into bfloat16).
uint16_t host_double_to_bf16(double d)
{
    float t = float(d);  // nearest; step one ulp towards zero when that rounded away from zero
    if (std::fabs(double(t)) > std::fabs(d))
        t = std::nextafter(t, 0.0f);
    uint32_t u;
    std::memcpy(&u, &t, 4);
    if (double(t) != d)
        u |= 1u;
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

unsigned grid_for(uint64_t work, int cu_count)
{
    const uint64_t want = (work + kBlock - 1) / kBlock;
    const uint64_t cap = uint64_t(cu_count > 0 ? cu_count : 256) * 16;
    return unsigned(want < cap ? (want > 0 ? want : 1) : cap);
}

}  // namespace

hipError_t launch_fill_uniform(grover_ctx *c)
{
    // 2^(-n/2), correctly rounded: exact for even n; sqrt(2) * 2^(-(n+1)/2) for odd n.
    const double a = (c->n % 2 == 0) ? ldexp(1.0, -int(c->n / 2)) : ldexp(sqrt(2.0), -int((c->n + 1) / 2));
    void *state = c->state;
    switch (c->dtype) {
    case GROVER_F64_REAL: {
        uint64_t nvec = c->N / 2;
        double2 v = make_double2(a, a);
        void *args[] = {&state, &nvec, &v};
        return hipLaunchKernel(reinterpret_cast<const void *>(&fill_kernel<F64Real>),
                               dim3(fill_grid(nvec, c->cu_count)), dim3(kFillBlock), args, 0, c->stream);
    }
    case GROVER_C64: {
        uint64_t nvec = c->N / 2;
        const float af = float(a);
        float4 v = make_float4(af, 0.0f, af, 0.0f);
        void *args[] = {&state, &nvec, &v};
        return hipLaunchKernel(reinterpret_cast<const void *>(&fill_kernel<C64>),
                               dim3(fill_grid(nvec, c->cu_count)), dim3(kFillBlock), args, 0, c->stream);
    }
    case GROVER_C128: {
        uint64_t nvec = c->N;
        double2 v = make_double2(a, 0.0);
        void *args[] = {&state, &nvec, &v};
        return hipLaunchKernel(reinterpret_cast<const void *>(&fill_kernel<C128>),
                               dim3(fill_grid(nvec, c->cu_count)), dim3(kFillBlock), args, 0, c->stream);
    }
    case GROVER_CBF16: {
        uint64_t nvec = c->N / 4;
        bf16x8 v;
        const uint16_t ab = host_double_to_bf16(a);
        for (int e = 0; e < 4; ++e) {
            v.h[2 * e] = ab;
            v.h[2 * e + 1] = 0;
        }
        void *args[] = {&state, &nvec, &v};
        return hipLaunchKernel(reinterpret_cast<const void *>(&fill_kernel<CBF16>),
                               dim3(fill_grid(nvec, c->cu_count)), dim3(kFillBlock), args, 0, c->stream);
    }
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_hash_marks(grover_ctx *c, uint64_t seed, uint32_t bits, uint64_t *out, uint64_t cap,
                             unsigned long long *count)
{
    uint64_t N = c->N;
    uint64_t mask = bits >= 64 ? ~uint64_t(0) : ((uint64_t(1) << bits) - 1u);
    void *args[] = {&N, &seed, &mask, &out, &cap, &count};
    return hipLaunchKernel(reinterpret_cast<const void *>(&hash_marks_kernel), dim3(grid_for(N, c->cu_count)),
                           dim3(kBlock), args, 0, c->stream);
}

}  // namespace grover
