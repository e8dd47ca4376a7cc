// Squared norm sum_i |c_i|^2 in binary64 (Background, "Quantum State": it equals 1 for every state the
// iteration produces).  Per-block partials over a fixed mapping of chunks to blocks, then one block adds them
// in block order, so the value is reproducible.
#include "internal.h"

namespace grover {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxBlocks = 2048;

constexpr int kUnroll = 4;  // 16-byte vectors in flight per thread

// Block b reads chunks of kBlock * kUnroll vectors, b, b + G, ... (G = gridDim.x); in a chunk, thread t reads
// vectors u * kBlock + t (one coalesced row per u), nontemporal: the state is not reused from the caches.
template <class T>
__global__ __launch_bounds__(kBlock) void norm_partials_kernel(const void *state, uint64_t nvec, double *partials)
{
    using V = typename T::vec;
    __shared__ double red[2 * (kBlock / kWave)];
    const V *st = static_cast<const V *>(state);
    double acc = 0.0, unused = 0.0;
    const uint64_t chunk = uint64_t(kBlock) * kUnroll;
    for (uint64_t c0 = uint64_t(blockIdx.x) * chunk; c0 < nvec; c0 += uint64_t(gridDim.x) * chunk) {
        V x[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t v = c0 + uint64_t(u) * kBlock + threadIdx.x;
            if (v < nvec)
                x[u] = load16<true>(st + v);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (c0 + uint64_t(u) * kBlock + threadIdx.x < nvec)
#pragma unroll
                for (int e = 0; e < T::EPV; ++e) {
                    const double r = T::re(x[u], e), i = T::im(x[u], e);
                    acc += __dadd_rn(__dmul_rn(r, r), __dmul_rn(i, i));
                }
        }
    }
    block_sum2(acc, unused, red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kBlock) void norm_finalize_kernel(const double *partials, int nblocks, double *out)
{
    __shared__ double red[2 * (kBlock / kWave)];
    double acc = 0.0, unused = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock)
        acc += partials[b];
    block_sum2(acc, unused, red);
    if (threadIdx.x == 0)
        out[0] = acc;
}

}  // namespace

hipError_t launch_norm(grover_ctx *c, double *dev_out)
{
    uint64_t nvec = c->N / elems_per_vec(c->dtype);
    const uint64_t want = (nvec + uint64_t(kBlock) * kUnroll - 1) / (uint64_t(kBlock) * kUnroll);
    int nb = int(want < uint64_t(kMaxBlocks) ? want : uint64_t(kMaxBlocks));
    const void *state = c->state;
    double *partials = c->red_partials;  // sized for kMaxBlocks * 2 doubles by the API layer
    const void *fn = nullptr;
    switch (c->dtype) {
    case GROVER_F64_REAL: fn = reinterpret_cast<const void *>(&norm_partials_kernel<F64Real>); break;
    case GROVER_C64: fn = reinterpret_cast<const void *>(&norm_partials_kernel<C64>); break;
    case GROVER_C128: fn = reinterpret_cast<const void *>(&norm_partials_kernel<C128>); break;
    case GROVER_CBF16: fn = reinterpret_cast<const void *>(&norm_partials_kernel<CBF16>); break;
    default: return hipErrorInvalidValue;
    }
    void *a1[] = {&state, &nvec, &partials};
    hipError_t e = hipLaunchKernel(fn, dim3(nb), dim3(kBlock), a1, 0, c->stream);
    if (e != hipSuccess)
        return e;
    const double *pc = partials;
    void *a2[] = {&pc, &nb, &dev_out};
    return hipLaunchKernel(reinterpret_cast<const void *>(&norm_finalize_kernel), dim3(1), dim3(kBlock), a2, 0,
                           c->stream);
}

}  // namespace grover
