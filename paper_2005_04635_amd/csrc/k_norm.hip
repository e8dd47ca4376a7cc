// Squared norm sum_i |c_i|^2 in binary64 (Background, "Quantum State": it equals 1 for every state the
// iteration produces).  Per-block partials over a fixed grid-stride mapping, then one block adds them in
// block order, so the value is reproducible.
#include "internal.h"

namespace grover {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxBlocks = 2048;

template <class T>
__global__ __launch_bounds__(kBlock) void norm_partials_kernel(const void *state, uint64_t nvec, double *partials)
{
    __shared__ double red[2 * (kBlock / kWave)];
    const typename T::vec *st = static_cast<const typename T::vec *>(state);
    double acc = 0.0, unused = 0.0;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t v = uint64_t(blockIdx.x) * kBlock + threadIdx.x; v < nvec; v += stride) {
        const typename T::vec x = st[v];
#pragma unroll
        for (int e = 0; e < T::EPV; ++e) {
            const double r = T::re(x, e), i = T::im(x, e);
            acc += __dadd_rn(__dmul_rn(r, r), __dmul_rn(i, i));
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
    const uint64_t want = (nvec + kBlock - 1) / kBlock;
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
