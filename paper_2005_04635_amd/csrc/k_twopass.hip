// Plain form of the proposed iteration, kept as the comparator: the paper's steps as separate kernels
// launched from the host each iteration,
//   1. the oracle (Algorithm 3): negate the m marked amplitudes in place,
//   2. the first loop of Algorithm 4: per-block sums of the state, then one block adds them in block order,
//   3. the second loop of Algorithm 4: c_i <- 2S/N - c_i over the whole state.
// Per iteration it reads the state twice and writes it once (48 bytes per complex128 amplitude), against
// one read and one write for the fused form.  Also hosts the oracle-flip kernel of the gate-level path.
#include "internal.h"

namespace grover {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxBlocks = 2048;

template <class T>
__device__ inline void negate_elem(void *state, uint64_t i)
{
    if (T::kComplex && T::EPV == 2) {  // complex64: one float2 per amplitude
        float2 *s = static_cast<float2 *>(state);
        float2 x = s[i];
        s[i] = make_float2(-x.x, -x.y);
    } else if (T::kComplex) {  // complex128
        double2 *s = static_cast<double2 *>(state);
        double2 x = s[i];
        s[i] = make_double2(-x.x, -x.y);
    } else {
        double *s = static_cast<double *>(state);
        s[i] = -s[i];
    }
}

template <class T>
__global__ void oracle_flip_kernel(void *state, const uint64_t *marks, uint64_t m)
{
    for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < m; j += uint64_t(gridDim.x) * blockDim.x)
        negate_elem<T>(state, marks[j]);
}

// Per-block sums of the (already flipped) state; block b covers a fixed grid-stride set of vectors.
template <class T>
__global__ __launch_bounds__(kBlock) void block_sum_kernel(const void *state, uint64_t nvec, double *partials)
{
    __shared__ double red[2 * (kBlock / kWave)];
    const typename T::vec *st = static_cast<const typename T::vec *>(state);
    AccF64 acc;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t v = uint64_t(blockIdx.x) * kBlock + threadIdx.x; v < nvec; v += stride)
        accum_vec<T>(st[v], 0u, acc);
    double ar = acc.r, ai = acc.i;
    block_sum2(ar, ai, red);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = ar;
        partials[2 * blockIdx.x + 1] = ai;
    }
}

// One block adds the per-block sums in block order.
__global__ __launch_bounds__(kBlock) void finalize_sum_kernel(const double *partials, int nblocks, double *out)
{
    __shared__ double red[2 * (kBlock / kWave)];
    double ar = 0.0, ai = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock) {
        ar += partials[2 * b];
        ai += partials[2 * b + 1];
    }
    block_sum2(ar, ai, red);
    if (threadIdx.x == 0) {
        out[0] = ar;
        out[1] = ai;
    }
}

// c_i <- 2S/N - c_i (the flip already happened in place).
template <class T>
__global__ __launch_bounds__(kBlock) void mean_update_kernel(void *state, uint64_t nvec, double N, const double *sum)
{
    typename T::vec *st = static_cast<typename T::vec *>(state);
    const double mr = (sum[0] * 2.0) / N, mi = (sum[1] * 2.0) / N;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    AccF64 unused;  // the sum is taken by the next iteration's own pass
    for (uint64_t v = uint64_t(blockIdx.x) * kBlock + threadIdx.x; v < nvec; v += stride) {
        typename T::vec x = st[v];
        update_vec<T>(x, mr, mi, 0u, unused);
        st[v] = x;
    }
}

struct Kernels {
    const void *flip, *bsum, *update;
};

template <class T>
Kernels kernels_of()
{
    return {reinterpret_cast<const void *>(&oracle_flip_kernel<T>),
            reinterpret_cast<const void *>(&block_sum_kernel<T>),
            reinterpret_cast<const void *>(&mean_update_kernel<T>)};
}

Kernels kernels_for(uint32_t dtype)
{
    switch (dtype) {
    case GROVER_F64_REAL: return kernels_of<F64Real>();
    case GROVER_C64: return kernels_of<C64>();
    default: return kernels_of<C128>();
    }
}

}  // namespace

int twopass_blocks(const grover_ctx *c)
{
    const uint64_t nvec = c->N / elems_per_vec(c->dtype);
    const uint64_t want = (nvec + kBlock - 1) / kBlock;
    return int(want < uint64_t(kMaxBlocks) ? want : uint64_t(kMaxBlocks));
}

hipError_t launch_oracle_flip(grover_ctx *c)
{
    const uint64_t m = c->marks.size();
    if (m == 0)
        return hipSuccess;
    const Kernels k = kernels_for(c->dtype);
    const uint64_t blocks = (m + kBlock - 1) / kBlock;
    void *state = c->state;
    const uint64_t *marks = c->marks_dev;
    uint64_t mm = m;
    void *args[] = {&state, &marks, &mm};
    return hipLaunchKernel(k.flip, dim3(unsigned(blocks < 65535 ? blocks : 65535)), dim3(kBlock), args, 0,
                           c->stream);
}

hipError_t launch_twopass_iterate(grover_ctx *c, uint64_t iters)
{
    const Kernels k = kernels_for(c->dtype);
    void *state = c->state;
    uint64_t nvec = c->N / elems_per_vec(c->dtype);
    double N = double(c->N);
    const int nb = twopass_blocks(c);
    double *partials = c->red_partials;
    double *sum = c->red_out;
    int nbv = nb;
    for (uint64_t it = 0; it < iters; ++it) {
        hipError_t e = launch_oracle_flip(c);
        if (e != hipSuccess)
            return e;
        const void *state_c = state;
        void *a1[] = {&state_c, &nvec, &partials};
        e = hipLaunchKernel(k.bsum, dim3(nb), dim3(kBlock), a1, 0, c->stream);
        if (e != hipSuccess)
            return e;
        const double *partials_c = partials;
        void *a2[] = {&partials_c, &nbv, &sum};
        e = hipLaunchKernel(reinterpret_cast<const void *>(&finalize_sum_kernel), dim3(1), dim3(kBlock), a2, 0,
                            c->stream);
        if (e != hipSuccess)
            return e;
        const double *sum_c = sum;
        void *a3[] = {&state, &nvec, &N, &sum_c};
        e = hipLaunchKernel(k.update, dim3(nb), dim3(kBlock), a3, 0, c->stream);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace grover
