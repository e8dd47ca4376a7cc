// Measurement (Background, step 6).  The paper plots outcome probabilities but gives no sampling procedure;
// this library samples by inverse transform over an integer CDF so that the result is a function of the
// state's bits alone:
//   p_i = re^2 + im^2 (binary64, no fused multiply-add), q_i = floor(p_i 2^62), Q_i = q_0 + ... + q_i,
//   t_j = floor(U_j Q_{N-1} / 2^53), shot j -> the smallest i with Q_i > t_j.
// Integer addition is associative, so the three-phase device scan (block totals, scan of the totals,
// per-block scan) yields exactly the sequential prefix sums; each shot is then a binary search.
#include "internal.h"

namespace grover {
namespace {

constexpr int kBlock = 1024;
constexpr int kPerThread = 4;
constexpr uint64_t kPerBlock = uint64_t(kBlock) * kPerThread;  // amplitudes per CDF block

template <class T>
__device__ inline uint64_t qval(const void *state, uint64_t i);

template <>
__device__ inline uint64_t qval<C64>(const void *state, uint64_t i)
{
    const float2 c = static_cast<const float2 *>(state)[i];
    const double r = c.x, m = c.y;
    const double p = __dadd_rn(__dmul_rn(r, r), __dmul_rn(m, m));
    return (uint64_t)__dmul_rn(p, 0x1p62);
}
template <>
__device__ inline uint64_t qval<C128>(const void *state, uint64_t i)
{
    const double2 c = static_cast<const double2 *>(state)[i];
    const double p = __dadd_rn(__dmul_rn(c.x, c.x), __dmul_rn(c.y, c.y));
    return (uint64_t)__dmul_rn(p, 0x1p62);
}
template <>
__device__ inline uint64_t qval<CBF16>(const void *state, uint64_t i)
{
    const uint16_t *h = static_cast<const uint16_t *>(state) + 2 * i;
    const double r = bf16_to_float(h[0]), m = bf16_to_float(h[1]);
    const double p = __dadd_rn(__dmul_rn(r, r), __dmul_rn(m, m));
    return (uint64_t)__dmul_rn(p, 0x1p62);
}
template <>
__device__ inline uint64_t qval<F64Real>(const void *state, uint64_t i)
{
    const double r = static_cast<const double *>(state)[i];
    const double p = __dadd_rn(__dmul_rn(r, r), 0.0);
    return (uint64_t)__dmul_rn(p, 0x1p62);
}

// Exclusive scan of one uint64 per thread across the block (Hillis-Steele in LDS); returns the exclusive
// prefix and leaves the block total in *total.
__device__ inline uint64_t block_exclusive_scan(uint64_t v, uint64_t *s, uint64_t *total)
{
    const unsigned t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (unsigned off = 1; off < kBlock; off <<= 1) {
        const uint64_t x = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += x;
        __syncthreads();
    }
    const uint64_t incl = s[t];
    *total = s[kBlock - 1];
    __syncthreads();
    return incl - v;
}

template <class T>
__global__ __launch_bounds__(kBlock) void q_block_total_kernel(const void *state, uint64_t N, uint64_t *block_sums)
{
    __shared__ uint64_t s[kBlock];
    const uint64_t base = uint64_t(blockIdx.x) * kPerBlock + uint64_t(threadIdx.x) * kPerThread;
    uint64_t acc = 0;
#pragma unroll
    for (int e = 0; e < kPerThread; ++e)
        if (base + e < N)
            acc += qval<T>(state, base + e);
    uint64_t total;
    block_exclusive_scan(acc, s, &total);
    if (threadIdx.x == 0)
        block_sums[blockIdx.x] = total;
}

// Single block: block_sums[b] <- sum of block_sums[0 .. b-1].
__global__ __launch_bounds__(kBlock) void scan_block_totals_kernel(uint64_t *block_sums, uint64_t nb)
{
    __shared__ uint64_t s[kBlock];
    const uint64_t per = (nb + kBlock - 1) / kBlock;
    const uint64_t lo = uint64_t(threadIdx.x) * per;
    const uint64_t hi = lo + per < nb ? lo + per : nb;
    uint64_t acc = 0;
    for (uint64_t j = lo; j < hi; ++j)
        acc += block_sums[j];
    uint64_t total;
    uint64_t run = block_exclusive_scan(acc, s, &total);
    for (uint64_t j = lo; j < hi; ++j) {
        const uint64_t x = block_sums[j];
        block_sums[j] = run;
        run += x;
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void cdf_kernel(const void *state, uint64_t N, const uint64_t *block_offsets,
                                                     uint64_t *cdf)
{
    __shared__ uint64_t s[kBlock];
    const uint64_t base = uint64_t(blockIdx.x) * kPerBlock + uint64_t(threadIdx.x) * kPerThread;
    uint64_t q[kPerThread];
    uint64_t acc = 0;
#pragma unroll
    for (int e = 0; e < kPerThread; ++e) {
        q[e] = base + e < N ? qval<T>(state, base + e) : 0u;
        acc += q[e];
    }
    uint64_t total;
    uint64_t run = block_offsets[blockIdx.x] + block_exclusive_scan(acc, s, &total);
#pragma unroll
    for (int e = 0; e < kPerThread; ++e) {
        run += q[e];
        if (base + e < N)
            cdf[base + e] = run;
    }
}

__global__ void search_kernel(const uint64_t *cdf, uint64_t N, const uint64_t *u53, uint64_t seed, int on_device,
                              uint64_t shots, uint64_t *out, uint32_t *err)
{
    const uint64_t total = cdf[N - 1];
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < shots; j += stride) {
        if (total == 0) {
            if (j == 0)
                *err = 1u;
            out[j] = 0;
            continue;
        }
        const uint64_t U = on_device ? (splitmix64(seed, j) >> 11) : (u53[j] & ((uint64_t(1) << 53) - 1u));
        const uint64_t hi = __umul64hi(U, total);
        const uint64_t lo = U * total;
        const uint64_t t = (hi << 11) | (lo >> 53);
        uint64_t a = 0, b = N - 1;
        while (a < b) {
            const uint64_t mid = a + ((b - a) >> 1);
            if (cdf[mid] > t)
                b = mid;
            else
                a = mid + 1;
        }
        out[j] = a;
    }
}

struct Kernels {
    const void *total, *cdf;
};

Kernels kernels_for(uint32_t dtype)
{
    switch (dtype) {
    case GROVER_F64_REAL:
        return {reinterpret_cast<const void *>(&q_block_total_kernel<F64Real>),
                reinterpret_cast<const void *>(&cdf_kernel<F64Real>)};
    case GROVER_C64:
        return {reinterpret_cast<const void *>(&q_block_total_kernel<C64>),
                reinterpret_cast<const void *>(&cdf_kernel<C64>)};
    case GROVER_CBF16:
        return {reinterpret_cast<const void *>(&q_block_total_kernel<CBF16>),
                reinterpret_cast<const void *>(&cdf_kernel<CBF16>)};
    default:
        return {reinterpret_cast<const void *>(&q_block_total_kernel<C128>),
                reinterpret_cast<const void *>(&cdf_kernel<C128>)};
    }
}

}  // namespace

size_t sample_block_count(uint64_t N) { return size_t((N + kPerBlock - 1) / kPerBlock); }

hipError_t launch_sample(grover_ctx *c, const uint64_t *u53_dev, uint64_t seed, bool device_uniforms,
                         uint64_t shots, uint64_t *out_dev)
{
    const Kernels k = kernels_for(c->dtype);
    const void *state = c->state;
    uint64_t N = c->N;
    uint64_t nb = sample_block_count(N);
    uint64_t *bs = c->block_sums;
    uint64_t *cdf = c->cdf;
    void *a1[] = {&state, &N, &bs};
    hipError_t e = hipLaunchKernel(k.total, dim3(unsigned(nb)), dim3(kBlock), a1, 0, c->stream);
    if (e != hipSuccess)
        return e;
    void *a2[] = {&bs, &nb};
    e = hipLaunchKernel(reinterpret_cast<const void *>(&scan_block_totals_kernel), dim3(1), dim3(kBlock), a2, 0,
                        c->stream);
    if (e != hipSuccess)
        return e;
    const uint64_t *bsc = bs;
    void *a3[] = {&state, &N, &bsc, &cdf};
    e = hipLaunchKernel(k.cdf, dim3(unsigned(nb)), dim3(kBlock), a3, 0, c->stream);
    if (e != hipSuccess)
        return e;
    if (shots == 0)
        return hipSuccess;
    const uint64_t *cdfc = cdf;
    int on_dev = device_uniforms ? 1 : 0;
    uint32_t *err = c->flag_dev;
    const uint64_t want = (shots + 255) / 256;
    const unsigned grid = unsigned(want < 65535 ? want : 65535);
    void *a4[] = {&cdfc, &N, &u53_dev, &seed, &on_dev, &shots, &out_dev, &err};
    return hipLaunchKernel(reinterpret_cast<const void *>(&search_kernel), dim3(grid), dim3(256), a4, 0,
                           c->stream);
}

}  // namespace grover
