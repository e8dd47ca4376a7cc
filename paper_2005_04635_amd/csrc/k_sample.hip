// Measurement (Background, step 6).  The paper plots outcome probabilities but gives no sampling procedure;
// this library samples by inverse transform over an integer CDF so that the result is a function of the
// state's bits alone:
//   p_i = re^2 + im^2 (binary64, no fused multiply-add), q_i = floor(p_i 2^62), Q_i = q_0 + ... + q_i,
//   t_j = floor(U_j Q_{N-1} / 2^53), shot j -> the smallest i with Q_i > t_j.
// Integer addition is associative, so the three-phase device scan (block totals, scan of the totals,
// per-block scan) yields exactly the sequential prefix sums; each shot is then a binary search.
//
// A CDF block covers kPerBlock = 4096 amplitudes, read by a workgroup of B threads as 4096 / EPV 16-byte
// vectors in R = 4096 / EPV / B coalesced rows (thread t reads vector u * B + t of row u), so every load
// instruction moves one contiguous row and each thread has R loads in flight.  The amplitudes of row u
// precede those of row u + 1, and within a row thread t's come before thread t + 1's, so the block's prefix
// sums are, row by row, an exclusive scan over the threads of each thread's row sum: a wave scan by lane
// shuffles, then one exchange of the wave totals through LDS.  The block totals use 256-thread workgroups
// that take CDF blocks b, b + G, ... (G = gridDim.x, a few per CU); the prefix sums one 1024-thread
// workgroup per CDF block (at n = 28 complex64: 0.77 ms against 0.81 ms for the strided 256-thread form,
// where the totals took 0.33 against 0.40 ms in one 1024-thread workgroup each).
#include "internal.h"

namespace grover {
namespace {

constexpr int kTotalBlock = 256;  // block totals: 256-thread workgroups striding over the CDF blocks
constexpr int kCdfBlock = 1024;   // prefix sums: one 1024-thread workgroup per CDF block (measured faster)
constexpr int kScanBlock = 256;   // scan of the block totals: one workgroup
constexpr uint64_t kPerBlock = 4096;  // amplitudes per CDF block

template <class T, int B>
constexpr int rows_of()
{
    return int(kPerBlock) / T::EPV / B;
}

__device__ inline uint64_t qval(double r, double m)
{
    const double p = __dadd_rn(__dmul_rn(r, r), __dmul_rn(m, m));
    return (uint64_t)__dmul_rn(p, 0x1p62);
}

// q of amplitude e of a storage vector
template <class T>
__device__ inline uint64_t qval_of(const typename T::vec &x, int e)
{
    return qval(T::re(x, e), T::im(x, e));
}

// Inclusive scan of one uint64 per lane across the wave, by lane shuffles (six steps).
__device__ inline uint64_t wave_inclusive_scan(uint64_t x)
{
    const unsigned lane = threadIdx.x % kWave;
#pragma unroll
    for (unsigned off = 1; off < kWave; off <<= 1) {
        const uint64_t y = __shfl_up(x, off, kWave);
        if (lane >= off)
            x += y;
    }
    return x;
}

// The R rows of CDF block b for workgroups of B threads: vector u * B + t of the block for thread t
// (nontemporal loads).
template <class T, int B>
__device__ inline void load_rows(const typename T::vec *st, uint64_t nvec, uint64_t b,
                                 typename T::vec (&x)[rows_of<T, B>()])
{
    const uint64_t v0 = b * (kPerBlock / T::EPV);
#pragma unroll
    for (int u = 0; u < rows_of<T, B>(); ++u) {
        const uint64_t v = v0 + uint64_t(u) * B + threadIdx.x;
        if (v < nvec)
            x[u] = load16<true>(st + v);
    }
}

template <class T>
__global__ __launch_bounds__(kTotalBlock) void q_block_total_kernel(const void *state, uint64_t nvec, uint64_t nb,
                                                                    uint64_t *block_sums)
{
    using V = typename T::vec;
    constexpr int kBlock = kTotalBlock, kWaves = kBlock / kWave;
    constexpr int R = rows_of<T, kBlock>();
    // wave values, alternating between two sets by iteration: a set is written again two iterations later,
    // after the next iteration's barrier, which thread 0 passes only after reading it here
    __shared__ uint64_t wt[2][kWaves];
    const V *st = static_cast<const V *>(state);
    unsigned it = 0;
    for (uint64_t b = blockIdx.x; b < nb; b += gridDim.x, ++it) {
        V x[R];
        load_rows<T, kBlock>(st, nvec, b, x);
        const uint64_t v0 = b * (kPerBlock / T::EPV);
        uint64_t acc = 0;
#pragma unroll
        for (int u = 0; u < R; ++u)
            if (v0 + uint64_t(u) * kBlock + threadIdx.x < nvec)
#pragma unroll
                for (int e = 0; e < T::EPV; ++e)
                    acc += qval_of<T>(x[u], e);
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1)
            acc += __shfl_xor(acc, off, kWave);
        if (threadIdx.x % kWave == 0)
            wt[it & 1u][threadIdx.x / kWave] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t sum = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w)
                sum += wt[it & 1u][w];
            block_sums[b] = sum;
        }
    }
}

// Single workgroup: block_sums[b] <- sum of block_sums[0 .. b-1].  Thread t owns a contiguous run of
// entries; the run sums are scanned across the workgroup, then each thread rewrites its run from its
// exclusive offset.
__global__ __launch_bounds__(kScanBlock) void scan_block_totals_kernel(uint64_t *block_sums, uint64_t nb)
{
    constexpr int kBlock = kScanBlock, kWaves = kBlock / kWave;
    __shared__ uint64_t wt[kWaves];
    const unsigned lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const uint64_t per = (nb + kBlock - 1) / kBlock;
    const uint64_t lo = uint64_t(threadIdx.x) * per;
    const uint64_t hi = lo + per < nb ? lo + per : nb;
    uint64_t acc = 0;
    for (uint64_t j = lo; j < hi; ++j)
        acc += block_sums[j];
    const uint64_t incl = wave_inclusive_scan(acc);
    if (lane == kWave - 1)
        wt[wave] = incl;
    __syncthreads();
    uint64_t run = incl - acc;
    for (unsigned w = 0; w < wave; ++w)
        run += wt[w];
    for (uint64_t j = lo; j < hi; ++j) {
        const uint64_t x = block_sums[j];
        block_sums[j] = run;
        run += x;
    }
}

// Stores the EPV prefix values of one vector: contiguous uint64 entries, 16 bytes at a time.
template <int EPV>
__device__ inline void store_prefix(uint64_t *cdf, uint64_t i, const uint64_t (&q)[EPV])
{
    if constexpr (EPV == 1) {
        __builtin_nontemporal_store(q[0], cdf + i);
    } else {
        typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int e = 0; e < EPV; e += 2) {
            u64x2 w;
            w.x = q[e];
            w.y = q[e + 1];
            __builtin_nontemporal_store(w, reinterpret_cast<u64x2 *>(cdf + i + e));
        }
    }
}

// Exclusive scan of one uint64 per thread over a workgroup of B threads (thread order), with the workgroup
// total.  `wt` holds B / 64 words; the caller alternates two sets between calls, so a call's writes never
// meet the previous call's reads (each call has one barrier, which every thread passes only after its reads
// of the call before).
template <int B>
__device__ inline uint64_t block_exclusive_scan(uint64_t v, uint64_t *wt, uint64_t &total)
{
    const unsigned lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const uint64_t incl = wave_inclusive_scan(v);
    if (lane == kWave - 1)
        wt[wave] = incl;
    __syncthreads();
    uint64_t before = 0, all = 0;
#pragma unroll
    for (unsigned w = 0; w < unsigned(B / kWave); ++w) {
        const uint64_t t = wt[w];
        before += w < wave ? t : 0u;
        all += t;
    }
    total = all;
    return before + incl - v;
}

// One workgroup per CDF block; the rows are scanned and stored one after another, so that a row's stores
// leave while the next row is being scanned.  (Scanning all rows with a single barrier and storing them
// afterwards took 0.95 instead of 0.77 ms at n = 28 complex64.)
template <class T>
__global__ __launch_bounds__(kCdfBlock) void cdf_kernel(const void *state, uint64_t nvec, const uint64_t *block_offsets,
                                                        uint64_t *cdf)
{
    using V = typename T::vec;
    constexpr int kBlock = kCdfBlock, kWaves = kBlock / kWave;
    constexpr int R = rows_of<T, kBlock>();
    __shared__ uint64_t wt[2][kWaves];
    const V *st = static_cast<const V *>(state);
    const uint64_t b = blockIdx.x;
    V x[R];
    load_rows<T, kBlock>(st, nvec, b, x);
    uint64_t base = block_offsets[b];
    const uint64_t v0 = b * (kPerBlock / T::EPV);
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const uint64_t v = v0 + uint64_t(u) * kBlock + threadIdx.x;
        const bool in = v < nvec;
        uint64_t q[T::EPV];
        uint64_t row = 0;
#pragma unroll
        for (int e = 0; e < T::EPV; ++e) {
            q[e] = in ? qval_of<T>(x[u], e) : 0u;
            row += q[e];
        }
        uint64_t total;
        uint64_t pre = base + block_exclusive_scan<kBlock>(row, wt[u & 1], total);
#pragma unroll
        for (int e = 0; e < T::EPV; ++e) {
            pre += q[e];
            q[e] = pre;
        }
        if (in)
            store_prefix<T::EPV>(cdf, v * T::EPV, q);
        base += total;
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

template <class T>
Kernels kernels_of()
{
    return {reinterpret_cast<const void *>(&q_block_total_kernel<T>), reinterpret_cast<const void *>(&cdf_kernel<T>)};
}

Kernels kernels_for(uint32_t dtype)
{
    switch (dtype) {
    case GROVER_F64_REAL: return kernels_of<F64Real>();
    case GROVER_C64: return kernels_of<C64>();
    case GROVER_CBF16: return kernels_of<CBF16>();
    default: return kernels_of<C128>();
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
    uint64_t nvec = N / elems_per_vec(c->dtype);
    uint64_t nb = sample_block_count(N);
    uint64_t *bs = c->block_sums;
    uint64_t *cdf = c->cdf;
    // block totals: a few workgroups per CU, each striding over the CDF blocks
    const uint64_t cap = uint64_t(c->cu_count > 0 ? c->cu_count : 256) * 8u;
    const unsigned grid = unsigned(nb < cap ? nb : cap);
    void *a1[] = {&state, &nvec, &nb, &bs};
    hipError_t e = hipLaunchKernel(k.total, dim3(grid), dim3(kTotalBlock), a1, 0, c->stream);
    if (e != hipSuccess)
        return e;
    void *a2[] = {&bs, &nb};
    e = hipLaunchKernel(reinterpret_cast<const void *>(&scan_block_totals_kernel), dim3(1), dim3(kScanBlock), a2, 0,
                        c->stream);
    if (e != hipSuccess)
        return e;
    const uint64_t *bsc = bs;
    void *a3[] = {&state, &nvec, &bsc, &cdf};
    e = hipLaunchKernel(k.cdf, dim3(unsigned(nb)), dim3(kCdfBlock), a3, 0, c->stream);
    if (e != hipSuccess)
        return e;
    if (shots == 0)
        return hipSuccess;
    const uint64_t *cdfc = cdf;
    int on_dev = device_uniforms ? 1 : 0;
    uint32_t *err = c->flag_dev;
    const uint64_t want = (shots + 255) / 256;
    const unsigned sgrid = unsigned(want < 65535 ? want : 65535);
    void *a4[] = {&cdfc, &N, &u53_dev, &seed, &on_dev, &shots, &out_dev, &err};
    return hipLaunchKernel(reinterpret_cast<const void *>(&search_kernel), dim3(sgrid), dim3(256), a4, 0,
                           c->stream);
}

}  // namespace grover
