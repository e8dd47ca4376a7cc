// Blocked Walsh-Hadamard transform for the gate-level comparison path (H^n of Algorithms 1 and 2).
//
// H^n factorises over qubits, and any set of qubits can be transformed together once their amplitudes are
// in one workgroup's LDS.  So instead of n passes over the state (one per qubit, Algorithm 1 literally), the
// transform takes ceil((n - L) / H) + 1 passes:
//   - a low pass: each workgroup loads 2^L contiguous amplitudes and applies the butterflies of qubits
//     0 .. L-1;
//   - high passes over qubits q0 .. q0+H-1: each workgroup loads a tile of 2^H rows (stride 2^q0) by C
//     contiguous columns (C amplitudes = one 128-byte or 256-byte segment per row, so loads coalesce) and
//     applies the butterflies along the rows.
// Butterflies are unnormalised, (a, b) -> (a + b, a - b), in binary64 in LDS, three stages per register
// round; the storage type is rounded once per pass.  The normalisation is one multiplication in the last
// pass: 2^(-n/2) for H^n alone (exact for even n), and for the conventional iteration H^n (2|0><0| - I) H^n
// the two transforms together need 2^(-n), an exact power of two, applied in the last pass of the second
// transform; the conditional phase shift (negate every amplitude but index 0) is applied in the last pass
// of the first.  At n = 28 with complex storage this is 3 passes per H^n instead of 28.
#include <cmath>

#include "wht.h"

namespace grover {
namespace {

constexpr int kWhtBlock = 512;
constexpr int kWhtCols = 16;           // columns of a high-pass tile
constexpr uint32_t kNegExceptZero = 1;  // store flags
constexpr uint32_t kScale = 2;

// Storage <-> binary64 value held in LDS.
template <class T>
struct Wht;
template <>
struct Wht<C64> {
    using E = float2;
    using V = double2;
    static constexpr int kLowQ = 12;   // 2^12 x 16 B = 64 KiB of LDS (+ 1/8 padding)
    static constexpr int kHighQ = 8;   // 2^8 rows x 16 columns x 16 B = 64 KiB
    __device__ static V in(E x) { return make_double2(x.x, x.y); }
    __device__ static E out(V x) { return make_float2(float(x.x), float(x.y)); }
};
template <>
struct Wht<C128> {
    using E = double2;
    using V = double2;
    static constexpr int kLowQ = 12;
    static constexpr int kHighQ = 8;
    __device__ static V in(E x) { return x; }
    __device__ static E out(V x) { return x; }
};
template <>
struct Wht<F64Real> {
    using E = double;
    using V = double;
    static constexpr int kLowQ = 13;  // 2^13 x 8 B = 64 KiB (+ 1/8 padding)
    static constexpr int kHighQ = 9;  // 2^9 x 16 x 8 B = 64 KiB
    __device__ static V in(E x) { return x; }
    __device__ static E out(V x) { return x; }
};

__device__ inline double2 vadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 vsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double vadd(double a, double b) { return a + b; }
__device__ inline double vsub(double a, double b) { return a - b; }
__device__ inline double2 vscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ inline double vscale(double a, double s) { return a * s; }
__device__ inline double2 vneg(double2 a) { return make_double2(-a.x, -a.y); }
__device__ inline double vneg(double a) { return -a; }

template <class V>
__device__ inline V finish(V v, uint64_t global_index, uint32_t flags, double scale)
{
    if (flags & kScale)
        v = vscale(v, scale);
    if ((flags & kNegExceptZero) && global_index != 0)
        v = vneg(v);
    return v;
}

// The block a workgroup transforms is a [rows][cols] array whose element (row, col) is amplitude
// base + row * 2^rowshift + col of the state, kept in LDS at buf[row * cols + col].  A single column (the
// low pass) is padded by one element every eight: the register rounds read eight rows 2^s apart per thread,
// and without the padding the lanes of a wavefront fall on half the LDS banks.  Rows of 16 columns (the
// high passes) already spread a wavefront over all banks.
template <class T>
struct Block {
    typename Wht<T>::E *st;
    typename Wht<T>::V *buf;
    uint64_t base;
    uint32_t rowshift;
    uint32_t rows;
    uint32_t cols;
    __device__ uint64_t global(uint32_t row, uint32_t col) const { return base + (uint64_t(row) << rowshift) + col; }
    __device__ uint32_t lds(uint32_t row, uint32_t col) const { return cols == 1 ? row + (row >> 3) : row * cols + col; }
};

// One round of R = 2^LR butterfly stages s .. s+LR-1 along the rows: each thread takes groups of R rows
// spaced 2^s apart (one column) and transforms them in registers.  The first round reads the state itself
// and the last one writes it (applying the store flags), so a pass touches LDS only between rounds.
template <class T, int LR, bool FIRST, bool LAST>
__device__ inline void wht_round(const Block<T> &B, uint32_t s, uint32_t flags, double scale)
{
    using W = Wht<T>;
    using V = typename W::V;
    constexpr int R = 1 << LR;
    const uint32_t h = 1u << s;
    const uint32_t groups = (B.rows >> LR) * B.cols;
    for (uint32_t g = threadIdx.x; g < groups; g += blockDim.x) {
        const uint32_t col = g % B.cols, rg = g / B.cols;
        const uint32_t row0 = ((rg >> s) << (s + LR)) | (rg & (h - 1u));
        V x[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const uint32_t row = row0 + uint32_t(k) * h;
            x[k] = FIRST ? W::in(B.st[B.global(row, col)]) : B.buf[B.lds(row, col)];
        }
#pragma unroll
        for (int t = 0; t < LR; ++t) {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                if (k & (1 << t))
                    continue;
                const V a = x[k], b = x[k | (1 << t)];
                x[k] = vadd(a, b);
                x[k | (1 << t)] = vsub(a, b);
            }
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const uint32_t row = row0 + uint32_t(k) * h;
            if (LAST) {
                const uint64_t gi = B.global(row, col);
                B.st[gi] = W::out(finish(x[k], gi, flags, scale));
            } else {
                B.buf[B.lds(row, col)] = x[k];
            }
        }
    }
    if (!LAST)
        __syncthreads();
}

template <class T, int LR>
__device__ inline void wht_round_at(const Block<T> &B, uint32_t s, bool first, bool last, uint32_t flags, double scale)
{
    if (first && last)
        wht_round<T, LR, true, true>(B, s, flags, scale);
    else if (first)
        wht_round<T, LR, true, false>(B, s, flags, scale);
    else if (last)
        wht_round<T, LR, false, true>(B, s, flags, scale);
    else
        wht_round<T, LR, false, false>(B, s, flags, scale);
}

// All q = log2(rows) stages along the rows, three at a time (the last round takes the remainder).
template <class T>
__device__ inline void wht_rows(const Block<T> &B, uint32_t q, uint32_t flags, double scale)
{
    uint32_t s = 0;
    while (s < q) {
        const uint32_t lr = q - s < 3u ? q - s : 3u;
        const bool first = s == 0, last = s + lr == q;
        if (lr == 3)
            wht_round_at<T, 3>(B, s, first, last, flags, scale);
        else if (lr == 2)
            wht_round_at<T, 2>(B, s, first, last, flags, scale);
        else
            wht_round_at<T, 1>(B, s, first, last, flags, scale);
        s += lr;
    }
}

// Low pass: qubits 0 .. L-1 of the block of 2^L amplitudes starting at blockIdx.x * 2^L.
template <class T>
__global__ __launch_bounds__(kWhtBlock) void wht_low_kernel(void *state, uint32_t L, uint32_t flags, double scale)
{
    using W = Wht<T>;
    __shared__ typename W::V buf[(1u << W::kLowQ) + (1u << W::kLowQ) / 8];
    const Block<T> B{static_cast<typename W::E *>(state), buf, uint64_t(blockIdx.x) << L, 0u, 1u << L, 1u};
    wht_rows<T>(B, L, flags, scale);
}

// High pass: qubits q0 .. q0+H-1.  Tile t covers the 2^H rows index = hi * 2^(q0+H) + row * 2^q0 + lo,
// lo in [c0, c0 + kWhtCols), with c0 = (t mod 2^q0 / kWhtCols) * kWhtCols and hi = t div (2^q0 / kWhtCols).
template <class T>
__global__ __launch_bounds__(kWhtBlock) void wht_high_kernel(void *state, uint32_t q0, uint32_t H, uint32_t flags,
                                                            double scale)
{
    using W = Wht<T>;
    __shared__ typename W::V buf[(1u << W::kHighQ) * kWhtCols];
    const uint64_t chunks = (uint64_t(1) << q0) / kWhtCols;
    const uint64_t t = blockIdx.x;
    const uint64_t base = ((t / chunks) << (q0 + H)) | ((t % chunks) * kWhtCols);
    const Block<T> B{static_cast<typename W::E *>(state), buf, base, q0, 1u << H, uint32_t(kWhtCols)};
    wht_rows<T>(B, H, flags, scale);
}

// The unnormalised transform of all n qubits, with `flags` / `scale` applied by its last pass.
template <class T>
hipError_t wht(grover_ctx *c, uint32_t flags, double scale)
{
    using W = Wht<T>;
    void *state = c->state;
    const uint32_t n = c->n;
    const uint32_t L = n < uint32_t(W::kLowQ) ? n : uint32_t(W::kLowQ);
    {
        uint32_t l = L, f = (L == n) ? flags : 0u;
        double sc = scale;
        void *args[] = {&state, &l, &f, &sc};
        const hipError_t e = hipLaunchKernel(reinterpret_cast<const void *>(&wht_low_kernel<T>),
                                             dim3(unsigned(c->N >> L)), dim3(kWhtBlock), args, 0, c->stream);
        if (e != hipSuccess)
            return e;
    }
    for (uint32_t q0 = L; q0 < n; q0 += uint32_t(W::kHighQ)) {
        uint32_t q = q0, h = n - q0 < uint32_t(W::kHighQ) ? n - q0 : uint32_t(W::kHighQ);
        uint32_t f = (q0 + h == n) ? flags : 0u;
        double sc = scale;
        void *args[] = {&state, &q, &h, &f, &sc};
        const uint64_t tiles = c->N >> h >> 4;  // 2^(n - h) / kWhtCols
        const hipError_t e = hipLaunchKernel(reinterpret_cast<const void *>(&wht_high_kernel<T>), dim3(unsigned(tiles)),
                                             dim3(kWhtBlock), args, 0, c->stream);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <class T>
hipError_t hadamard_all_blocked(grover_ctx *c)
{
    // 2^(-n/2): exact for even n; for odd n 2^(-(n+1)/2) * sqrt(2) rounded once to binary64
    const int n = int(c->n);
    const double s = (n % 2 == 0) ? std::ldexp(1.0, -n / 2) : std::ldexp(std::sqrt(2.0), -(n + 1) / 2);
    return wht<T>(c, kScale, s);
}

template <class T>
hipError_t diffusion_blocked(grover_ctx *c)
{
    hipError_t e = wht<T>(c, kNegExceptZero, 1.0);
    if (e != hipSuccess)
        return e;
    return wht<T>(c, kScale, std::ldexp(1.0, -int(c->n)));
}

}  // namespace

hipError_t launch_hadamard_all_blocked(grover_ctx *c)
{
    switch (c->dtype) {
    case GROVER_F64_REAL: return hadamard_all_blocked<F64Real>(c);
    case GROVER_C64: return hadamard_all_blocked<C64>(c);
    case GROVER_C128: return hadamard_all_blocked<C128>(c);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gate_diffusion_blocked(grover_ctx *c)
{
    switch (c->dtype) {
    case GROVER_F64_REAL: return diffusion_blocked<F64Real>(c);
    case GROVER_C64: return diffusion_blocked<C64>(c);
    case GROVER_C128: return diffusion_blocked<C128>(c);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace grover
