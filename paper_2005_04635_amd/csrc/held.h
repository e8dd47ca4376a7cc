// Device code for states held on chip by a team of workgroups for all iterations (the batched kernel's
// resident phases and the single-state held form): one iteration's update of a thread's held vectors and
// the handling of the marked amplitudes around it.  Thread tid of a member holds its vectors
// e * 1024 + tid, e < ne: the first kHeldRegE in registers (x[e]), the others in its own slots of LDS
// (held[(e - kHeldRegE) * 1024 + tid]; no other thread touches them, so they need no workgroup barrier).
// Marked bits travel packed, two per vector (bits 2e, 2e + 1 of `mask` for vector e).
#pragma once

#include "stream.h"

namespace grover {

constexpr int kHeldRegE = 8;                       // 16-byte vectors a thread holds in registers
constexpr int kHeldLdsE = 8;                       // ... and in its own slots of LDS (128 KiB per workgroup)
constexpr int kHeldHoldE = kHeldRegE + kHeldLdsE;  // 16 vectors = 32 complex64 amplitudes per thread

// Update of one held vector as if it held no marked amplitude (c' = 2S/N - c per amplitude, the stored
// values accumulated).  Marked amplitudes are handled around the sweep: their stored values are negated
// before it (exactly), which makes this update produce 2S/N + c, their correct new value bit for bit, and
// the sum is corrected after it by -2c' per marked amplitude (so it holds s c' for them, as the inversion
// about the mean needs).  Every thread thus runs the same short update, and the few threads with marks
// only add a few operations; the slowest wave sets the pace of every iteration.
__device__ inline void unmarked_update(float4 &v, double mr, double mi, AccF64 &acc)
{
    v.x = float(mr - double(v.x));
    v.y = float(mi - double(v.y));
    v.z = float(mr - double(v.z));
    v.w = float(mi - double(v.w));
    acc.add(double(v.x), double(v.y));
    acc.add(double(v.z), double(v.w));
}

// The same update in binary32 from 2S/N rounded to binary32 (mr, mi): one binary32 subtraction per part,
// where the binary64 form takes a conversion, a binary64 subtraction and a rounding conversion.  A negated
// marked value gives mr + c, the marked result of fl32(mr - s c), as above.
__device__ inline void unmarked_update(float4 &v, float mr, float mi, AccF64 &acc)
{
    v.x = mr - v.x;
    v.y = mi - v.y;
    v.z = mr - v.z;
    v.w = mi - v.w;
    acc.add(double(v.x), double(v.y));
    acc.add(double(v.z), double(v.w));
}

// Negates the stored values of the marked amplitudes among a thread's held vectors (bits 2e, 2e + 1 of
// `mask` for vector e).
__device__ inline void negate_marked(float4 (&x)[kHeldRegE], float4 *held, uint32_t mask)
{
#pragma unroll
    for (int e = 0; e < kHeldHoldE; ++e) {
        const unsigned b = (mask >> (2 * e)) & 3u;
        if (b != 0u) {
            float4 v = e < kHeldRegE ? x[e] : held[(e - kHeldRegE) * kStreamBlock + threadIdx.x];
            if (b & 1u) {
                v.x = -v.x;
                v.y = -v.y;
            }
            if (b & 2u) {
                v.z = -v.z;
                v.w = -v.w;
            }
            if (e < kHeldRegE)
                x[e] = v;
            else
                held[(e - kHeldRegE) * kStreamBlock + threadIdx.x] = v;
        }
    }
}

// After the sweep: the sum holds +c' for the marked amplitudes; subtracting 2c' makes it s c'.
__device__ inline void correct_marked(const float4 (&x)[kHeldRegE], const float4 *held, uint32_t mask, AccF64 &acc)
{
#pragma unroll
    for (int e = 0; e < kHeldHoldE; ++e) {
        const unsigned b = (mask >> (2 * e)) & 3u;
        if (b != 0u) {
            const float4 v = e < kHeldRegE ? x[e] : held[(e - kHeldRegE) * kStreamBlock + threadIdx.x];
            if (b & 1u)
                acc.add(-2.0 * double(v.x), -2.0 * double(v.y));
            if (b & 2u)
                acc.add(-2.0 * double(v.z), -2.0 * double(v.w));
        }
    }
}

// One iteration over a thread's held vectors (e < ne in order: x[e] in registers for e < kHeldRegE, then the
// LDS slots), each updated as unmarked.  When all 16 are held, the LDS vectors are loaded four at a time,
// each group while the previous one (or the register half) is being updated, so that their latency hides
// behind arithmetic.  M is the type of 2S/N: double for the binary64 update, float (already rounded) for
// the binary32 one.
template <class M>
__device__ inline void held_sweep(float4 (&x)[kHeldRegE], float4 *held, unsigned ne, M mr, M mi, AccF64 &acc)
{
    const unsigned tid = threadIdx.x;
    if (ne == unsigned(kHeldHoldE)) {
        constexpr int kG = 4;
        static_assert(2 * kG == kHeldLdsE, "two groups cover the LDS half");
        float4 y[kG], z[kG];
#pragma unroll
        for (int g = 0; g < kG; ++g)
            y[g] = held[g * kStreamBlock + tid];
#pragma unroll
        for (int e = 0; e < kHeldRegE; ++e)
            unmarked_update(x[e], mr, mi, acc);
#pragma unroll
        for (int g = 0; g < kG; ++g)
            z[g] = held[(kG + g) * kStreamBlock + tid];
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            unmarked_update(y[g], mr, mi, acc);
            held[g * kStreamBlock + tid] = y[g];
        }
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            unmarked_update(z[g], mr, mi, acc);
            held[(kG + g) * kStreamBlock + tid] = z[g];
        }
    } else {
#pragma unroll
        for (int e = 0; e < kHeldRegE; ++e)
            if (unsigned(e) < ne)
                unmarked_update(x[e], mr, mi, acc);
    }
}

// The sum of a thread's held vectors as they stand (e < ne in order, each vector's two amplitudes as
// held_sweep adds them), without the signs: correct_marked then makes it the oracle-signed sum.  Adds in
// exactly the order of an iteration, so a sum computed here from a stored state equals, bit for bit, the
// one the iteration that stored it produced.
__device__ inline void held_accumulate(const float4 (&x)[kHeldRegE], const float4 *held, unsigned ne, AccF64 &acc)
{
#pragma unroll
    for (int e = 0; e < kHeldHoldE; ++e)
        if (unsigned(e) < ne) {
            const float4 v = e < kHeldRegE ? x[e] : held[(e - kHeldRegE) * kStreamBlock + threadIdx.x];
            acc.add(double(v.x), double(v.y));
            acc.add(double(v.z), double(v.w));
        }
}

}  // namespace grover
