// Measured bandwidth ceiling of the fused iteration's memory access pattern (a measurement helper, not a
// step of the paper's method).  The probe runs the fused kernel's streaming skeleton with the arithmetic
// taken out: the same persistent grid (one 512-thread workgroup per CU), the same tiles (eight 16-byte
// vectors per thread, tile t owned by workgroup t mod G for every pass) and the same nontemporal buffer
// loads and stores as for a complex64 state (one descriptor per tile, nt on both), each element negated in
// place (read + write), or only read, or only written.  Full tiles take the same unchecked path as the
// fused kernel's (per-vector bounds checks on every tile cost the stream 6 %, 5.40 against 5.73 TB/s in
// place on MI355X).  The narrow form moves the same tiles with 1024 threads of four vectors each, the shape
// the fused kernel keeps for complex bfloat16.  In one launch the workgroups run through the passes freely;
// with one launch per pass, every pass starts only when the previous one has ended everywhere, as the fused
// kernel's grid barrier makes every iteration do, so that the whole grid streams one window of the buffer
// at a time.  What it reaches is what an in-place streaming pass of this shape can reach on the device; the
// fused kernel's own rate is then read against it.
#include "internal.h"

namespace grover {
namespace {

constexpr int kBlock = 512;
constexpr int kUnroll = 8;
constexpr int kTile = kBlock * kUnroll;
constexpr int kNarrowBlock = 1024;
constexpr int kNarrowUnroll = 4;

// WRITE: read, negate, write back; READ: only read; neither: only write (a constant).  B threads per
// workgroup, U vectors per thread per tile (B * U = kTile: 64 KiB tiles either way).
template <bool WRITE, bool READ = true, int B = kBlock, int U = kUnroll>
__global__ __launch_bounds__(B) void stream_probe_kernel(float4 *st, uint64_t nvec, uint32_t passes, uint32_t *sink)
{
    static_assert(B * U == kTile, "64 KiB tiles");
    constexpr int kBlock = B, kUnroll = U;
    const uint64_t ntiles = (nvec + kTile - 1) / kTile;
    const unsigned tid = threadIdx.x;
    uint32_t acc = 0u;
    // w: the vector's index within its tile
    auto visit = [&](float4 (&x)[kUnroll], __amdgpu_buffer_rsrc_t rs, uint32_t w, int u) {
        if (!READ) {
            bstore16<kBufNT>(x[u], rs, w * 16u);
        } else if (WRITE) {
            x[u].x = -x[u].x;
            x[u].y = -x[u].y;
            x[u].z = -x[u].z;
            x[u].w = -x[u].w;
            bstore16<kBufNT>(x[u], rs, w * 16u);
        } else {
            acc ^= __float_as_uint(x[u].x) ^ __float_as_uint(x[u].y) ^ __float_as_uint(x[u].z) ^
                   __float_as_uint(x[u].w);
        }
    };
    for (uint32_t p = 0; p < passes; ++p) {
        for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
            const uint64_t v0 = t * kTile;
            const uint64_t n = nvec - v0 < uint64_t(kTile) ? nvec - v0 : uint64_t(kTile);
            const auto rs = buffer_rsrc(st + v0, uint32_t(n * 16u));
            float4 x[kUnroll];
            if (n == uint64_t(kTile)) {
                // a full tile, like the fused kernel's: no bounds checks
#pragma unroll
                for (int u = 0; u < kUnroll; ++u)
                    x[u] = READ ? bload16<kBufNT, float4>(rs, (uint32_t(u) * kBlock + tid) * 16u)
                                : make_float4(float(p), 0.0f, float(p), 0.0f);
#pragma unroll
                for (int u = 0; u < kUnroll; ++u)
                    visit(x, rs, uint32_t(u) * kBlock + tid, u);
            } else {
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const uint32_t w = uint32_t(u) * kBlock + tid;
                    if (w < n)
                        x[u] = READ ? bload16<kBufNT, float4>(rs, w * 16u)
                                    : make_float4(float(p), 0.0f, float(p), 0.0f);
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const uint32_t w = uint32_t(u) * kBlock + tid;
                    if (w < n)
                        visit(x, rs, w, u);
                }
            }
        }
    }
    // the read-only probe must keep its loads: their values feed a store that (practically) never happens
    if (READ && !WRITE && acc == 0x9E3779B9u && sink)
        sink[0] = acc;
}

}  // namespace
}  // namespace grover

using namespace grover;

extern "C" int grover_stream_probe(void *hip_stream, void *buf_dev, size_t bytes, uint32_t passes, uint32_t mode,
                                   float *ms_out)
{
    if (!buf_dev || (reinterpret_cast<uintptr_t>(buf_dev) & 15u) != 0 || bytes < 16 || !ms_out ||
        (mode & ~uint32_t(GROVER_PROBE_READ_ONLY | GROVER_PROBE_LAUNCH_PER_PASS | GROVER_PROBE_WRITE_ONLY |
                          GROVER_PROBE_NARROW)) != 0u ||
        (mode & GROVER_PROBE_READ_ONLY) && (mode & GROVER_PROBE_WRITE_ONLY))
        return GROVER_E_INVAL;
    const bool read_only = (mode & GROVER_PROBE_READ_ONLY) != 0u;
    const bool write_only = (mode & GROVER_PROBE_WRITE_ONLY) != 0u;
    const bool narrow = (mode & GROVER_PROBE_NARROW) != 0u;
    const bool per_pass = (mode & GROVER_PROBE_LAUNCH_PER_PASS) != 0u;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess)
        return GROVER_E_HIP;
    uint64_t nvec = bytes / 16;
    const uint64_t ntiles = (nvec + kTile - 1) / kTile;
    const unsigned grid = unsigned(uint64_t(cus > 0 ? cus : 1) < ntiles ? uint64_t(cus > 0 ? cus : 1) : ntiles);
    float4 *st = static_cast<float4 *>(buf_dev);
    uint32_t *sink = nullptr;  // never written in practice; a null sink disables the store altogether
    uint32_t launch_passes = per_pass ? 1u : passes;
    const uint32_t launches = per_pass ? passes : (passes > 0u ? 1u : 0u);
    void *args[] = {&st, &nvec, &launch_passes, &sink};
    const void *fn = nullptr;
    constexpr int NB = kNarrowBlock, NU = kNarrowUnroll;
    if (narrow)
        fn = read_only    ? reinterpret_cast<const void *>(&stream_probe_kernel<false, true, NB, NU>)
             : write_only ? reinterpret_cast<const void *>(&stream_probe_kernel<false, false, NB, NU>)
                          : reinterpret_cast<const void *>(&stream_probe_kernel<true, true, NB, NU>);
    else
        fn = read_only    ? reinterpret_cast<const void *>(&stream_probe_kernel<false>)
             : write_only ? reinterpret_cast<const void *>(&stream_probe_kernel<false, false>)
                          : reinterpret_cast<const void *>(&stream_probe_kernel<true>);
    const unsigned block = narrow ? unsigned(kNarrowBlock) : unsigned(kBlock);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    if (e == hipSuccess)
        e = hipEventRecord(e0, stream);
    for (uint32_t l = 0; l < launches && e == hipSuccess; ++l)
        e = hipLaunchKernel(fn, dim3(grid), dim3(block), args, 0, stream);
    if (e == hipSuccess)
        e = hipEventRecord(e1, stream);
    if (e == hipSuccess)
        e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, e0, e1);
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return GROVER_E_HIP;
    }
    *ms_out = ms;
    return GROVER_OK;
}
