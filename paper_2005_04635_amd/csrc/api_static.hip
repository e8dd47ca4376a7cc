// grover_iterate_static: the fused iteration (Algorithm 5's loop of Algorithm 3's oracle and Algorithm 4's
// inversion about the mean) for callers that cannot allocate device memory.  The only device memory it
// uses beyond the caller's state, marked list and status word is the grid barrier's: a fixed array of this
// translation unit, one copy per GPU, whose address is looked up once per device.
#include <algorithm>
#include <mutex>

#include "internal.h"

using namespace grover;

namespace {

constexpr int kStaticMaxGrid = 256;    // workgroups of the persistent grid (one per CU, at most this many)
constexpr int kStaticMaxDevices = 64;  // devices whose scratch address is remembered
constexpr uint64_t kSyncWords = sizeof(GridSync) / sizeof(uint64_t);
constexpr uint64_t kSlotWords = 8u * kStaticMaxGrid + 8u;  // tagged slots [2][grid][4] and the sum [2][4]
constexpr uint64_t kScratchWords = kSyncWords + kSlotWords;  // 2184 words = 17472 bytes

// The barrier's memory: the GridSync words (error word, ...) first, then the slots.  In host code this name
// is only a stand-in for the symbol; its device address comes from hipGetSymbolAddress.
static __device__ __align__(256) uint64_t scratch[kScratchWords];

struct DeviceScratch {
    uint64_t *ptr = nullptr;  // this device's copy of `scratch`
    int cu_count = 0;
    uint64_t ticks_per_ms = 0;  // device wall clock
};

std::mutex g_setup_mutex;
DeviceScratch g_dev[kStaticMaxDevices];

// Zeroes the barrier words and slots before every call: generations start at 1 each time, so a call (or a
// replay of a captured call) never accepts a value an earlier one left.  A kernel, not a memset, so that
// the call can be captured into a graph.
__global__ void static_clear_kernel(uint64_t *words, uint64_t n)
{
    for (uint64_t i = threadIdx.x; i < n; i += blockDim.x)
        words[i] = 0u;
}

// The kernels rely on a strictly increasing marked list of indices < N; a list that is not sets the error
// word to 2, which makes the iteration kernel return before it touches the state.
__global__ void static_check_marks_kernel(const uint64_t *marks, uint64_t m, uint64_t N, GridSync *sync)
{
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < m; i += stride)
        if (marks[i] >= N || (i > 0 && marks[i - 1] >= marks[i]))
            __hip_atomic_store(&sync->error, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void static_status_kernel(const GridSync *sync, uint32_t *status)
{
    status[0] = __hip_atomic_load(&sync->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

int fail(int status, const std::string &msg)
{
    set_thread_error(msg);
    return status;
}

int hip_fail(hipError_t e, const char *what)
{
    (void)hipGetLastError();
    return fail(e == hipErrorCooperativeLaunchTooLarge ? GROVER_E_COOP : GROVER_E_HIP,
                std::string(what) + ": " + hipGetErrorString(e));
}

// Set-up of the current device, once: the address of its copy of `scratch` and the launch facts.
int device_scratch(DeviceScratch *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "current device");
    if (dev < 0 || dev >= kStaticMaxDevices)
        return fail(GROVER_E_UNSUPPORTED, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_setup_mutex);
    DeviceScratch &d = g_dev[dev];
    if (!d.ptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_fail(e, "address of the static scratch array");
        int cus = 0, khz = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
        if (e != hipSuccess)
            return hip_fail(e, "device query");
        d.cu_count = cus;
        d.ticks_per_ms = uint64_t(khz > 0 ? khz : 100000);
        d.ptr = static_cast<uint64_t *>(p);
    }
    *out = d;
    return GROVER_OK;
}

}  // namespace

extern "C" int grover_iterate_static(void *hip_stream, void *state_dev, uint32_t n, uint32_t dtype,
                                     const uint64_t *marks_dev, uint64_t m, uint64_t k, uint32_t *status_dev)
{
    if (n < 1 || n > kMaxQubits)
        return fail(GROVER_E_INVAL, "n outside 1 .. 34");
    if (dtype > GROVER_CBF16)
        return fail(GROVER_E_INVAL, "unknown element type");
    const uint64_t N = uint64_t(1) << n;
    if (N < elems_per_vec(dtype))
        return fail(GROVER_E_UNSUPPORTED, "state smaller than one 16-byte vector");
    if (!state_dev || (reinterpret_cast<uintptr_t>(state_dev) & 15u) != 0)
        return fail(GROVER_E_INVAL, "state must be a 16-byte aligned device pointer");
    if (m > N || (m > 0 && !marks_dev))
        return fail(GROVER_E_INVAL, "marked list larger than the state, or missing");
    if (k >= (uint64_t(1) << 32) - 2u)
        return fail(GROVER_E_INVAL, "k must stay below 2^32 - 2 (barrier generations of one call)");
    DeviceScratch d;
    if (int st = device_scratch(&d))
        return st;
    // one workgroup per CU, never more than the scratch holds slots for, nor more than the state has tiles
    int64_t grid = std::min<int64_t>(d.cu_count > 0 ? d.cu_count : 1, kStaticMaxGrid);
    const uint64_t tiles = fused_tiles_of(dtype, N);
    if (uint64_t(grid) > tiles)
        grid = int64_t(tiles);
    if (grid < 1 || grid > kStaticMaxGrid)
        return fail(GROVER_E_INVAL, "persistent grid beyond the static scratch (at most 256 workgroups)");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    uint64_t *words = d.ptr;
    uint64_t nwords = kSyncWords + 8u * uint64_t(grid) + 8u;
    GridSync *sync = reinterpret_cast<GridSync *>(d.ptr);
    void *ca[] = {&words, &nwords};
    hipError_t e = hipLaunchKernel(reinterpret_cast<const void *>(&static_clear_kernel), dim3(1), dim3(256), ca, 0,
                                   stream);
    if (e != hipSuccess)
        return hip_fail(e, "clearing the barrier scratch");
    if (m > 0) {
        const uint64_t want = (m + 255u) / 256u;
        const unsigned blocks = unsigned(want < 1024u ? want : 1024u);
        uint64_t n_amps = N;
        void *ma[] = {&marks_dev, &m, &n_amps, &sync};
        e = hipLaunchKernel(reinterpret_cast<const void *>(&static_check_marks_kernel), dim3(blocks), dim3(256), ma, 0,
                            stream);
        if (e != hipSuccess)
            return hip_fail(e, "marked list check");
    }
    if (k > 0) {
        FusedExternal x;
        x.state = state_dev;
        x.dtype = dtype;
        x.N = N;
        x.marks = marks_dev;
        x.m = m;
        x.k = k;
        x.grid = int(grid);
        x.slots = d.ptr + kSyncWords;
        x.sync = sync;
        x.timeout_ticks = d.ticks_per_ms * 10000u;  // 10 s per barrier wait
        x.stream = stream;
        e = launch_fused_external(x);
        if (e != hipSuccess)
            return hip_fail(e, "fused iterate launch");
    }
    if (status_dev) {
        const GridSync *cs = sync;
        void *sa[] = {&cs, &status_dev};
        e = hipLaunchKernel(reinterpret_cast<const void *>(&static_status_kernel), dim3(1), dim3(1), sa, 0, stream);
        if (e != hipSuccess)
            return hip_fail(e, "status copy");
    }
    return GROVER_OK;
}
