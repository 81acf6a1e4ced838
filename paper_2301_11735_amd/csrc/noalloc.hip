// Batched observables with no device memory from the caller: the staging
// records the reduction kernel writes (10 int64 per lattice) live in a
// file-scope device array of the library instead of a caller buffer.  For
// callers that cannot allocate device memory (tight serving loops, harnesses
// that forbid it).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "internal.h"

namespace {

constexpr int kNoAllocMaxLattices = 1024;  // 80 KiB of records per device
constexpr int kNoAllocMaxDevices = 64;

// Device-side staging of every call on a device; the last call's records stay
// until the next call overwrites them.  Host code never passes this name to
// a kernel or a copy: it uses the address looked up for the current device.
static __device__ __align__(256) unsigned long long scratch[10 * kNoAllocMaxLattices];

std::mutex g_scratch_mu;
unsigned long long *g_scratch_dev[kNoAllocMaxDevices];  // address of `scratch` on device d, once looked up

// Address of `scratch` on the calling thread's current device, looked up with
// hipGetSymbolAddress on the first call made with that device current.
int scratch_on_current_device(unsigned long long **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return lat::detail::hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kNoAllocMaxDevices) return lat::detail::fail(LAT_EINVAL, "device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return lat::detail::hip_fail(e, "hipGetSymbolAddress of the static scratch");
        g_scratch_dev[dev] = (unsigned long long *)p;
    }
    *out = g_scratch_dev[dev];
    return LAT_OK;
}

}  // namespace

extern "C" int lattice_observables_batch_noalloc(lattice *const *hs, int32_t count, lat_obs *out, void *hip_stream)
{
    using namespace lat::detail;
    return guarded("lattice_observables_batch_noalloc", [&]() -> int {
        if (count < 0 || (count > 0 && (!hs || !out))) return fail(LAT_EINVAL, "bad batch");
        if (count > kNoAllocMaxLattices)
            return fail(LAT_EINVAL, "more than 1024 lattices in one lattice_observables_batch_noalloc call");
        for (int32_t i = 0; i < count; ++i)
            if (!live(hs[i])) return fail(LAT_ESTATE, "null or destroyed handle in batch");
        if (count == 0) return LAT_OK;
        unsigned long long *dev = nullptr;
        int rc = scratch_on_current_device(&dev);
        if (rc) return rc;
        hipStream_t stream = (hipStream_t)hip_stream;
        rc = enqueue_observables_batch(hs, count, dev, stream);  // the kernel zeroes its own records
        if (rc) return rc;
        int64_t v[10 * lat::kMaxBatch];  // host staging on the stack, one launch's worth at a time
        for (int32_t b = 0; b < count; b += lat::kMaxBatch) {
            const int32_t n = std::min<int32_t>(lat::kMaxBatch, count - b);
            hipError_t e = hipMemcpyAsync(v, dev + 10 * (size_t)b, (size_t)n * 80u, hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_fail(e, "lattice_observables_batch_noalloc");
            for (int32_t i = 0; i < n; ++i) fill_obs(hs[b + i], &v[10 * (size_t)i], &out[b + i]);
        }
        // lattices swept by the persistent kernel: its bounded device-wide
        // barrier flags a time-out in the lattice's error word
        for (int32_t i = 0; i < count; ++i) {
            if (!barrier_may_time_out(hs[i])) continue;
            uint32_t err = 0;
            const hipError_t e = hipMemcpy(&err, hs[i]->d_scratch + lat::kScrErr, sizeof(err), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "lattice_observables_batch_noalloc");
            if (err & 1u) return fail(LAT_EHIP, "a device-wide phase barrier timed out; the state is invalid");
        }
        return LAT_OK;
    });
}
