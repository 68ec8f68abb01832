// Device side of the allocation-free batched launch: the batched form's descriptor and work tables in
// a fixed file-scope array (one copy per GPU), filled by two small kernels in stream order before the
// tiled kernel runs. Nothing here allocates, copies from the host or clears memory with a memset, so
// the three launches can also be captured in a graph.
#include <hip/hip_runtime.h>

#include <mutex>

#include "nsa_internal.h"

// Holds the batched form's tables for every call on a GPU; each call rewrites the part it uses.
static __device__ __align__(256) unsigned char scratch[nsa::kStaticBytes];

namespace nsa {
namespace {

constexpr int kMaxDevices = 64;

// One lane per member of the chunk: its descriptor and first tile; lane count also writes the first
// tile after the chunk (the next chunk rewrites it with the same value).
__global__ __launch_bounds__(64) void k_put_desc(DescChunk c, TileArgs *desc, int64_t *toff) {
    const int i = (int)threadIdx.x;
    if (i < c.count) desc[c.first + i] = c.d[i];
    if (i <= c.count) toff[c.first + i] = c.toff[i];
}

// work[t] = (member, tile of that member) for t < total: the last member whose first tile is <= t
// (members without tiles share their first tile with the next one and are never chosen).
__global__ __launch_bounds__(256) void k_fill_work(const int64_t *__restrict__ toff, int32_t nmesh,
                                                   int2 *__restrict__ work, int64_t total) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    int32_t lo = 0, hi = nmesh;  // toff[lo] <= t < toff[hi]
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (toff[mid] <= t)
            lo = mid;
        else
            hi = mid;
    }
    work[t] = make_int2(lo, (int)(t - toff[lo]));
}

}  // namespace

hipError_t static_scratch(char **ptr) {
    static std::mutex mu;
    static char *per_device[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!per_device[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || ((uintptr_t)p % 256)) return hipErrorInvalidSymbol;
        per_device[dev] = (char *)p;
    }
    *ptr = per_device[dev];
    return hipSuccess;
}

hipError_t launch_put_desc(char *base, const DescChunk &c, hipStream_t s) {
    if (c.count <= 0 || c.count > kDescChunk || c.first < 0 || c.first + c.count > kStaticMeshes)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, c, reinterpret_cast<TileArgs *>(base),
                       reinterpret_cast<int64_t *>(base + kStaticToffOff));
    return hipGetLastError();
}

hipError_t launch_fill_work(char *base, int32_t nmesh, int64_t total, hipStream_t s) {
    if (nmesh <= 0 || nmesh > kStaticMeshes || total < 0 || total > kStaticTiles) return hipErrorInvalidValue;
    if (total == 0) return hipSuccess;
    const unsigned grid = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(k_fill_work, dim3(grid), dim3(256), 0, s,
                       reinterpret_cast<const int64_t *>(base + kStaticToffOff), nmesh,
                       reinterpret_cast<int2 *>(base + kStaticWorkOff), total);
    return hipGetLastError();
}

}  // namespace nsa
