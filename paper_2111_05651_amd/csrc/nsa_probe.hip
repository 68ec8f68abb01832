// Bandwidth probes: what this part's HBM delivers to plain streams, measured beside the assembly so
// that its achieved bandwidth can be set against a ceiling of the same device, not only the nominal
// 8 TB/s. Each workgroup streams contiguous 256 KB chunks (16-byte accesses, one pass; the same shape as
// a tile's write-out, which measured faster than a grid-stride walk).
#include <hip/hip_runtime.h>

#include "nsa_internal.h"

namespace nsa {
namespace {

constexpr int64_t kChunk = 16384;  // 16-byte items per chunk (256 KB)

__global__ __launch_bounds__(256) void k_probe_read(const double2 *__restrict__ src, int64_t n2, double *sink) {
    double a = 0.0, b = 0.0;
    for (int64_t c = blockIdx.x; c * kChunk < n2; c += gridDim.x) {
        const int64_t lo = c * kChunk, hi = lo + kChunk < n2 ? lo + kChunk : n2;
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            const double2 v = src[i];
            a += v.x;
            b += v.y;
        }
    }
    // never true for finite data; keeps the loads
    if (a == 1.0e300 && b == -1.0e300) sink[0] = a + b;
}

__global__ __launch_bounds__(256) void k_probe_write(double2 *__restrict__ dst, int64_t n2, double v) {
    for (int64_t c = blockIdx.x; c * kChunk < n2; c += gridDim.x) {
        const int64_t lo = c * kChunk, hi = lo + kChunk < n2 ? lo + kChunk : n2;
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) dst[i] = make_double2(v, v);
    }
}

__global__ __launch_bounds__(256) void k_probe_copy(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                                    int64_t n2) {
    for (int64_t c = blockIdx.x; c * kChunk < n2; c += gridDim.x) {
        const int64_t lo = c * kChunk, hi = lo + kChunk < n2 ? lo + kChunk : n2;
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) dst[i] = src[i];
    }
}

}  // namespace

hipError_t launch_probe(int kind, const double *src, double *dst, int64_t n, int grid, hipStream_t s) {
    const int64_t n2 = n / 2;
    if (n2 <= 0) return hipSuccess;
    const dim3 g((unsigned)grid), b(256);
    if (kind == 0)
        hipLaunchKernelGGL(k_probe_read, g, b, 0, s, reinterpret_cast<const double2 *>(src), n2, dst);
    else if (kind == 1)
        hipLaunchKernelGGL(k_probe_write, g, b, 0, s, reinterpret_cast<double2 *>(dst), n2, 1.0);
    else
        hipLaunchKernelGGL(k_probe_copy, g, b, 0, s, reinterpret_cast<const double2 *>(src),
                           reinterpret_cast<double2 *>(dst), n2);
    return hipGetLastError();
}

}  // namespace nsa
