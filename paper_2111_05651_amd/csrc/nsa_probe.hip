// Bandwidth probes: what this part's HBM delivers to plain streams, measured beside the assembly so
// that its achieved bandwidth can be set against a ceiling of the same device, not only the nominal
// 8 TB/s. 16-byte accesses, one pass. Each stream takes the launch shape that measured fastest for
// it on this part: reads grid-stride with four loads in flight per lane over 32 workgroups per CU;
// writes and copies as contiguous 256 KB chunks per workgroup (the shape of a tile's write-out) over
// 2 workgroups per CU.
#include <hip/hip_runtime.h>

#include "nsa_internal.h"

namespace nsa {
namespace {

constexpr int64_t kChunk = 16384;  // 16-byte items per chunk (256 KB)

__global__ __launch_bounds__(256) void k_probe_read(const double2 *__restrict__ src, int64_t n2, double *sink) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double a = 0.0, b = 0.0;
    for (; i + 3 * stride < n2; i += 4 * stride) {
        const double2 v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride], v3 = src[i + 3 * stride];
        a += (v0.x + v1.x) + (v2.x + v3.x);
        b += (v0.y + v1.y) + (v2.y + v3.y);
    }
    for (; i < n2; i += stride) {
        const double2 v = src[i];
        a += v.x;
        b += v.y;
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

hipError_t launch_probe(int kind, const double *src, double *dst, int64_t n, int ncu, hipStream_t s) {
    const int64_t n2 = n / 2;
    if (n2 <= 0) return hipSuccess;
    const dim3 b(256);
    if (kind == 0)
        hipLaunchKernelGGL(k_probe_read, dim3((unsigned)(32 * ncu)), b, 0, s, reinterpret_cast<const double2 *>(src),
                           n2, dst);
    else if (kind == 1)
        hipLaunchKernelGGL(k_probe_write, dim3((unsigned)(2 * ncu)), b, 0, s, reinterpret_cast<double2 *>(dst), n2, 1.0);
    else
        hipLaunchKernelGGL(k_probe_copy, dim3((unsigned)(2 * ncu)), b, 0, s, reinterpret_cast<const double2 *>(src),
                           reinterpret_cast<double2 *>(dst), n2);
    return hipGetLastError();
}

}  // namespace nsa
