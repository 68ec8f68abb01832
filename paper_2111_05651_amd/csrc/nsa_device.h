// Device helpers shared by the assembly kernels: streaming loads and stores, FP64 reciprocal and
// inverse cube root, and the FP64 geometry of a linear tetrahedron.
#pragma once

#include <hip/hip_runtime.h>

namespace nsa {

// Streaming accesses (the nt bit): data read or written once per launch -- a tile's run or element
// records, its block-image or row write-out -- so that it does not displace the node data that
// neighbouring tiles read again from L2.
typedef double stream_d2 __attribute__((ext_vector_type(2)));
typedef unsigned stream_u2 __attribute__((ext_vector_type(2)));
typedef unsigned stream_u4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void store_stream(double2 *p, double2 v) {
    __builtin_nontemporal_store((stream_d2){v.x, v.y}, reinterpret_cast<stream_d2 *>(p));
}
__device__ __forceinline__ void store_stream(double *p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ uint2 load_stream2(const uint2 *p) {
    const stream_u2 t = __builtin_nontemporal_load(reinterpret_cast<const stream_u2 *>(p));
    return make_uint2(t.x, t.y);
}
__device__ __forceinline__ uint4 load_stream(const uint4 *p) {
    const stream_u4 t = __builtin_nontemporal_load(reinterpret_cast<const stream_u4 *>(p));
    return make_uint4(t.x, t.y, t.z, t.w);
}

// Velocity of node g from vel[g][d] (soa == 0) or vel[d][g] (soa = the node count), as node stride sn
// and component stride sc: (3, 1) or (1, npoin). No branch, so the gathers of several nodes issue
// back to back whatever the layout.
__device__ __forceinline__ void load_vel3(const double *vel, int64_t soa, int64_t g, double &u, double &v, double &w) {
    const int64_t sn = soa ? 1 : 3, sc = soa ? soa : 1;
    const double *p = vel + g * sn;
    u = p[0];
    v = p[sc];
    w = p[2 * sc];
}
__device__ __forceinline__ double2 load_vel2(const double *vel, int64_t soa, int64_t g) {
    const int64_t sn = soa ? 1 : 2, sc = soa ? soa : 1;
    const double *p = vel + g * sn;
    return make_double2(p[0], p[sc]);
}

// Reciprocal: hardware estimate refined by two Newton steps (full FP64 accuracy for normal x).
__device__ __forceinline__ double fast_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Norm of the element's mean velocity for the stabilisation parameters, from its square x2: the
// hardware reciprocal square root (about 23 correct bits) and one Newton step y += (r/2)(x2 - y^2),
// which leaves a relative error of about 1.5 * 2^-46, against the 18 instructions of a correctly
// rounded sqrt (range scaling, two iterations, two corrections, special-value select). Below 1e-300
// (and for x2 = 0, where the estimate is infinite) the norm is taken as 0; it then only enters tau
// beside rho/dt and is negligible there.
__device__ __forceinline__ double tau_norm(double x2) {
    const double r = __builtin_amdgcn_rsq(x2);
    const double y = x2 * r;
    const double y1 = fma(0.5 * r, fma(-y, y, x2), y);
    return x2 > 1e-300 ? y1 : 0.0;
}
__device__ __forceinline__ float tau_norm(float x2) { return __builtin_amdgcn_sqrtf(x2); }

// x^(-1/3) for x > 0: FP32 estimate (2^(-log2(x)/3), relative error a few 1e-6 over the range) refined
// by two Newton steps r += r (1 - x r^3) / 3, each of which about squares the relative error (2e-6 ->
// ~1e-11 -> below FP64 rounding).
__device__ __forceinline__ double rcbrt(double x) {
    if (!(x > 1e-30 && x < 1e30)) return 1.0 / cbrt(x);  // outside the FP32 estimate's range
    float xf = (float)x;
    double r = (double)__builtin_amdgcn_exp2f(-__builtin_amdgcn_logf(xf) * (1.0f / 3.0f));
#pragma unroll
    for (int it = 0; it < 2; it++) r = fma(r * (1.0 / 3.0), fma(-x * r, r * r, 1.0), r);
    return r;
}

// Geometry in FP64: grad N_a, V, h = (6V)^(1/3) = |det|^(1/3) and 1/h.
struct Geo2 {
    double G[4][3];
    double V, h, rh;
};

__device__ __forceinline__ void geometry2(const double X[4][3], Geo2 &g) {
    double J[3][3];
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int s = 0; s < 3; s++) J[r][s] = X[s + 1][r] - X[0][r];
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double c10 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    const double c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    const double c12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    const double c20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    const double c21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    const double c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double inv = fast_rcp(det);
    g.G[1][0] = c00 * inv; g.G[1][1] = c10 * inv; g.G[1][2] = c20 * inv;
    g.G[2][0] = c01 * inv; g.G[2][1] = c11 * inv; g.G[2][2] = c21 * inv;
    g.G[3][0] = c02 * inv; g.G[3][1] = c12 * inv; g.G[3][2] = c22 * inv;
#pragma unroll
    for (int d = 0; d < 3; d++) g.G[0][d] = -(g.G[1][d] + g.G[2][d] + g.G[3][d]);
    const double adet = fabs(det);
    g.V = adet * (1.0 / 6.0);
    g.rh = rcbrt(adet);
    g.h = adet * g.rh * g.rh;
}

}  // namespace nsa
