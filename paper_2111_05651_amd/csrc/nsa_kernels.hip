// HIP kernels for gfx950: P1-tetrahedron incompressible Navier-Stokes element assembly into a
// block-CSR matrix plus RHS (the element loop of the paper's Listing 1 with the block-CSR matrix
// as the assembly target).
//
// Element body. The paper evaluates its operators Gauss point by Gauss point (Listing 1's PGAUS
// loops; Listings 3/4). For linear tetrahedra every integrand is a product of at most two linear
// fields, so the 4-point rule is exact and each integral has a closed form in the barycentric
// coordinates, int N_k N_l = (V/20)(1 + delta_kl) and int N_k = V/4. With d[k][b] = U_k . grad N_b
// (the nodal values of a . grad N_b) and s_b = sum_k d[k][b]:
//   int N_a (a.grad N_b)           = V/20 (s_b + d[a][b])
//   int (a.grad N_a) N_b           = V/20 (s_a + d[b][a])
//   int (a.grad N_a)(a.grad N_b)   = V/20 (s_a s_b + sum_k d[k][a] d[k][b])
//   int a.grad N_a                 = V/4 s_a
//   int u_c N_a                    = V/20 (sum_k U_k[c] + U_a[c])
//   int (a.grad N_a) u_c           = V/20 (s_a sum_k U_k[c] + sum_k d[k][a] U_k[c])
// which replaces the per-Gauss-point loops with ~0.7k FP64 operations per element. The result is
// the same integral as the Gauss rule, up to rounding.
//
// Geometry (Jacobian, determinant, inverse, volume, element length) is always FP64; the element
// integration runs in the template type R (double, or float in the mixed-precision form); every
// contribution is converted to FP64 before it is added into the global arrays.
#include <hip/hip_runtime.h>

#include "nsa_internal.h"

namespace nsa {
namespace {

constexpr int kMaxThreads = 256;

struct Geo {
    double G[4][3];  // grad N_a
    double V;        // volume
    double h;        // element length (6V)^(1/3)
};

__device__ __forceinline__ void geometry(const double X[4][3], Geo &g) {
    double J[3][3];
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int s = 0; s < 3; s++) J[r][s] = X[s + 1][r] - X[0][r];
    // cofactors; inverse = transpose(cofactor) / det, grad N_{s+1}[d] = inverse[s][d] = cof[d][s]/det
    double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    double c10 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    double c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    double c12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    double c20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    double c21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    double c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    double inv = 1.0 / det;
    g.G[1][0] = c00 * inv; g.G[1][1] = c10 * inv; g.G[1][2] = c20 * inv;
    g.G[2][0] = c01 * inv; g.G[2][1] = c11 * inv; g.G[2][2] = c21 * inv;
    g.G[3][0] = c02 * inv; g.G[3][1] = c12 * inv; g.G[3][2] = c22 * inv;
#pragma unroll
    for (int d = 0; d < 3; d++) g.G[0][d] = -(g.G[1][d] + g.G[2][d] + g.G[3][d]);
    double adet = fabs(det);
    g.V = adet * (1.0 / 6.0);
    g.h = cbrt(adet);
}

// Per-element quantities in the integration precision R.
template <typename R>
struct Elem {
    R G[4][3];
    R d[4][4];   // d[k][b] = U_k . grad N_b
    R s[4];      // s_b = sum_k d[k][b] = 4 abar . grad N_b
    R rdt, rho;
    R v4, v20, muV, t2V, t1V, t1, t1rho;
};

template <typename R>
__device__ __forceinline__ void element_setup(const Geo &g, const double Ud[4][3], double rho_d,
                                              double mu_d, double dt_d, Elem<R> &E, R rb[16]) {
    R U[4][3];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            U[a][c] = (R)Ud[a][c];
            E.G[a][c] = (R)g.G[a][c];
        }
    const R V = (R)g.V, h = (R)g.h, rho = (R)rho_d, mu = (R)mu_d;
    const R rdt = (R)(rho_d / dt_d);
    R su[3];
#pragma unroll
    for (int c = 0; c < 3; c++) su[c] = U[0][c] + U[1][c] + U[2][c] + U[3][c];
    const R q = (R)0.25;
    R an = sqrt(su[0] * su[0] * q * q + su[1] * su[1] * q * q + su[2] * su[2] * q * q);
    R t1 = (R)1 / (rdt + (R)4 * mu / (h * h) + (R)2 * rho * an / h);
    R t2 = mu + (R)0.5 * rho * an * h;
#pragma unroll
    for (int k = 0; k < 4; k++)
#pragma unroll
        for (int b = 0; b < 4; b++) E.d[k][b] = U[k][0] * E.G[b][0] + U[k][1] * E.G[b][1] + U[k][2] * E.G[b][2];
#pragma unroll
    for (int b = 0; b < 4; b++) E.s[b] = E.d[0][b] + E.d[1][b] + E.d[2][b] + E.d[3][b];
    E.rdt = rdt;
    E.rho = rho;
    E.v4 = V * (R)0.25;
    E.v20 = V * (R)0.05;
    E.muV = mu * V;
    E.t2V = t2 * V;
    E.t1V = t1 * V;
    E.t1 = t1;
    E.t1rho = t1 * rho;
    // RHS: (rho/dt) int u_c N_a + tau1 rho (rho/dt) int (a.grad N_a) u_c ; PSPG tau1 (rho/dt) V/4 s_a
#pragma unroll
    for (int a = 0; a < 4; a++) {
#pragma unroll
        for (int c = 0; c < 3; c++) {
            R un = E.v20 * (su[c] + U[a][c]);
            R au = E.v20 * (E.s[a] * su[c] + E.d[0][a] * U[0][c] + E.d[1][a] * U[1][c] +
                            E.d[2][a] * U[2][c] + E.d[3][a] * U[3][c]);
            rb[4 * a + c] = rdt * (un + E.t1rho * au);
        }
        rb[4 * a + 3] = t1 * rdt * E.v4 * E.s[a];
    }
}

// 4x4 block (a, b) of the element matrix: blk[4c + c'], rows c (test), columns c' (trial).
template <typename R>
__device__ __forceinline__ void element_block(const Elem<R> &E, int a, int b, R blk[16]) {
    const R K = E.G[a][0] * E.G[b][0] + E.G[a][1] * E.G[b][1] + E.G[a][2] * E.G[b][2];
    const R gram = E.d[0][a] * E.d[0][b] + E.d[1][a] * E.d[1][b] + E.d[2][a] * E.d[2][b] + E.d[3][a] * E.d[3][b];
    const R mass = (a == b) ? E.v20 * (R)2 : E.v20;
    const R conv = E.v20 * (E.s[b] + E.d[a][b]);
    const R cnvt = E.v20 * (E.s[a] + E.d[b][a]);
    const R aa = E.v20 * (E.s[a] * E.s[b] + gram);
    const R T = E.rdt * mass + E.rho * conv + E.muV * K + E.t1rho * (E.rho * aa + E.rdt * cnvt);
#pragma unroll
    for (int c = 0; c < 3; c++)
#pragma unroll
        for (int cp = 0; cp < 3; cp++) {
            R v = E.muV * E.G[a][cp] * E.G[b][c] + E.t2V * E.G[a][c] * E.G[b][cp];
            blk[4 * c + cp] = (c == cp) ? v + T : v;
        }
    const R iag_a = E.v4 * E.s[a];
    const R rb = E.rho * E.v4 * E.s[b] + E.rdt * E.v4;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        blk[4 * c + 3] = -E.v4 * E.G[a][c] + E.t1rho * iag_a * E.G[b][c];
        blk[12 + c] = E.v4 * E.G[b][c] + E.t1 * E.G[a][c] * rb;
    }
    blk[15] = E.t1V * K;
}

template <typename R, bool COLOUR>
__global__ __launch_bounds__(kMaxThreads) void k_assemble(AsmArgs A) {
    const int64_t e = A.e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= A.e1) return;
    int n[4];
#pragma unroll
    for (int a = 0; a < 4; a++) n[a] = A.ln[a * A.ld + e];
    double X[4][3], U[4][3];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int d = 0; d < 3; d++) {
            X[a][d] = A.coord[d * A.npoin + n[a]];
            U[a][d] = A.vel[3 * (int64_t)n[a] + d];
        }
    Geo g;
    geometry(X, g);
    Elem<R> E;
    R rb[16];
    element_setup<R>(g, U, A.rho, A.mu, A.dt, E, rb);
#pragma unroll
    for (int a = 0; a < 4; a++) {
        double *r = A.rhs + 4 * (int64_t)n[a];
        if (COLOUR) {
            double2 *r2 = reinterpret_cast<double2 *>(r);
            double2 v0 = r2[0], v1 = r2[1];
            v0.x += (double)rb[4 * a + 0];
            v0.y += (double)rb[4 * a + 1];
            v1.x += (double)rb[4 * a + 2];
            v1.y += (double)rb[4 * a + 3];
            r2[0] = v0;
            r2[1] = v1;
        } else {
#pragma unroll
            for (int c = 0; c < 4; c++) unsafeAtomicAdd(r + c, (double)rb[4 * a + c]);
        }
    }
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) {
            R blk[16];
            element_block<R>(E, a, b, blk);
            double *p = A.values + 16 * (int64_t)A.emap[(4 * a + b) * A.ld + e];
            if (COLOUR) {
                double2 *p2 = reinterpret_cast<double2 *>(p);
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    double2 v = p2[i];
                    v.x += (double)blk[2 * i];
                    v.y += (double)blk[2 * i + 1];
                    p2[i] = v;
                }
            } else {
#pragma unroll
                for (int i = 0; i < 16; i++) unsafeAtomicAdd(p + i, (double)blk[i]);
            }
        }
}

__global__ void k_fill_zero(double2 *p, int64_t n2) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride)
        p[i] = make_double2(0.0, 0.0);
}

__global__ void k_fill_zero_tail(double *p, int64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && (n & 1)) p[n - 1] = 0.0;
}

}  // namespace

hipError_t launch_fill_zero(double *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t n2 = n / 2;
    if (n2 > 0) {
        int64_t blocks = std::min<int64_t>((n2 + 255) / 256, 256 * 32);
        hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<double2 *>(p), n2);
    }
    if (n & 1) hipLaunchKernelGGL(k_fill_zero_tail, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_assemble(Kern k, const AsmArgs &a, int threads, hipStream_t s) {
    const int64_t n = a.e1 - a.e0;
    if (n <= 0) return hipSuccess;
    if (threads > kMaxThreads) threads = kMaxThreads;
    const dim3 grid((unsigned)((n + threads - 1) / threads)), block(threads);
    switch (k) {
        case Kern::AtomicF64: hipLaunchKernelGGL((k_assemble<double, false>), grid, block, 0, s, a); break;
        case Kern::AtomicMixed: hipLaunchKernelGGL((k_assemble<float, false>), grid, block, 0, s, a); break;
        case Kern::ColourF64: hipLaunchKernelGGL((k_assemble<double, true>), grid, block, 0, s, a); break;
        case Kern::ColourMixed: hipLaunchKernelGGL((k_assemble<float, true>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

}  // namespace nsa
