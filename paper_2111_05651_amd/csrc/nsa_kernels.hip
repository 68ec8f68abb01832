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

#include <map>
#include <type_traits>
#include <mutex>

#include "nsa_device.h"
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
    for (int a = 0; a < 4; a++) {
#pragma unroll
        for (int d = 0; d < 3; d++) X[a][d] = A.coord[d * A.npoin + n[a]];
        load_vel3(A.vel, A.vel_soa, n[a], U[a][0], U[a][1], U[a][2]);
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

// Seeded uniform values for synthetic inputs: value i is lo + (hi - lo) u_i with u_i the top 53
// bits of splitmix64 (Steele, Lea and Flood's mixing function) at counter seed + (i + 1) * gamma,
// gamma = 2^64 / golden ratio. Multiply and add are rounded separately so that any other
// implementation of the same definition gives the same bits.
__global__ void k_fill_uniform(double *p, int64_t n, uint64_t seed, double lo, double span) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const double u = (double)(z >> 11) * 0x1.0p-53;
        p[i] = __dadd_rn(lo, __dmul_rn(span, u));
    }
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

hipError_t launch_fill_uniform(double *p, int64_t n, uint64_t seed, double lo, double hi, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 256 * 64);
    hipLaunchKernelGGL(k_fill_uniform, dim3((unsigned)blocks), dim3(256), 0, s, p, n, seed, lo, hi - lo);
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

// ================================================================================================
// Row-tiled assembly (the default path).
//
// One workgroup owns a tile of contiguous block rows and the contiguous range of blocks they hold.
// It stages the coordinates and velocities of the nodes its elements touch in LDS, keeps an FP64
// image of its blocks (and of its RHS rows) in LDS, runs every element that touches one of its rows
// from a precomputed 24-byte record, adds the contributions of the owned rows into the LDS image
// with FP64 LDS atomics (ds_add_f64), and finally writes the image to HBM once, coalesced. No
// global atomics, no zero-fill pass, and every value line is written exactly once. Elements on a
// tile boundary are evaluated by each tile they touch; only their owned rows are integrated there.
//
// The LDS atomics set the pace: the LDS serves an 8-byte atomic 16 lanes at a time, one pass per
// lane on the busiest bank pair, so the throughput plan orders its records such that the 16 lanes
// of each group add into blocks on distinct bank pairs as far as it can (host planner).
//
// Two plans use this kernel. The throughput plan gives a tile to a workgroup of four wavefronts;
// the order in which their LDS atomics land on one block varies from run to run. The deterministic
// plan gives each (smaller) tile to a single wavefront: every LDS word of the tile is then updated
// only by that wavefront's instructions, which the LDS executes in issue order, lanes of one
// instruction in a fixed order, so the sums are bit-reproducible; its records take the same
// bank-aware order as the throughput plan's.
// ================================================================================================
namespace {

// Element state in the integration precision R, for the closed-form integrals of the header.
template <typename R>
struct ElemT {
    R G[4][3];
    R d[4][4];   // d[k][b] = U_k . grad N_b
    R s[4];      // s_b = sum_k d[k][b]
    R U[4][3];
    R su[3];     // sum_k U_k
    R rdt, rho, v4, v20, muV, t2V, t1V, t1, t1rho;
    R Mo, Md;    // mass coefficients (rho/dt) V/20 for a != b and a == b
    R c1, c2, c3;  // rho V/20, tau1 rho^2 V/20, tau1 rho (rho/dt) V/20
};

template <typename R>
__device__ __forceinline__ void setup_t(const Geo2 &g, const double Ud[4][3], double rho_d, double mu_d, double dt_d,
                                        ElemT<R> &E) {
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            E.U[a][c] = (R)Ud[a][c];
            E.G[a][c] = (R)g.G[a][c];
        }
    const R V = (R)g.V, h = (R)g.h, rh = (R)g.rh, rho = (R)rho_d, mu = (R)mu_d;
    const R rdt = (R)(rho_d / dt_d);
#pragma unroll
    for (int c = 0; c < 3; c++) E.su[c] = E.U[0][c] + E.U[1][c] + E.U[2][c] + E.U[3][c];
    const R an = (R)0.25 * tau_norm(E.su[0] * E.su[0] + E.su[1] * E.su[1] + E.su[2] * E.su[2]);
    const R t1 = fast_rcp(rdt + (R)4 * mu * rh * rh + (R)2 * rho * an * rh);
    const R t2 = mu + (R)0.5 * rho * an * h;
#pragma unroll
    for (int k = 0; k < 4; k++)
#pragma unroll
        for (int b = 0; b < 4; b++) E.d[k][b] = E.U[k][0] * E.G[b][0] + E.U[k][1] * E.G[b][1] + E.U[k][2] * E.G[b][2];
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
    E.Mo = rdt * E.v20;
    E.Md = E.Mo + E.Mo;
    E.c1 = rho * E.v20;
    E.c2 = E.t1rho * rho * E.v20;
    E.c3 = E.t1rho * rdt * E.v20;
}

// Row a of the element: RHS (4 values) and the four 4x4 blocks (a, b), each handed to put(b, blk).
// Per row the coefficients that depend on a only are formed once; a block then costs ~40 operations:
//   T    = (rho/dt) V/20 (1 + d_ab) + rho V/20 (s_b + d[a][b]) + mu V K_ab
//          + tau1 rho (rho V/20 (s_a s_b + gram_ab) + (rho/dt) V/20 (s_a + d[b][a]))
//   uu   = T I + mu V G_b G_a^T + tau2 V G_a G_b^T         (diagonal: G_b[c] (mu V + tau2 V) G_a[c] + T)
//   up   = -V/4 G_a + tau1 rho V/4 s_a G_b
//   pu   = V/4 G_b + tau1 G_a (rho V/4 s_b + (rho/dt) V/4)
//   pp   = tau1 V K_ab
template <typename R, typename Put>
__device__ __forceinline__ void element_row(const ElemT<R> &E, int a, R rb[4], Put put) {
    const R ga[3] = {E.G[a][0], E.G[a][1], E.G[a][2]};
    const R sa = E.s[a];
    // RHS: (rho/dt) int u_c N_a + tau1 rho (rho/dt) int (a.grad N_a) u_c ; PSPG tau1 (rho/dt) V/4 s_a
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const R un = E.su[c] + E.U[a][c];
        const R au = sa * E.su[c] + E.d[0][a] * E.U[0][c] + E.d[1][a] * E.U[1][c] + E.d[2][a] * E.U[2][c] +
                     E.d[3][a] * E.U[3][c];
        rb[c] = E.rdt * E.v20 * (un + E.t1rho * au);
    }
    rb[3] = E.t1 * E.rdt * E.v4 * sa;
    R gm[3], gt[3], gmt[3], pa[3], tg[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        gm[c] = E.muV * ga[c];
        gt[c] = E.t2V * ga[c];
        gmt[c] = gm[c] + gt[c];
        pa[c] = -E.v4 * ga[c];
        tg[c] = E.t1 * ga[c];
    }
    const R qa = E.t1rho * E.v4 * sa;
    const R tbase = E.Mo + E.c3 * sa;        // a-only part of T
    const R ksb = E.c1 + E.c2 * sa;          // coefficient of s_b in T
    const R rv4 = E.rho * E.v4, dv4 = E.rdt * E.v4;
#pragma unroll
    for (int b = 0; b < 4; b++) {
        const R gb[3] = {E.G[b][0], E.G[b][1], E.G[b][2]};
        const R sb = E.s[b];
        const R K = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
        const R gram = E.d[0][a] * E.d[0][b] + E.d[1][a] * E.d[1][b] + E.d[2][a] * E.d[2][b] + E.d[3][a] * E.d[3][b];
        R T = tbase + ksb * sb + E.c1 * E.d[a][b] + E.c3 * E.d[b][a] + E.c2 * gram + E.muV * K;
        if (a == b) T += E.Mo;
        R blk[16];
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
            for (int cp = 0; cp < 3; cp++)
                blk[4 * c + cp] = (c == cp) ? gb[c] * gmt[c] + T : gm[cp] * gb[c] + gt[c] * gb[cp];
        const R rbb = rv4 * sb + dv4;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            blk[4 * c + 3] = pa[c] + qa * gb[c];
            blk[12 + c] = E.v4 * gb[c] + tg[c] * rbb;
        }
        blk[15] = E.t1V * K;
        put(b, blk);
    }
}

__device__ __forceinline__ void lds_add(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Coordinates and velocity of local node l from the tile's LDS node table.
__device__ __forceinline__ void node_load(const double *nodes, int l, double X[3], double U[3]) {
    const double2 *nd = reinterpret_cast<const double2 *>(nodes + 6 * l);
    const double2 q0 = nd[0], q1 = nd[1], q2 = nd[2];
    X[0] = q0.x;
    X[1] = q0.y;
    X[2] = q1.x;
    U[0] = q1.y;
    U[1] = q2.x;
    U[2] = q2.y;
}

__device__ __forceinline__ void lds_add16(double *p, const double v[16]) {
#pragma unroll
    for (int i = 0; i < 16; i++) lds_add(p + i, v[i]);
}

// Row 0 of an element (its local vertex 0 is the run's row node): what the four blocks (0, b) and the
// RHS row need, reduced to per-column scalars so that the gradient products and the velocity die
// before the blocks are formed. With d[k][b] = U_k . grad N_b and s_b = sum_k d[k][b] (see
// element_row), for column b:
//   T_b = (rho/dt) V/20 (1 + d_0b) + rho V/20 (s_b + d[0][b]) + mu V K_0b
//         + tau1 rho (rho V/20 (s_0 s_b + gram_0b) + (rho/dt) V/20 (s_0 + d[b][0]))
// and the block is uu = T_b I + mu V G_b G_0^T + tau2 V G_0 G_b^T, up = -V/4 G_0 + tau1 rho V/4 s_0 G_b,
// pu = V/4 G_b + tau1 G_0 (rho V/4 s_b + (rho/dt) V/4), pp = tau1 V K_0b.
template <typename R>
struct Row0 {
    R gb[4][3];                         // grad N_b
    R T[4], K[4], s[4];
    R gm[3], gt[3], gmt[3], pa[3], tg[3];
    R qa, v4, t1V, rv4, dv4;
};

template <typename R>
__device__ __forceinline__ void row0_setup(const Geo2 &g, const double Ud[4][3], double rho_d, double mu_d,
                                           double rdt_d, Row0<R> &C, R rb[4]) {
    R U[4][3];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            U[a][c] = (R)Ud[a][c];
            C.gb[a][c] = (R)g.G[a][c];
        }
    const R V = (R)g.V, h = (R)g.h, rh = (R)g.rh, rho = (R)rho_d, mu = (R)mu_d;
    const R rdt = (R)rdt_d;
    R su[3];
#pragma unroll
    for (int c = 0; c < 3; c++) su[c] = U[0][c] + U[1][c] + U[2][c] + U[3][c];
    const R an = (R)0.25 * tau_norm(su[0] * su[0] + su[1] * su[1] + su[2] * su[2]);
    const R t1 = fast_rcp(rdt + (R)4 * mu * rh * rh + (R)2 * rho * an * rh);
    const R t2 = mu + (R)0.5 * rho * an * h;
    const R v4 = V * (R)0.25, v20 = V * (R)0.05, muV = mu * V, t2V = t2 * V, t1rho = t1 * rho;
    const R Mo = rdt * v20, c1 = rho * v20, c2 = t1rho * rho * v20, c3 = t1rho * rdt * v20;
    const R *g0 = C.gb[0];
    R dk0[4];  // d[k][0]
#pragma unroll
    for (int k = 0; k < 4; k++) dk0[k] = U[k][0] * g0[0] + U[k][1] * g0[1] + U[k][2] * g0[2];
    const R s0 = dk0[0] + dk0[1] + dk0[2] + dk0[3];
    // w = sum_k d[k][0] U_k: then sum_k d[k][0] d[k][b] = w . grad N_b and sum_k d[k][b] = su . grad N_b,
    // so no d[k][b] with b > 0 is formed
    R w[3];
#pragma unroll
    for (int c = 0; c < 3; c++) w[c] = dk0[0] * U[0][c] + dk0[1] * U[1][c] + dk0[2] * U[2][c] + dk0[3] * U[3][c];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const R un = su[c] + U[0][c];
        const R au = s0 * su[c] + w[c];
        rb[c] = rdt * v20 * (un + t1rho * au);
    }
    rb[3] = t1 * rdt * v4 * s0;
    const R tbase = Mo + c3 * s0, ksb = c1 + c2 * s0;
    // T_b = tbase + c3 d[b][0] + ksb s_b + c1 d[0][b] + c2 gram_0b + muV K_0b, and each of s_b, d[0][b],
    // gram_0b, K_0b is a dot product with grad N_b: T_b = tbase + c3 d[b][0] + z . grad N_b with
    // z = ksb su + c1 U_0 + c2 w + muV grad N_0
    R z[3];
#pragma unroll
    for (int c = 0; c < 3; c++) z[c] = ksb * su[c] + c1 * U[0][c] + c2 * w[c] + muV * g0[c];
#pragma unroll
    for (int b = 0; b < 4; b++) {
        const R *gb = C.gb[b];
        const R sb = su[0] * gb[0] + su[1] * gb[1] + su[2] * gb[2];        // sum_k d[k][b]
        const R K = g0[0] * gb[0] + g0[1] * gb[1] + g0[2] * gb[2];
        R T = tbase + c3 * dk0[b] + (z[0] * gb[0] + z[1] * gb[1] + z[2] * gb[2]);
        if (b == 0) T += Mo;
        C.T[b] = T;
        C.K[b] = K;
        C.s[b] = sb;
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
        C.gm[c] = muV * g0[c];
        C.gt[c] = t2V * g0[c];
        C.gmt[c] = C.gm[c] + C.gt[c];
        C.pa[c] = -v4 * g0[c];
        C.tg[c] = t1 * g0[c];
    }
    C.qa = t1rho * v4 * s0;
    C.v4 = v4;
    C.t1V = t1 * V;
    C.rv4 = rho * v4;
    C.dv4 = rdt * v4;
}

// acc (+)= block (0, b) of the element: FRESH overwrites, otherwise adds (FP64: folded into the
// multiply-adds; mixed: each FP32 value converted, then added in FP64).
template <typename R, bool FRESH>
__device__ __forceinline__ void block0(const Row0<R> &C, int b, double acc[16]) {
    const R *gb = C.gb[b];
    const R T = C.T[b], K = C.K[b];
    const R rbb = C.rv4 * C.s[b] + C.dv4;
    if constexpr (std::is_same<R, double>::value) {
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
            for (int cp = 0; cp < 3; cp++) {
                double &a = acc[4 * c + cp];
                if (c == cp)
                    a = FRESH ? fma(gb[c], C.gmt[c], T) : fma(gb[c], C.gmt[c], a) + T;
                else
                    a = FRESH ? fma(C.gm[cp], gb[c], C.gt[c] * gb[cp]) : fma(C.gt[c], gb[cp], fma(C.gm[cp], gb[c], a));
            }
#pragma unroll
        for (int c = 0; c < 3; c++) {
            double &u = acc[4 * c + 3];
            u = FRESH ? fma(C.qa, gb[c], C.pa[c]) : fma(C.qa, gb[c], u) + C.pa[c];
            double &p = acc[12 + c];
            p = FRESH ? fma(C.v4, gb[c], C.tg[c] * rbb) : fma(C.tg[c], rbb, fma(C.v4, gb[c], p));
        }
        acc[15] = FRESH ? C.t1V * K : fma(C.t1V, K, acc[15]);
    } else {
        R v[16];
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
            for (int cp = 0; cp < 3; cp++)
                v[4 * c + cp] = (c == cp) ? gb[c] * C.gmt[c] + T : C.gm[cp] * gb[c] + C.gt[c] * gb[cp];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            v[4 * c + 3] = C.pa[c] + C.qa * gb[c];
            v[12 + c] = C.v4 * gb[c] + C.tg[c] * rbb;
        }
        v[15] = C.t1V * K;
#pragma unroll
        for (int i = 0; i < 16; i++) acc[i] = FRESH ? (double)v[i] : acc[i] + (double)v[i];
    }
}

// One run (RunRec as two uint4: h = row, hinge, k0, len, diag, jslot, last, pad; k = knew[4],
// kslot[4]). Element q of the run has the vertices (row, hinge, k_old(q), k_new(q)); only row `row`
// (local vertex 0) is integrated. The lane sums in FP64 registers the diagonal block and the RHS
// row (every element of the run adds to them), the block (row, hinge) (likewise) and the block
// (row, k_new(q)), which element q+1 adds to again as its (row, k_old); that sum is complete after
// element q+1 and goes into the LDS image then. Per element one block is added into LDS, per run
// three blocks and the RHS row.
enum NodeLoads { NL_ALL, NL_AHEAD };

template <typename R, int NL>
__device__ __forceinline__ void tile_run(const TileArgs &A, double rdt, const uint4 h, const uint4 k, double *acc,
                                         double *racc, const double *nodes) {
    const int row = (int)(h.x & 0xffffu), hinge = (int)(h.x >> 16);
    const int len = (int)(h.y >> 16);
    const int dslot = (int)(h.z & 0xffffu), jslot = (int)(h.z >> 16), last = (int)(h.w & 0xffffu);
    // The mixed form stores the first element's block sums instead of adding them to zeroed registers
    // (48 fewer moves per run, 128^3 mixed -1.7 %); the FP64 form zeroes them (storing costs the batched
    // FP64 kernel 4 spilled registers).
    constexpr bool kFirstStores = !std::is_same<R, double>::value;
    double sd[16], sj[16], sa[16], sr[4];
    if (!kFirstStores) {
#pragma unroll
        for (int i = 0; i < 16; i++) sd[i] = sj[i] = sa[i] = 0.0;
#pragma unroll
        for (int c = 0; c < 4; c++) sr[c] = 0.0;
    }
    // Node reads (NL): consecutive elements share the row, the hinge and one more node, so with
    // NL_AHEAD each element reads one new node from the node table and keeps the others in registers,
    // reading it one element ahead, before the current element's LDS adds (LDS operations complete in
    // order, so a read issued after 16 adds waits for them). NL_ALL reads all four nodes per element
    // (fewest registers: the FP64 form keeps no node data across elements).
    constexpr bool kAhead = NL == NL_AHEAD;
    double Xr[3], Ur[3], Xh[3], Uh[3], Xo[3], Uo[3], Xn[3], Un[3];
    if (NL != NL_ALL) {
        node_load(nodes, row, Xr, Ur);
        node_load(nodes, hinge, Xh, Uh);
        node_load(nodes, (int)(h.y & 0xffffu), Xo, Uo);
    }
    if (kAhead) node_load(nodes, (int)(k.x & 0xffffu), Xn, Un);
    int kold = (int)(h.y & 0xffffu);
    for (int q = 0; q < len; q++) {
        const int sh = (q & 1) * 16;
        const int ks = (int)(((q < 2 ? k.z : k.w) >> sh) & 0xffffu);
        const int kn = (int)(((q < 2 ? k.x : k.y) >> sh) & 0xffffu);
        if (NL == NL_ALL) {
            node_load(nodes, row, Xr, Ur);
            node_load(nodes, hinge, Xh, Uh);
            node_load(nodes, kold, Xo, Uo);
        }
        if (!kAhead) node_load(nodes, kn, Xn, Un);
        kold = kn;
        Row0<R> C;
        R rb[4];
        {
            double X[4][3], U[4][3];
#pragma unroll
            for (int c = 0; c < 3; c++) {
                X[0][c] = Xr[c];
                X[1][c] = Xh[c];
                X[2][c] = Xo[c];
                X[3][c] = Xn[c];
                U[0][c] = Ur[c];
                U[1][c] = Uh[c];
                U[2][c] = Uo[c];
                U[3][c] = Un[c];
            }
            Geo2 g;
            geometry2(X, g);
            row0_setup<R>(g, U, A.rho, A.mu, rdt, C, rb);
        }
#pragma unroll
        for (int c = 0; c < 3; c++) {
            Xo[c] = Xn[c];
            Uo[c] = Un[c];
        }
        if (kAhead && q + 1 < len) {
            const int sh1 = ((q + 1) & 1) * 16;
            node_load(nodes, (int)(((q + 1 < 2 ? k.x : k.y) >> sh1) & 0xffffu), Xn, Un);
        }
        if (kFirstStores && q == 0) {
#pragma unroll
            for (int c = 0; c < 4; c++) sr[c] = (double)rb[c];
            block0<R, true>(C, 0, sd);
            block0<R, true>(C, 1, sj);
            block0<R, true>(C, 2, sa);
        } else {
#pragma unroll
            for (int c = 0; c < 4; c++) sr[c] += (double)rb[c];
            block0<R, false>(C, 0, sd);
            block0<R, false>(C, 1, sj);
            block0<R, false>(C, 2, sa);
        }
        lds_add16(acc + kBlkStride * ks, sa);
        block0<R, true>(C, 3, sa);
    }
    lds_add16(acc + kBlkStride * last, sa);
    lds_add16(acc + kBlkStride * jslot, sj);
    lds_add16(acc + kBlkStride * dslot, sd);
    double *r = racc + kRhsStride * row;
#pragma unroll
    for (int c = 0; c < 4; c++) lds_add(r + c, sr[c]);
}

// One tile from prologue to write-out. Ends with a barrier so that the caller may start the next
// tile's prologue on the same LDS.
template <typename R, int NT, int NL>
__device__ __forceinline__ void run_tile(const TileArgs &A, int64_t tile, double *smem) {
    const int tid = threadIdx.x;
    // Throughput plan: the prologue runs at raised wave priority, so that its gathers issue ahead of
    // the element code of the CU's other workgroup and the tile starts sooner (128^3: -4 %). The
    // one-wavefront tiles of the deterministic plan, eight per CU, lose with it.
    if constexpr (NT > 64) __builtin_amdgcn_s_setprio(2);
    // The node ids sit at a fixed stride per tile (padded with a node of the tile), so the first
    // kSpec passes of node gathers need no tile header: they are issued first and wait for one round
    // trip (ids, then coordinates and velocities) while the header loads are in flight; only their
    // LDS stores depend on the tile's node count. Two passes: they cover the throughput plan's tiles
    // (about 440 nodes at 128^3), and in the one-wavefront 128-block tiles (about 115 nodes) two
    // measured faster than three or four (128^3 FP64 1.527 / 1.537 / 1.544 ms).
    constexpr int kSpec = 2;
    const int32_t *nid = A.tile_npad + tile * A.cap_nodes;
    int64_t gs[kSpec];
#pragma unroll
    for (int q = 0; q < kSpec; q++) gs[q] = tid + q * NT < A.cap_nodes ? nid[tid + q * NT] : 0;
    double4 cs[kSpec];
    double us[kSpec][3];
#pragma unroll
    for (int q = 0; q < kSpec; q++) {
        cs[q] = A.coord[gs[q]];
        load_vel3(A.vel, A.vel_soa, gs[q], us[q][0], us[q][1], us[q][2]);
    }
    const int r0 = A.tile_row[tile], r1 = A.tile_row[tile + 1], nrows = r1 - r0;
    const int64_t b0 = A.tile_b0[tile];
    const int nblk = (int)(A.tile_b0[tile + 1] - b0);
    const int nnod = (int)(A.tile_nptr[tile + 1] - A.tile_nptr[tile]);
    // block image at a padded stride (a block's 16 values sit at immediate offsets from one base and
    // neighbouring slots start on different banks), RHS rows, node table
    double *acc = smem;
    double *racc = smem + lds_racc_off(nblk);
    double *nodes = smem + lds_nodes_off(nblk, nrows);
    const int64_t p0 = A.tile_rptr[tile], p1 = A.tile_rptr[tile + 1];
    // issue the first run record and the node gathers before the LDS clears and the barrier
    int64_t p = p0 + tid;
    uint4 h = make_uint4(0u, 0u, 0u, 0u), kk = h;
    if (p < p1) {
        h = load_stream(A.runs + 2 * p);
        kk = load_stream(A.runs + 2 * p + 1);
    }
#pragma unroll
    for (int q = 0; q < kSpec; q++) {
        const int i = tid + q * NT;
        if (i < nnod) {
            double2 *nd = reinterpret_cast<double2 *>(nodes + 6 * i);
            nd[0] = make_double2(cs[q].x, cs[q].y);
            nd[1] = make_double2(cs[q].z, us[q][0]);
            nd[2] = make_double2(us[q][1], us[q][2]);
        }
    }
    for (int i = tid + kSpec * NT; i < nnod; i += NT) {
        const int64_t gnode = nid[i];
        const double4 c = A.coord[gnode];
        double v[3];
        load_vel3(A.vel, A.vel_soa, gnode, v[0], v[1], v[2]);
        double2 *nd = reinterpret_cast<double2 *>(nodes + 6 * i);
        nd[0] = make_double2(c.x, c.y);
        nd[1] = make_double2(c.z, v[0]);
        nd[2] = make_double2(v[1], v[2]);
    }
    {
        double2 *a2 = reinterpret_cast<double2 *>(acc);
        const int n2 = (kBlkStride * nblk + 1) >> 1;
        for (int i = tid; i < n2; i += NT) a2[i] = make_double2(0.0, 0.0);
    }
    for (int i = tid; i < kRhsStride * nrows; i += NT) racc[i] = 0.0;
    __syncthreads();
    if constexpr (NT > 64) __builtin_amdgcn_s_setprio(0);
    // one run per lane (a tile with more runs than lanes takes several rounds)
    const double rdt = A.rho / A.dt;
    while (p < p1) {
        tile_run<R, NL>(A, rdt, h, kk, acc, racc, nodes);
        p += NT;
        if (p < p1) {
            h = load_stream(A.runs + 2 * p);
            kk = load_stream(A.runs + 2 * p + 1);
        }
    }
    __syncthreads();
    // write the image out: block k, value pair j -> values[(b0 + k) * 16 + 2j]
    double2 *out = reinterpret_cast<double2 *>(A.values + 16 * b0);
    for (int i = tid; i < 8 * nblk; i += NT) {
        const int k = i >> 3, j = i & 7;
        const double *src = acc + kBlkStride * k + 2 * j;
        double2 v = make_double2(src[0], src[1]);
        if (A.accumulate) {
            const double2 o = out[i];
            v.x += o.x;
            v.y += o.y;
        }
        store_stream(out + i, v);
    }
    double *rout = A.rhs + 4 * (int64_t)r0;
    for (int i = tid; i < 4 * nrows; i += NT) {
        const int r = i >> 2, c = i & 3;
        double v = racc[kRhsStride * r + c];
        if (A.accumulate) v += rout[i];
        rout[i] = v;
    }
    __syncthreads();
}

template <typename R, int NT>
__global__ __launch_bounds__(NT, 2) void k_tiled(TileArgs A) {
    extern __shared__ double smem[];
    // XCD-aware order (xcd_item): runs of consecutive tiles per XCD, drawn from the whole mesh
    const int64_t tile = xcd_item(blockIdx.x);
    if (tile >= A.ntiles) return;
    // FP64 reads all four nodes per element: 238 registers and no spills, where keeping the shared
    // nodes in registers spilled 5 and was 1.5 % slower at 128^3 (reading ahead spills 11). The batched
    // FP64 kernel reads the same way, so a mesh's deterministic result is the same bits alone and batched.
    constexpr bool f64 = std::is_same<R, double>::value;
    run_tile<R, NT, f64 ? NL_ALL : NL_AHEAD>(A, tile, smem);
}

// Batched form: one launch over the tiles of many meshes. work[t] = (mesh, tile of that mesh) with
// each mesh's tiles contiguous; desc[mesh] holds that mesh's arrays, outputs and parameters. XCD-aware
// (workgroup w runs on XCD w % 8). Two grids: one workgroup per work item, in the order of k_tiled
// (xcd_item), or (PERSIST) a persistent grid whose workgroups walk every (G/8)-th item of their
// XCD's contiguous eighth [x*per, (x+1)*per) of the work table. The persistent loop
// keeps more of the tile body's state live (the FP64 form spills more), so which is faster depends on
// the batch; the autotuner times both.
// A member's arguments as wavefront-uniform values: every lane loads the same words, and
// readfirstlane keeps them in scalar registers for the whole tile (a plain copy would hold them in
// vector registers, which the FP64 element code needs).
__device__ __forceinline__ TileArgs uniform_args(const TileArgs *p) {
    static_assert(sizeof(TileArgs) % 4 == 0, "TileArgs is a whole number of words");
    constexpr int kWords = (int)(sizeof(TileArgs) / 4);
    const uint32_t *src = reinterpret_cast<const uint32_t *>(p);
    uint32_t w[kWords];
#pragma unroll
    for (int i = 0; i < kWords; i++) w[i] = __builtin_amdgcn_readfirstlane(src[i]);
    TileArgs a;
    __builtin_memcpy(&a, w, sizeof a);
    return a;
}

template <typename R, int NT, bool PERSIST>
__global__ __launch_bounds__(NT, 2) void k_tiled_batch(const TileArgs *__restrict__ desc, const int2 *__restrict__ work,
                                                      int64_t total) {
    extern __shared__ double smem[];
    // the batched FP64 form keeps a member's arguments live as well: node data are re-read per element
    constexpr int kBatchNL = std::is_same<R, double>::value ? NL_ALL : NL_AHEAD;
    if (PERSIST) {
        const int64_t per = (total + 7) / 8;
        const int64_t lo = (int64_t)(blockIdx.x & 7) * per;
        const int64_t nslot = gridDim.x >> 3;
        const int64_t hi = lo + per < total ? lo + per : total;
        for (int64_t t = lo + (blockIdx.x >> 3); t < hi; t += nslot) {
            const int2 w =
                make_int2(__builtin_amdgcn_readfirstlane(work[t].x), __builtin_amdgcn_readfirstlane(work[t].y));
            const TileArgs A = uniform_args(desc + w.x);
            run_tile<R, NT, kBatchNL>(A, w.y, smem);
        }
    } else {
        const int64_t t = xcd_item(blockIdx.x);
        if (t >= total) return;
        const int2 w = make_int2(__builtin_amdgcn_readfirstlane(work[t].x), __builtin_amdgcn_readfirstlane(work[t].y));
        const TileArgs A = uniform_args(desc + w.x);
        run_tile<R, NT, kBatchNL>(A, w.y, smem);
    }
}

// ================================================================================================
// err_out report of nsa_assemble: each sampled element evaluated with the tiled kernel's per-row code
// (row0_setup, block0) in FP64 and, for the mixed form, in the mixed precision as well; every vertex in
// turn is the local vertex 0 (the others in cyclic order; the geometry does not depend on the vertex
// order). Per class the largest difference and the largest FP64 magnitude go into err[0..5] and
// err[6..11] with atomic maxima on the bit patterns (non-negative doubles order as their bits).
// ================================================================================================

__device__ __forceinline__ void atomic_max_nonneg(double *p, double v) {
    atomicMax(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ int err_class(int i) {  // entry i of a 4x4 block: uu, up, pu or pp
    const int r = i >> 2, c = i & 3;
    return r < 3 ? (c < 3 ? 0 : 1) : (c < 3 ? 2 : 3);
}

template <bool MIXED>
__global__ __launch_bounds__(256) void k_err_sample(const int4 *__restrict__ samp, int ns,
                                                    const double4 *__restrict__ coord, const double *__restrict__ vel,
                                                    int64_t vel_soa, double rho, double mu, double rdt, double *err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double md[6], mr[6];
#pragma unroll
    for (int k = 0; k < 6; k++) md[k] = mr[k] = 0.0;
    if (i < ns) {
        const int4 e = samp[i];
        const int n[4] = {e.x, e.y, e.z, e.w};
        double X[4][3], U[4][3];
#pragma unroll
        for (int a = 0; a < 4; a++) {
            const double4 c = coord[n[a]];
            X[a][0] = c.x;
            X[a][1] = c.y;
            X[a][2] = c.z;
            load_vel3(vel, vel_soa, n[a], U[a][0], U[a][1], U[a][2]);
        }
        for (int a = 0; a < 4; a++) {
            double Xa[4][3], Ua[4][3];
#pragma unroll
            for (int k = 0; k < 4; k++)
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    Xa[k][d] = X[(a + k) & 3][d];
                    Ua[k][d] = U[(a + k) & 3][d];
                }
            Geo2 g;
            geometry2(Xa, g);
            Row0<double> C;
            double rb[4];
            row0_setup<double>(g, Ua, rho, mu, rdt, C, rb);
            Row0<float> Cf;
            float rbf[4];
            if (MIXED) row0_setup<float>(g, Ua, rho, mu, rdt, Cf, rbf);
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const int k = c < 3 ? 4 : 5;
                mr[k] = fmax(mr[k], fabs(rb[c]));
                if (MIXED) md[k] = fmax(md[k], fabs((double)rbf[c] - rb[c]));
            }
            for (int b = 0; b < 4; b++) {
                double v[16], vf[16];
                block0<double, true>(C, b, v);
                if (MIXED) block0<float, true>(Cf, b, vf);
#pragma unroll
                for (int j = 0; j < 16; j++) {
                    const int k = err_class(j);
                    mr[k] = fmax(mr[k], fabs(v[j]));
                    if (MIXED) md[k] = fmax(md[k], fabs(vf[j] - v[j]));
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 6; k++)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            md[k] = fmax(md[k], __shfl_xor(md[k], o));
            mr[k] = fmax(mr[k], __shfl_xor(mr[k], o));
        }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 6; k++) {
            atomic_max_nonneg(err + k, md[k]);
            atomic_max_nonneg(err + 6 + k, mr[k]);
        }
    }
}

// ================================================================================================
// Explicit residual (the outputs of Listing 2 instead of a matrix): per owned row of an element,
// the momentum residual RHS - sum_b A_uu(a, b) U_b (pressure zero), and the tau- and rho-weighted
// lumped masses tau1 V/4 and rho V/4. The advection field and the previous-step velocity are the
// same nodal field, so the RHS equals the transient parts of A_uu applied to U exactly:
//   (rho/dt) int u N_a = sum_b (rho/dt) M_ab U_b   and   tau1 rho (rho/dt) int (a.grad N_a) u =
//   sum_b tau1 rho (rho/dt) int (a.grad N_a) N_b U_b.
// The residual is therefore formed directly as minus the spatial part applied to U,
//   r_a = -sum_b [ (rho V/20 (s_b + d[a][b]) + tau1 rho^2 V/20 (s_a s_b + gram_ab) + mu V K_ab) U_b
//                  + mu V G_b (G_a . U_b) + tau2 V G_a (G_b . U_b) ],
// the same value without the cancellation of the two large transient terms (which costs the mixed
// form its accuracy). An (element, owned row) pair adds five values into the tile's LDS
// accumulators instead of 68.
// ================================================================================================

// Precomputed geometry (CACHED): an element's stored values v (its own vertex order) in the record's
// vertex order, perm bits 2a..2a+1 = the element vertex at local vertex a.
struct GeoRaw {
    double v[kGeoDoubles];
};

__device__ __forceinline__ void geo_load(const ResArgs &A, uint32_t elem, GeoRaw &r) {
    const double2 *src = reinterpret_cast<const double2 *>(A.geo + (int64_t)kGeoDoubles * elem);
#pragma unroll
    for (int i = 0; i < kGeoDoubles / 2; i++) {
        const double2 q = src[i];
        r.v[2 * i] = q.x;
        r.v[2 * i + 1] = q.y;
    }
}

__device__ __forceinline__ void cached_geometry(const GeoRaw &r, uint32_t perm, Geo2 &g) {
    const double *v = r.v;
#pragma unroll
    for (int a = 0; a < 4; a++) {
        const int e = (int)((perm >> (2 * a)) & 3u);
        // select instead of indexing v with a run-time index (which would put v in scratch memory)
#pragma unroll
        for (int d = 0; d < 3; d++)
            g.G[a][d] = e == 0 ? v[d] : e == 1 ? v[3 + d] : e == 2 ? v[6 + d] : v[9 + d];
    }
    g.V = v[12];
    g.h = v[13];
    g.rh = v[14];
}

template <typename R, bool CACHED>
__device__ __forceinline__ void residual_element(const ResArgs &A, uint2 w, const GeoRaw &gr, uint32_t perm, int nrows,
                                                 const double *nodes, double *racc) {
    const int loc[4] = {(int)(w.x & 0xffffu), (int)(w.x >> 16), (int)(w.y & 0xffffu), (int)(w.y >> 16)};
    int nown = 0;
#pragma unroll
    for (int a = 0; a < 4; a++) nown += loc[a] < nrows;
    double X[4][3], U[4][3];
#pragma unroll
    for (int a = 0; a < 4; a++) {
        const double2 *nd = reinterpret_cast<const double2 *>(nodes + 6 * loc[a]);
        const double2 q0 = nd[0], q1 = nd[1], q2 = nd[2];
        X[a][0] = q0.x;
        X[a][1] = q0.y;
        X[a][2] = q1.x;
        U[a][0] = q1.y;
        U[a][1] = q2.x;
        U[a][2] = q2.y;
    }
    Geo2 g;
    if (CACHED)
        cached_geometry(gr, perm, g);
    else
        geometry2(X, g);
    ElemT<R> E;
    setup_t<R>(g, U, A.rho, A.mu, A.dt, E);
    const R mt = E.t1V * (R)0.25, mr = E.rho * E.v4;
#pragma unroll
    for (int a = 0; a < 4; a++) {
        if (a >= nown) break;
        const R ga[3] = {E.G[a][0], E.G[a][1], E.G[a][2]};
        const R sa = E.s[a];
        const R ksb = E.c1 + E.c2 * sa;
        R r[3] = {(R)0, (R)0, (R)0};
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const R gb[3] = {E.G[b][0], E.G[b][1], E.G[b][2]};
            const R K = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
            const R gram = E.d[0][a] * E.d[0][b] + E.d[1][a] * E.d[1][b] + E.d[2][a] * E.d[2][b] + E.d[3][a] * E.d[3][b];
            const R Tsp = ksb * E.s[b] + E.c1 * E.d[a][b] + E.c2 * gram + E.muV * K;
            const R gaU = ga[0] * E.U[b][0] + ga[1] * E.U[b][1] + ga[2] * E.U[b][2];
            const R gbU = gb[0] * E.U[b][0] + gb[1] * E.U[b][1] + gb[2] * E.U[b][2];
#pragma unroll
            for (int c = 0; c < 3; c++) r[c] -= Tsp * E.U[b][c] + E.muV * gb[c] * gaU + E.t2V * ga[c] * gbU;
        }
        double *q = racc + kResStride * loc[a];
#pragma unroll
        for (int c = 0; c < 3; c++) lds_add(q + c, (double)r[c]);
        lds_add(q + 3, (double)mt);
        lds_add(q + 4, (double)mr);
    }
}

template <typename R, int NT, bool CACHED>
__global__ __launch_bounds__(NT, 2) void k_residual(ResArgs A) {
    extern __shared__ double smem[];
    const int64_t tile = xcd_item(blockIdx.x);  // XCD-aware order as in k_tiled
    if (tile >= A.ntiles) return;
    const int tid = threadIdx.x;
    const int r0 = A.tile_row[tile], nrows = A.tile_row[tile + 1] - r0;
    const int64_t n0 = A.tile_nptr[tile];
    const int nnod = (int)(A.tile_nptr[tile + 1] - n0);
    double *nodes = smem;
    double *racc = smem + 6 * (int64_t)nnod;
    const int64_t p0 = A.tile_eptr[tile], p1 = A.tile_eptr[tile + 1];
    int64_t p = p0 + tid;
    uint2 cur = make_uint2(0u, 0u);
    if (p < p1) cur = load_stream2(A.rec + p);
    // CACHED: the geometry of the next record is loaded while the current one is integrated, and the
    // element id of the one after it an iteration earlier still, so no load waits on another in the loop
    GeoRaw gc, gn;
    uint2 ec = make_uint2(0u, 0u), en = ec;
    if (CACHED) {
        if (p < p1) {
            ec = A.rgel[p];
            geo_load(A, ec.x, gc);
        }
        if (p + NT < p1) en = A.rgel[p + NT];
    }
    // node gathers four passes at a time: the ids, then the node data, then the LDS stores, so the
    // passes wait for one round trip together
    for (int i0 = tid; i0 < nnod; i0 += 4 * NT) {
        int64_t g[4];
#pragma unroll
        for (int u = 0; u < 4; u++) g[u] = A.tile_nodes[n0 + min(i0 + u * NT, nnod - 1)];
        double4 c[4];
        double v[4][3];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            c[u] = A.coord[g[u]];
            load_vel3(A.vel, A.vel_soa, g[u], v[u][0], v[u][1], v[u][2]);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            if (i0 + u * NT < nnod) {
                double2 *nd = reinterpret_cast<double2 *>(nodes + 6 * (i0 + u * NT));
                nd[0] = make_double2(c[u].x, c[u].y);
                nd[1] = make_double2(c[u].z, v[u][0]);
                nd[2] = make_double2(v[u][1], v[u][2]);
            }
        }
    }
    for (int i = tid; i < kResStride * nrows; i += NT) racc[i] = 0.0;
    __syncthreads();
    while (p < p1) {
        const int64_t pn = p + NT;
        uint2 nxt = make_uint2(0u, 0u);
        if (pn < p1) nxt = load_stream2(A.rec + pn);
        uint2 en2 = make_uint2(0u, 0u);
        if (CACHED) {
            if (pn < p1) geo_load(A, en.x, gn);
            if (pn + NT < p1) en2 = A.rgel[pn + NT];
        }
        residual_element<R, CACHED>(A, cur, gc, ec.y, nrows, nodes, racc);
        cur = nxt;
        p = pn;
        if (CACHED) {
            gc = gn;
            ec = en;
            en = en2;
        }
    }
    __syncthreads();
    for (int i = tid; i < 3 * nrows; i += NT) {
        const int r = i / 3, c = i - 3 * r;
        double v = racc[kResStride * r + c];
        double *o = A.rhsid + 3 * (int64_t)r0 + i;
        if (A.accumulate) v += *o;
        store_stream(o, v);
    }
    for (int i = tid; i < nrows; i += NT) {
        double t = racc[kResStride * i + 3], m = racc[kResStride * i + 4];
        if (A.accumulate) {
            t += A.dt_rho[r0 + i];
            m += A.mass_rho[r0 + i];
        }
        store_stream(A.dt_rho + r0 + i, t);
        store_stream(A.mass_rho + r0 + i, m);
    }
}

}  // namespace

// Raise a kernel's dynamic-LDS limit once (not at every launch, so launches can be captured).
hipError_t ensure_lds(const void *kern, size_t bytes) {
    static std::mutex mu;
    static std::map<const void *, size_t> done;
    std::lock_guard<std::mutex> g(mu);
    size_t &have = done[kern];
    if (have >= bytes) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) have = bytes;
    return e;
}

hipError_t launch_tiled(TileKern k, const TileArgs &a, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    const size_t lds = (size_t)a.lds_bytes;
    const int nt = (a.threads == 64 || a.threads == 128 || a.threads == 192) ? a.threads : 256;
    const dim3 grid((unsigned)xcd_grid(a.ntiles)), block(nt);
    auto go = [&](auto kern) -> hipError_t {
        hipError_t e = ensure_lds(reinterpret_cast<const void *>(kern), lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, grid, block, lds, s, a);
        return hipGetLastError();
    };
    const bool mixed = k == TileKern::Mixed;
    if (nt == 64) return mixed ? go(k_tiled<float, 64>) : go(k_tiled<double, 64>);
    if (nt == 128) return mixed ? go(k_tiled<float, 128>) : go(k_tiled<double, 128>);
    if (nt == 192) return mixed ? go(k_tiled<float, 192>) : go(k_tiled<double, 192>);
    return mixed ? go(k_tiled<float, 256>) : go(k_tiled<double, 256>);
}

hipError_t launch_err_sample(const int4 *samp, int ns, const double4 *coord, const double *vel, int64_t vel_soa,
                             double rho, double mu, double rdt, bool mixed, double *err, hipStream_t s) {
    if (ns <= 0) return hipSuccess;
    const dim3 grid((unsigned)((ns + 255) / 256)), block(256);
    if (mixed)
        hipLaunchKernelGGL(k_err_sample<true>, grid, block, 0, s, samp, ns, coord, vel, vel_soa, rho, mu, rdt, err);
    else
        hipLaunchKernelGGL(k_err_sample<false>, grid, block, 0, s, samp, ns, coord, vel, vel_soa, rho, mu, rdt, err);
    return hipGetLastError();
}

hipError_t launch_residual(TileKern k, const ResArgs &a, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    const size_t lds = (size_t)a.lds_bytes;
    const dim3 grid((unsigned)xcd_grid(a.ntiles)), block(256);
    auto go = [&](auto kern) -> hipError_t {
        hipError_t e = ensure_lds(reinterpret_cast<const void *>(kern), lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, grid, block, lds, s, a);
        return hipGetLastError();
    };
    if (a.geo) return k == TileKern::Mixed ? go(k_residual<float, 256, true>) : go(k_residual<double, 256, true>);
    return k == TileKern::Mixed ? go(k_residual<float, 256, false>) : go(k_residual<double, 256, false>);
}

hipError_t prepare_batch(int threads, size_t lds) {
    hipError_t e = hipSuccess;
    for (const void *k : {reinterpret_cast<const void *>(k_tiled_batch<double, 64, false>),
                          reinterpret_cast<const void *>(k_tiled_batch<float, 64, false>),
                          reinterpret_cast<const void *>(k_tiled_batch<double, 128, false>),
                          reinterpret_cast<const void *>(k_tiled_batch<float, 128, false>),
                          reinterpret_cast<const void *>(k_tiled_batch<double, 192, false>),
                          reinterpret_cast<const void *>(k_tiled_batch<float, 192, false>),
                          reinterpret_cast<const void *>(k_tiled_batch<double, 192, true>),
                          reinterpret_cast<const void *>(k_tiled_batch<float, 192, true>),
                          reinterpret_cast<const void *>(k_tiled_batch<double, 256, false>),
                          reinterpret_cast<const void *>(k_tiled_batch<float, 256, false>),
                          reinterpret_cast<const void *>(k_tiled_batch<double, 64, true>),
                          reinterpret_cast<const void *>(k_tiled_batch<float, 64, true>),
                          reinterpret_cast<const void *>(k_tiled_batch<double, 128, true>),
                          reinterpret_cast<const void *>(k_tiled_batch<float, 128, true>),
                          reinterpret_cast<const void *>(k_tiled_batch<double, 256, true>),
                          reinterpret_cast<const void *>(k_tiled_batch<float, 256, true>)})
        if (e == hipSuccess) e = ensure_lds(k, lds);
    (void)threads;
    return e;
}

hipError_t launch_tiled_batch(TileKern k, const TileArgs *desc, const int2 *work, int64_t total, int threads,
                              int64_t lds, int grid_wgs, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    const int nt = (threads == 64 || threads == 128 || threads == 192) ? threads : 256;
    const int64_t items = 8 * ((total + 7) / 8);
    const bool persist = grid_wgs > 0 && grid_wgs < items;
    const dim3 grid((unsigned)(persist ? std::max(8, grid_wgs & ~7) : xcd_grid(total))), block(nt);
    const bool mixed = k == TileKern::Mixed;
#define NSA_LAUNCH_BATCH(T, N, P) \
    hipLaunchKernelGGL((k_tiled_batch<T, N, P>), grid, block, (size_t)lds, s, desc, work, total)
#define NSA_LAUNCH_BATCH_NT(P)                                                                  \
    if (nt == 64) {                                                                             \
        if (mixed) NSA_LAUNCH_BATCH(float, 64, P); else NSA_LAUNCH_BATCH(double, 64, P);       \
    } else if (nt == 128) {                                                                     \
        if (mixed) NSA_LAUNCH_BATCH(float, 128, P); else NSA_LAUNCH_BATCH(double, 128, P);     \
    } else if (nt == 192) {                                                                     \
        if (mixed) NSA_LAUNCH_BATCH(float, 192, P); else NSA_LAUNCH_BATCH(double, 192, P);     \
    } else {                                                                                    \
        if (mixed) NSA_LAUNCH_BATCH(float, 256, P); else NSA_LAUNCH_BATCH(double, 256, P);     \
    }
    if (persist) {
        NSA_LAUNCH_BATCH_NT(true)
    } else {
        NSA_LAUNCH_BATCH_NT(false)
    }
#undef NSA_LAUNCH_BATCH_NT
#undef NSA_LAUNCH_BATCH
    return hipGetLastError();
}

}  // namespace nsa
