// HIP kernel for gfx950: the 2-D element family -- bilinear quadrilaterals (four nodes, two space
// dimensions, dofs u v p, 3x3 blocks) -- assembled into a block-CSR matrix plus RHS (the element loop of
// the paper's Listing 1 for Table 2's two 2-D benchmarks).
//
// The Jacobian of a bilinear map varies over the element, so unlike the tetrahedra there are no closed
// forms: every term is integrated with the 2x2 Gauss-Legendre rule, point by point, as in Listing 1's
// PGAUS loops. Geometry (Jacobian, determinant, inverse, Cartesian derivatives, area and length) is
// FP64; the integration runs in the template type R (double, or float in the mixed form); every block
// entry is converted to FP64 before it is added into the tile image.
//
// Layout and scatter follow the tetrahedral row-tiled kernel: one workgroup owns a tile of contiguous
// block rows, stages its nodes (x, y, u, v) in LDS, adds the contributions of its owned rows into an
// FP64 LDS image of its blocks with ds_add_f64 and writes the image to HBM once, coalesced. One lane
// takes one (element, tile) record and integrates the element's owned rows; the throughput plan runs
// a tile on two wavefronts, the deterministic plan on one wavefront, whose LDS adds come in program order.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <type_traits>

#include "nsa_device.h"
#include "nsa_internal.h"

namespace nsa {
namespace {

__device__ __forceinline__ void lds_add_q1(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// slot of block (a, b) of a record: 16-bit field 4a + b of the slot words (words 3 .. 10 of the record)
__device__ __forceinline__ int q1_slot(const uint4 r0, const uint4 r1, const uint4 r2, int i) {
    const int w = 3 + (i >> 1);
    const uint32_t word = w == 3 ? r0.w : w == 4 ? r1.x : w == 5 ? r1.y : w == 6 ? r1.z : w == 7 ? r1.w
                                                  : w == 8 ? r2.x : w == 9 ? r2.y : r2.z;
    return (int)((word >> (16 * (i & 1))) & 0xffffu);
}

template <typename R>
__device__ __forceinline__ void q1_element(const Q1Args &A, double rdt_d, const uint4 r0, const uint4 r1,
                                           const uint4 r2, const double *nodes, double *acc, double *racc) {
    const int loc[4] = {(int)(r0.x & 0xffffu), (int)(r0.x >> 16), (int)(r0.y & 0xffffu), (int)(r0.y >> 16)};
    const uint32_t own = r0.z & 0xfu;
    double X[4][2];
    R U[4][2];
#pragma unroll
    for (int a = 0; a < 4; a++) {
        const double2 *nd = reinterpret_cast<const double2 *>(nodes + 4 * loc[a]);
        const double2 q0 = nd[0], q1 = nd[1];
        X[a][0] = q0.x;
        X[a][1] = q0.y;
        U[a][0] = (R)q1.x;
        U[a][1] = (R)q1.y;
    }
    // reference vertices (counter-clockwise) and the 2x2 Gauss-Legendre points, weights 1
    constexpr double XI[4] = {-1.0, 1.0, 1.0, -1.0}, ETA[4] = {-1.0, -1.0, 1.0, 1.0};
    constexpr double GP = 0.57735026918962576451;  // 1/sqrt(3)
    R G[4][4][2];  // G[g][a][d] = d N_a / d x_d at Gauss point g
    R N[4][4];     // N[g][a]
    R w[4];        // |det J(g)|
    double area = 0.0;
#pragma unroll
    for (int g = 0; g < 4; g++) {
        const double xi = (g & 1) ? GP : -GP, eta = (g & 2) ? GP : -GP;
        double dx[4], de[4];
#pragma unroll
        for (int a = 0; a < 4; a++) {
            N[g][a] = (R)(0.25 * (1.0 + XI[a] * xi) * (1.0 + ETA[a] * eta));
            dx[a] = 0.25 * XI[a] * (1.0 + ETA[a] * eta);
            de[a] = 0.25 * ETA[a] * (1.0 + XI[a] * xi);
        }
        double J00 = 0.0, J01 = 0.0, J10 = 0.0, J11 = 0.0;  // J[r][s] = d x_r / d xi_s
#pragma unroll
        for (int a = 0; a < 4; a++) {
            J00 = fma(X[a][0], dx[a], J00);
            J01 = fma(X[a][0], de[a], J01);
            J10 = fma(X[a][1], dx[a], J10);
            J11 = fma(X[a][1], de[a], J11);
        }
        const double det = J00 * J11 - J01 * J10;
        const double inv = fast_rcp(det);
#pragma unroll
        for (int a = 0; a < 4; a++) {
            G[g][a][0] = (R)((dx[a] * J11 - de[a] * J10) * inv);
            G[g][a][1] = (R)((de[a] * J00 - dx[a] * J01) * inv);
        }
        w[g] = (R)fabs(det);
        area += fabs(det);
    }
    // h = area^(1/2) and 1/h from one reciprocal square root: the hardware estimate (about 23 correct
    // bits) and one Newton step r (3 - area r^2) / 2 (relative error about 1.5 * 2^-46); the area of a
    // valid element is positive and far inside the estimate's range
    double rhd = __builtin_amdgcn_rsq(area);
    rhd = rhd * fma(-0.5 * area, rhd * rhd, 1.5);
    const R h = (R)(area * rhd), rh = (R)rhd, rho = (R)A.rho, mu = (R)A.mu, rdt = (R)rdt_d;
    R ab[2] = {(R)0.25 * (U[0][0] + U[1][0] + U[2][0] + U[3][0]), (R)0.25 * (U[0][1] + U[1][1] + U[2][1] + U[3][1])};
    const R an = tau_norm(ab[0] * ab[0] + ab[1] * ab[1]);
    const R t1 = fast_rcp(rdt + (R)4 * mu * rh * rh + (R)2 * rho * an * rh);
    const R t2 = mu + (R)0.5 * rho * an * h;
    R ug[4][2], ag[4][4];  // velocity at g, a_g . grad N_a
#pragma unroll
    for (int g = 0; g < 4; g++) {
#pragma unroll
        for (int c = 0; c < 2; c++)
            ug[g][c] = N[g][0] * U[0][c] + N[g][1] * U[1][c] + N[g][2] * U[2][c] + N[g][3] * U[3][c];
#pragma unroll
        for (int a = 0; a < 4; a++) ag[g][a] = ug[g][0] * G[g][a][0] + ug[g][1] * G[g][a][1];
    }
    const R t1r = t1 * rho;
#pragma unroll
    for (int a = 0; a < 4; a++) {
        if (!((own >> a) & 1u)) continue;
        // RHS row a
        R rb[3] = {(R)0, (R)0, (R)0};
#pragma unroll
        for (int g = 0; g < 4; g++) {
            const R wa = w[g] * rdt;
#pragma unroll
            for (int c = 0; c < 2; c++) rb[c] += wa * ug[g][c] * (N[g][a] + t1r * ag[g][a]);
            rb[2] += wa * t1 * (G[g][a][0] * ug[g][0] + G[g][a][1] * ug[g][1]);
        }
        double *rr = racc + 3 * loc[a];
#pragma unroll
        for (int c = 0; c < 3; c++) lds_add_q1(rr + c, (double)rb[c]);
#pragma unroll
        for (int b = 0; b < 4; b++) {
            R T = 0, V00 = 0, V01 = 0, V10 = 0, V11 = 0, up0 = 0, up1 = 0, pu0 = 0, pu1 = 0, pp = 0;
#pragma unroll
            for (int g = 0; g < 4; g++) {
                const R wg = w[g], Na = N[g][a], Nb = N[g][b], aga = ag[g][a], agb = ag[g][b];
                const R ga0 = G[g][a][0], ga1 = G[g][a][1], gb0 = G[g][b][0], gb1 = G[g][b][1];
                const R K = ga0 * gb0 + ga1 * gb1;
                T += wg * (rdt * Na * Nb + rho * Na * agb + t1r * aga * (rho * agb + rdt * Nb) + mu * K);
                const R wm = wg * mu, wt = wg * t2;
                V00 += wm * ga0 * gb0 + wt * ga0 * gb0;
                V01 += wm * ga1 * gb0 + wt * ga0 * gb1;
                V10 += wm * ga0 * gb1 + wt * ga1 * gb0;
                V11 += wm * ga1 * gb1 + wt * ga1 * gb1;
                const R su = t1r * aga;
                up0 += wg * (su * gb0 - Nb * ga0);
                up1 += wg * (su * gb1 - Nb * ga1);
                const R sp = t1 * (rdt * Nb + rho * agb);
                pu0 += wg * (Na * gb0 + sp * ga0);
                pu1 += wg * (Na * gb1 + sp * ga1);
                pp += wg * t1 * K;
            }
            double *blk = acc + 9 * q1_slot(r0, r1, r2, 4 * a + b);
            lds_add_q1(blk + 0, (double)(T + V00));
            lds_add_q1(blk + 1, (double)V01);
            lds_add_q1(blk + 2, (double)up0);
            lds_add_q1(blk + 3, (double)V10);
            lds_add_q1(blk + 4, (double)(T + V11));
            lds_add_q1(blk + 5, (double)up1);
            lds_add_q1(blk + 6, (double)pu0);
            lds_add_q1(blk + 7, (double)pu1);
            lds_add_q1(blk + 8, (double)pp);
        }
    }
}

// The FP64 form needs more than the 256 registers of two waves per SIMD (it spilled ~100 of them at that
// bound); it runs one wave per SIMD. The mixed form fits two.
template <typename R>
constexpr int q1_min_blocks() {
    return std::is_same<R, double>::value ? 1 : 2;
}

template <typename R, int NT>
__global__ __launch_bounds__(NT, q1_min_blocks<R>()) void k_q1(Q1Args A) {
    extern __shared__ double smem[];
    const int64_t tile = xcd_item(blockIdx.x);  // XCD-aware order as in the tetrahedral kernel
    if (tile >= A.ntiles) return;
    const int tid = threadIdx.x;
    // throughput plan: the prologue at raised wave priority, as in the tetrahedral kernel (2048^2: -1.7 %)
    if constexpr (NT > 64) __builtin_amdgcn_s_setprio(2);
    const int r0 = A.tile_row[tile], nrows = A.tile_row[tile + 1] - r0;
    const int64_t b0 = A.tile_b0[tile];
    const int nblk = (int)(A.tile_b0[tile + 1] - b0);
    const int64_t n0 = A.tile_nptr[tile];
    const int nnod = (int)(A.tile_nptr[tile + 1] - n0);
    const int64_t p0 = A.tile_eptr[tile], p1 = A.tile_eptr[tile + 1];
    double *acc = smem;
    double *racc = smem + q1_racc_off(nblk);
    double *nodes = smem + q1_nodes_off(nblk, nrows);
    // node gathers two passes at a time: the ids, then the node data, then the LDS stores, so the
    // passes wait for one round trip together
    for (int i0 = tid; i0 < nnod; i0 += 2 * NT) {
        int64_t g[2];
#pragma unroll
        for (int u = 0; u < 2; u++) g[u] = A.tile_nodes[n0 + min(i0 + u * NT, nnod - 1)];
        double2 c[2], v[2];
#pragma unroll
        for (int u = 0; u < 2; u++) {
            c[u] = A.coord[g[u]];
            v[u] = load_vel2(A.vel, A.vel_soa, g[u]);
        }
#pragma unroll
        for (int u = 0; u < 2; u++) {
            if (i0 + u * NT < nnod) {
                double2 *nd = reinterpret_cast<double2 *>(nodes + 4 * (i0 + u * NT));
                nd[0] = c[u];
                nd[1] = v[u];
            }
        }
    }
    for (int i = tid; i < 9 * nblk; i += NT) acc[i] = 0.0;
    for (int i = tid; i < 3 * nrows; i += NT) racc[i] = 0.0;
    __syncthreads();
    if constexpr (NT > 64) __builtin_amdgcn_s_setprio(0);
    const double rdt = A.rho / A.dt;
    for (int64_t p = p0 + tid; p < p1; p += NT) {
        const uint4 *rp = A.recs + 3 * p;
        q1_element<R>(A, rdt, load_stream(rp), load_stream(rp + 1), load_stream(rp + 2), nodes, acc, racc);
    }
    __syncthreads();
    // the tile's 9 nblk values are contiguous: written as 16-byte pairs, with one 8-byte value first
    // when the range starts off 16-byte alignment and one last when a value is left over
    double *out = A.values + 9 * b0;
    const int n = 9 * nblk;
    const int lead = (int)((reinterpret_cast<uintptr_t>(out) >> 3) & 1);
    const int npair = (n - lead) >> 1;
    double2 *out2 = reinterpret_cast<double2 *>(out + lead);
    for (int i = tid; i < npair; i += NT) {
        const double *src = acc + lead + 2 * i;
        double2 v = make_double2(src[0], src[1]);
        if (A.accumulate) {
            const double2 o = out2[i];
            v.x += o.x;
            v.y += o.y;
        }
        store_stream(out2 + i, v);
    }
    if (tid < 2) {
        const int i = tid == 0 ? (lead ? 0 : -1) : (((n - lead) & 1) ? n - 1 : -1);
        if (i >= 0) {
            double v = acc[i];
            if (A.accumulate) v += out[i];
            store_stream(out + i, v);
        }
    }
    double *rout = A.rhs + 3 * (int64_t)r0;
    for (int i = tid; i < 3 * nrows; i += NT) {
        double v = racc[i];
        if (A.accumulate) v += rout[i];
        rout[i] = v;
    }
}

}  // namespace

hipError_t launch_q1(TileKern k, const Q1Args &a, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    const size_t lds = (size_t)a.lds_bytes;
    const dim3 grid((unsigned)xcd_grid(a.ntiles));
    auto go = [&](auto kern, int nt) -> hipError_t {
        hipError_t e = ensure_lds(reinterpret_cast<const void *>(kern), lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, grid, dim3(nt), lds, s, a);
        return hipGetLastError();
    };
    const bool mixed = k == TileKern::Mixed;
    if (a.threads == 64) return mixed ? go(k_q1<float, 64>, 64) : go(k_q1<double, 64>, 64);
    if (a.threads == 128) return mixed ? go(k_q1<float, 128>, 128) : go(k_q1<double, 128>, 128);
    return mixed ? go(k_q1<float, 256>, 256) : go(k_q1<double, 256>, 256);
}

}  // namespace nsa
