// Gather assembly for gfx950: every block of the global matrix is summed in registers by one lane
// and written to HBM once, with no atomics of any kind.
//
// A workgroup owns a tile of contiguous block rows (as the row-tiled kernel does) and runs in two
// phases over LDS:
//   1. per element touching the tile (one lane each): FP64 geometry from the LDS node table, then
//      the element data the blocks are made of, in the integration precision R: for each vertex a,
//      grad N_a, s_a = sum_k d[k][a] and the column d[.][a] (d[k][b] = U_k . grad N_b), plus eleven
//      per-element coefficients (volume and stabilisation factors folded in);
//   2. per owned block (one lane each, in slot order): the sum over its contribution list, element
//      by element in ascending element order, of the element's 4x4 block (a, b), formed from the
//      data of vertices a and b only (~60 operations, see the closed forms of the element body in
//      the other kernel file) and added in FP64 registers; a diagonal block's lane also sums the
//      RHS row. Then the 16 values (and the RHS row) are stored.
// Each block's sum runs in a fixed order, whatever the schedule: results are bit-reproducible and
// independent of the tiling, so one kernel serves both the throughput and the deterministic mode.
#include <hip/hip_runtime.h>

#include "nsa_device.h"
#include "nsa_internal.h"

namespace nsa {
namespace {

template <typename R>
struct GRec;
template <>
struct GRec<float> {
    static constexpr int S = kGatherRecF32;
};
template <>
struct GRec<double> {
    static constexpr int S = kGatherRecF64;
};

// 16-byte vector loads and stores of R data in LDS (4 floats or 2 doubles).
__device__ __forceinline__ void st16(float *p, float a, float b, float c, float d) {
    *reinterpret_cast<float4 *>(p) = make_float4(a, b, c, d);
}
__device__ __forceinline__ void st16(double *p, double a, double b, double c, double d) {
    reinterpret_cast<double2 *>(p)[0] = make_double2(a, b);
    reinterpret_cast<double2 *>(p)[1] = make_double2(c, d);
}
__device__ __forceinline__ void ld16(const float *p, float &a, float &b, float &c, float &d) {
    const float4 v = *reinterpret_cast<const float4 *>(p);
    a = v.x; b = v.y; c = v.z; d = v.w;
}
__device__ __forceinline__ void ld16(const double *p, double &a, double &b, double &c, double &d) {
    const double2 v0 = reinterpret_cast<const double2 *>(p)[0], v1 = reinterpret_cast<const double2 *>(p)[1];
    a = v0.x; b = v0.y; c = v1.x; d = v1.y;
}

// Phase 1 for one record: element data at e (S values of R).
template <typename R>
__device__ __forceinline__ void element_data(const int loc[4], const double *nodes, double rho_d, double mu_d,
                                             double dt_d, R *e) {
    double X[4][3], Ud[4][3];
#pragma unroll
    for (int a = 0; a < 4; a++) {
        const double2 *nd = reinterpret_cast<const double2 *>(nodes + 6 * loc[a]);
        const double2 q0 = nd[0], q1 = nd[1], q2 = nd[2];
        X[a][0] = q0.x;
        X[a][1] = q0.y;
        X[a][2] = q1.x;
        Ud[a][0] = q1.y;
        Ud[a][1] = q2.x;
        Ud[a][2] = q2.y;
    }
    Geo2 g;
    geometry2(X, g);
    R G[4][3], U[4][3];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            G[a][c] = (R)g.G[a][c];
            U[a][c] = (R)Ud[a][c];
        }
    const R V = (R)g.V, h = (R)g.h, rh = (R)g.rh, rho = (R)rho_d, mu = (R)mu_d;
    const R rdt = (R)(rho_d / dt_d);
    R su[3];
#pragma unroll
    for (int c = 0; c < 3; c++) su[c] = U[0][c] + U[1][c] + U[2][c] + U[3][c];
    const R an = (R)0.25 * tau_norm(su[0] * su[0] + su[1] * su[1] + su[2] * su[2]);
    const R t1 = fast_rcp(rdt + (R)4 * mu * rh * rh + (R)2 * rho * an * rh);
    const R t2 = mu + (R)0.5 * rho * an * h;
#pragma unroll
    for (int b = 0; b < 4; b++) {
        R d[4];
#pragma unroll
        for (int k = 0; k < 4; k++) d[k] = U[k][0] * G[b][0] + U[k][1] * G[b][1] + U[k][2] * G[b][2];
        const R sb = d[0] + d[1] + d[2] + d[3];
        st16(e + 8 * b, G[b][0], G[b][1], G[b][2], sb);
        st16(e + 8 * b + 4, d[0], d[1], d[2], d[3]);
    }
    const R v20 = V * (R)0.05, v4 = V * (R)0.25, t1rho = t1 * rho;
    st16(e + 32, rdt * v20, rho * v20, t1rho * rho * v20, t1rho * rdt * v20);  // Mo, c1, c2, c3
    st16(e + 36, mu * V, t2 * V, t1 * V, v4);                                   // muV, t2V, t1V, v4
    st16(e + 40, t1rho * v4, t1 * rdt * v4, t1rho, (R)0);                       // t1rho v4, t1 (rho/dt) v4, t1 rho
}

// Phase 2 for one contribution: element block (a, b) from the element data at e, added into acc.
//   T  = Mo (1 + delta_ab) + c3 s_a + (c1 + c2 s_a) s_b + c1 d[a][b] + c3 d[b][a] + c2 gram + muV K
//   uu = T I + muV G_b G_a^T + t2V G_a G_b^T ; up = -V/4 G_a + tau1 rho V/4 s_a G_b
//   pu = V/4 G_b + G_a (tau1 rho V/4 s_b + tau1 (rho/dt) V/4) ; pp = t1V K
// with K = G_a . G_b and gram = sum_k d[k][a] d[k][b].
template <typename R>
__device__ __forceinline__ void add_block(const R *e, int a, int b, double acc[16], R dA[4], R &sa_out) {
    // d[a][b] sits in vertex b's column at row a, d[b][a] in vertex a's column at row b
    const R dab = e[8 * b + 4 + a], dba = e[8 * a + 4 + b];
    R ga0, ga1, ga2, sa, gb0, gb1, gb2, sb, dB[4];
    ld16(e + 8 * a, ga0, ga1, ga2, sa);
    ld16(e + 8 * a + 4, dA[0], dA[1], dA[2], dA[3]);
    ld16(e + 8 * b, gb0, gb1, gb2, sb);
    ld16(e + 8 * b + 4, dB[0], dB[1], dB[2], dB[3]);
    R Mo, c1, c2, c3, muV, t2V, t1V, v4, trv4, tdv4, t1rho_unused, pad;
    ld16(e + 32, Mo, c1, c2, c3);
    ld16(e + 36, muV, t2V, t1V, v4);
    ld16(e + 40, trv4, tdv4, t1rho_unused, pad);
    (void)t1rho_unused;
    (void)pad;
    const R K = ga0 * gb0 + ga1 * gb1 + ga2 * gb2;
    const R gram = dA[0] * dB[0] + dA[1] * dB[1] + dA[2] * dB[2] + dA[3] * dB[3];
    R T = Mo + c3 * sa + (c1 + c2 * sa) * sb + c1 * dab + c3 * dba + c2 * gram + muV * K;
    if (a == b) T += Mo;
    const R ga[3] = {ga0, ga1, ga2}, gb[3] = {gb0, gb1, gb2};
    const R qa = trv4 * sa, rbb = trv4 * sb + tdv4;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const R gm = muV * gb[c], gt = t2V * ga[c];
#pragma unroll
        for (int cp = 0; cp < 3; cp++) {
            R v = ga[cp] * gm + gt * gb[cp];
            if (c == cp) v += T;
            acc[4 * c + cp] += (double)v;
        }
        acc[4 * c + 3] += (double)(qa * gb[c] - v4 * ga[c]);
        acc[12 + c] += (double)(v4 * gb[c] + rbb * ga[c]);
    }
    acc[15] += (double)(t1V * K);
    sa_out = sa;
}

template <typename R, int NT>
__global__ __launch_bounds__(NT, 512 / NT) void k_gather(GatherArgs A) {
    extern __shared__ double smem[];
    constexpr int S = GRec<R>::S;
    const int64_t per = (A.ntiles + 7) / 8;
    const int64_t tile = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (tile >= A.ntiles) return;
    const int tid = threadIdx.x;
    const int r0 = A.tile_row[tile], r1 = A.tile_row[tile + 1];
    const int64_t b0 = A.bptr[r0];
    const int nblk = (int)(A.bptr[r1] - b0);
    const int64_t n0 = A.tile_nptr[tile];
    const int nnod = (int)(A.tile_nptr[tile + 1] - n0);
    const int64_t e0 = A.tile_eptr[tile];
    const int nrec = (int)(A.tile_eptr[tile + 1] - e0);
    const int64_t q0 = A.tile_pptr[tile];
    const int npair = (int)(A.tile_pptr[tile + 1] - q0);
    constexpr bool f64 = sizeof(R) == 8;
    double *nodes = smem;
    R *elem = reinterpret_cast<R *>(reinterpret_cast<char *>(smem) + gather_elem_off(nnod));
    uint2 *locs = reinterpret_cast<uint2 *>(reinterpret_cast<char *>(smem) + gather_loc_off(nnod, nrec, f64));
    uint16_t *lpairs = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(smem) + gather_pair_off(nnod, nrec, f64));
    for (int i = tid; i < nnod; i += NT) {
        const int64_t gnode = A.tile_nodes[n0 + i];
        const double4 c = A.coord[gnode];
        double v[3];
        load_vel3(A.vel, A.vel_soa, gnode, v[0], v[1], v[2]);
        double2 *nd = reinterpret_cast<double2 *>(nodes + 6 * i);
        nd[0] = make_double2(c.x, c.y);
        nd[1] = make_double2(c.z, v[0]);
        nd[2] = make_double2(v[1], v[2]);
    }
    {
        // the tile's contribution lists, read in phase 2 from LDS
        const uint16_t *src = A.pairs + q0;
        for (int i = tid; i < npair; i += NT) lpairs[i] = src[i];
    }
    // rows without blocks (nodes in no element) still get their RHS row written
    if (!A.accumulate)
        for (int i = tid; i < r1 - r0; i += NT)
            if (A.bptr[r0 + i + 1] == A.bptr[r0 + i])
            {
                double2 *ro = reinterpret_cast<double2 *>(A.rhs + 4 * (int64_t)(r0 + i));
                ro[0] = make_double2(0.0, 0.0);
                ro[1] = make_double2(0.0, 0.0);
            }
    __syncthreads();
    for (int r = tid; r < nrec; r += NT) {
        const uint2 w = A.rec[e0 + r];
        const int loc[4] = {(int)(w.x & 0xffffu), (int)(w.x >> 16), (int)(w.y & 0xffffu), (int)(w.y >> 16)};
        element_data<R>(loc, nodes, A.rho, A.mu, A.dt, elem + (int64_t)r * S);
        locs[r] = w;
    }
    __syncthreads();
    const uint32_t *slot = A.slot + b0;
    double2 *out = reinterpret_cast<double2 *>(A.values + 16 * b0);
    for (int s = tid; s < nblk; s += NT) {
        const uint32_t w = slot[s];
        const int blk = (int)(w >> 16), pb = (int)(w & 0xffffu);
        const int pe = s + 1 < nblk ? (int)(slot[s + 1] & 0xffffu) : npair;
        double acc[16], racc[4];
#pragma unroll
        for (int i = 0; i < 16; i++) acc[i] = 0.0;
#pragma unroll
        for (int i = 0; i < 4; i++) racc[i] = 0.0;
        int row = -1;
        uint32_t nxt = pb < pe ? lpairs[pb] : 0u;
        for (int p = pb; p < pe; p++) {
            const uint32_t pr = nxt;
            if (p + 1 < pe) nxt = lpairs[p + 1];
            const int r = (int)(pr >> 4), a = (int)((pr >> 2) & 3u), b = (int)(pr & 3u);
            const R *e = elem + (int64_t)r * S;
            R dA[4], sa;
            add_block<R>(e, a, b, acc, dA, sa);
            if (a == b) {
                // RHS row of vertex a: (rho/dt) V/20 (su + U_a + tau1 rho (s_a su + sum_k d[k][a] U_k)),
                // and tau1 (rho/dt) V/4 s_a
                const uint2 lw = locs[r];
                const int loc[4] = {(int)(lw.x & 0xffffu), (int)(lw.x >> 16), (int)(lw.y & 0xffffu),
                                    (int)(lw.y >> 16)};
                const int loca = reinterpret_cast<const uint16_t *>(locs + r)[a];
                R U[4][3];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const double *nd = nodes + 6 * loc[k] + 3;
                    U[k][0] = (R)nd[0];
                    U[k][1] = (R)nd[1];
                    U[k][2] = (R)nd[2];
                }
                const R Mo = e[32], tdv4 = e[41], t1rho = e[42];
                const double *nda = nodes + 6 * loca + 3;
                const R ua[3] = {(R)nda[0], (R)nda[1], (R)nda[2]};
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const R su = U[0][c] + U[1][c] + U[2][c] + U[3][c];
                    const R au = sa * su + dA[0] * U[0][c] + dA[1] * U[1][c] + dA[2] * U[2][c] + dA[3] * U[3][c];
                    racc[c] += (double)(Mo * (su + ua[c] + t1rho * au));
                }
                racc[3] += (double)(tdv4 * sa);
                row = r0 + loca;
            }
        }
        double2 *o = out + 8 * (int64_t)blk;
        if (A.accumulate) {
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const double2 v = o[j];
                acc[2 * j] += v.x;
                acc[2 * j + 1] += v.y;
            }
        }
#pragma unroll
        for (int j = 0; j < 8; j++) o[j] = make_double2(acc[2 * j], acc[2 * j + 1]);
        if (row >= 0) {
            double2 *ro = reinterpret_cast<double2 *>(A.rhs + 4 * (int64_t)row);
            if (A.accumulate) {
                const double2 v0 = ro[0], v1 = ro[1];
                racc[0] += v0.x;
                racc[1] += v0.y;
                racc[2] += v1.x;
                racc[3] += v1.y;
            }
            ro[0] = make_double2(racc[0], racc[1]);
            ro[1] = make_double2(racc[2], racc[3]);
        }
    }
}

}  // namespace

hipError_t launch_gather(TileKern k, const GatherArgs &a, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    const size_t lds = (size_t)a.lds_bytes;
    const int64_t per = (a.ntiles + 7) / 8;
    const int nt = a.threads == 512 ? 512 : 256;
    const dim3 grid((unsigned)(8 * per)), block(nt);
    auto go = [&](auto kern) -> hipError_t {
        hipError_t e = ensure_lds(reinterpret_cast<const void *>(kern), lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, grid, block, lds, s, a);
        return hipGetLastError();
    };
    const bool mixed = k == TileKern::Mixed;
    if (nt == 512) return mixed ? go(k_gather<float, 512>) : go(k_gather<double, 512>);
    return mixed ? go(k_gather<float, 256>) : go(k_gather<double, 256>);
}

}  // namespace nsa
