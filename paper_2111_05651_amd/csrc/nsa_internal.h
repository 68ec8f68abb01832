// Internal declarations shared by the host library (nsa_host.cpp) and the HIP kernels
// (nsa_kernels.hip). Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nsa.h"

namespace nsa {

// One device region inside a mesh workspace.
struct Region {
    size_t off = 0, bytes = 0;
};

// Arguments of one direct (element-per-lane) launch. Element data are SoA with leading dimension
// ld: ln[a*ld + e] (a = 0..3) and emap[k*ld + e] (k = 4a+b, 0..15); coordinates are SoA
// coord[d*npoin + node]; the velocity is the caller's AoS vel[3*node + d].
struct AsmArgs {
    int64_t e0 = 0, e1 = 0;      // element range [e0, e1) of the SoA arrays
    int64_t ld = 0;              // leading dimension of ln / emap
    int64_t npoin = 0;
    const int32_t *ln = nullptr;
    const int32_t *emap = nullptr;
    const double *coord = nullptr;
    const double *vel = nullptr;
    int64_t vel_soa = 0;         // 0: vel [npoin][3]; npoin: vel [3][npoin]
    double rho = 1, mu = 0, dt = 1;
    double *values = nullptr;
    double *rhs = nullptr;
};

enum class Kern { AtomicF64, AtomicMixed, ColourF64, ColourMixed };

hipError_t launch_fill_zero(double *p, int64_t n, hipStream_t s);
hipError_t launch_fill_uniform(double *p, int64_t n, uint64_t seed, double lo, double hi, hipStream_t s);
hipError_t launch_assemble(Kern k, const AsmArgs &a, int threads, hipStream_t s);
// err_out report over ns sampled elements (node ids in samp): per class the largest |value - FP64
// value| (0 unless mixed) and the largest |FP64 value| into err[0..5] and err[6..11], which must hold
// zeros or earlier maxima (non-negative) on entry.
hipError_t launch_err_sample(const int4 *samp, int ns, const double4 *coord, const double *vel, int64_t vel_soa,
                             double rho, double mu, double rdt, bool mixed, double *err, hipStream_t s);

// Row tiles: tile t owns the contiguous block rows [row[t], row[t+1]) and therefore the contiguous
// blocks [bptr[r0], bptr[r1]). Its nodes tile_nodes[nptr[t] .. nptr[t+1]) are the owned rows (local
// ids 0 .. nrows-1) followed by every other node its elements touch. Its work is a list of runs
// runs[rptr[t] .. rptr[t+1]): every pair (element, owned row i) of the tile lies in exactly one
// run. A run is a sequence of up to kRunMax elements that all contain the row node i and a second
// node j (the hinge), each sharing a face (i, j, k) with the next one: element q of the run has the
// vertices (i, j, k_old(q), k_new(q)) with k_old(0) = k0 and k_old(q+1) = k_new(q). One lane walks a
// run and integrates only row i of each element, keeping in registers the sums of the diagonal block
// (i, i), the RHS row i, the block (i, j) (every element of the run adds to it) and the block
// (i, k_new(q)) (the next element adds to it again as its (i, k_old)); it adds into the tile's LDS
// image once per element (the finished (i, k_old) block) and once per run for the rest.
// Slots are block indices inside the tile (block bptr[r0] + slot); node fields are local node ids.
constexpr int kRunMax = 4;
struct RunRec {
    uint16_t row, hinge, k0, len;      // local row i (= its local node id), hinge j, k_old(0), elements
    uint16_t diag, jslot, last, pad;   // slots of (i, i), (i, j) and (i, k_new(len-1)); pad = 0
    uint16_t knew[kRunMax];            // k_new(q)
    uint16_t kslot[kRunMax];           // slot of (i, k_old(q))
};
static_assert(sizeof(RunRec) == 32, "run record layout");

struct TileArgs {
    int64_t ntiles = 0;
    int64_t lds_bytes = 0;               // dynamic LDS per workgroup (the largest tile's layout)
    const int32_t *tile_row = nullptr;   // [ntiles+1]
    const int64_t *tile_rptr = nullptr;  // [ntiles+1] run offsets
    const uint4 *runs = nullptr;         // [sum] RunRec as 2 x uint4
    const int64_t *tile_nptr = nullptr;  // [ntiles+1]
    const int32_t *tile_nodes = nullptr; // [sum]
    // the prologue's loads without a dependent round trip: tile_b0[t] = bptr[tile_row[t]] ([ntiles+1])
    // and each tile's node ids at a fixed stride cap_nodes, padded with a node of the tile
    const int64_t *tile_b0 = nullptr;
    const int32_t *tile_npad = nullptr;  // [ntiles * cap_nodes]
    int32_t cap_nodes = 0;
    const int64_t *bptr = nullptr;       // [npoin+1]
    const double4 *coord = nullptr;      // [npoin] (x, y, z, 0)
    const double *vel = nullptr;         // [npoin][3], or [3][npoin] with vel_soa = npoin
    int64_t vel_soa = 0;
    double rho = 1, mu = 0, dt = 1;
    int32_t accumulate = 0;
    int32_t threads = 256;               // workgroup size: 64, 128 or 256
    double *values = nullptr;
    double *rhs = nullptr;
};

// LDS layout of a tile workgroup (sized per tile), in doubles from the start of dynamic LDS: the
// block image at a padded stride of 17 doubles, the RHS rows at a stride of 5, then the node table
// (x, y, z, u, v, w) at a 16-byte aligned offset.
constexpr int kBlkStride = 17;
constexpr int kRhsStride = 5;
__host__ __device__ constexpr int64_t lds_racc_off(int32_t nblk) { return (int64_t)kBlkStride * nblk; }
__host__ __device__ constexpr int64_t lds_nodes_off(int32_t nblk, int32_t nrows) {
    return (lds_racc_off(nblk) + (int64_t)kRhsStride * nrows + 1) & ~int64_t(1);
}
__host__ __device__ constexpr int64_t lds_tile_doubles(int32_t nblk, int32_t nrows, int32_t nnodes) {
    return lds_nodes_off(nblk, nrows) + 6 * (int64_t)nnodes;
}
// LDS bytes of a tile workgroup.
inline size_t tile_lds_bytes(int32_t nblk, int32_t nrows, int32_t nnodes) {
    return (size_t)lds_tile_doubles(nblk, nrows, nnodes) * 8;
}

// Workgroup-to-tile order of the row-tiled kernels. Workgroup w runs on XCD w % 8; XCD x takes the
// runs x, x + 8, x + 16, ... of kXcdRun consecutive tiles, in dispatch order. Neighbouring tiles of a
// run share nodal data in that XCD's L2, and every XCD draws runs from the whole row range: tiles at
// the two ends of a bandwidth-reducing order take longer, so one contiguous eighth per XCD left some
// XCDs finishing several percent after the others. The map is one-to-one from [0, xcd_grid(n)) onto
// [0, xcd_grid(n)) and so covers every tile below n; workgroups mapped at or beyond n return at once.
constexpr int kXcdRun = 16;
__host__ __device__ constexpr int64_t xcd_grid(int64_t n) {
    return 8 * (((n + kXcdRun - 1) / kXcdRun + 7) / 8) * kXcdRun;
}
__host__ __device__ constexpr int64_t xcd_item(int64_t w) {
    return (((w >> 3) / kXcdRun) * 8 + (w & 7)) * kXcdRun + (w >> 3) % kXcdRun;
}

enum class TileKern { F64, Mixed };
hipError_t launch_tiled(TileKern k, const TileArgs &a, hipStream_t s);
// Batched form: desc[mesh] in device memory, work[t] = (mesh, local tile). grid_wgs 0: one workgroup
// per item; otherwise a persistent grid of that many workgroups (a multiple of 8, fewer than the items).
hipError_t prepare_batch(int threads, size_t lds);
hipError_t launch_tiled_batch(TileKern k, const TileArgs *desc, const int2 *work, int64_t total, int threads,
                              int64_t lds, int grid_wgs, hipStream_t s);

hipError_t ensure_lds(const void *kern, size_t bytes);

// Batched form without a workspace: the member descriptors, the tile offsets and the work table sit
// in one file-scope device array per GPU (its address from static_scratch, taken once per device with
// that device current). Layout: desc [kStaticMeshes] TileArgs, toff [kStaticMeshes + 1] int64 (first
// tile of each member in the work list, toff[nmesh] = total), work [kStaticTiles] int2.
constexpr int32_t kStaticMeshes = 256;
constexpr int64_t kStaticTiles = int64_t(1) << 20;
constexpr size_t kStaticToffOff = ((size_t)kStaticMeshes * sizeof(TileArgs) + 255) & ~size_t(255);
constexpr size_t kStaticWorkOff = (kStaticToffOff + (size_t)(kStaticMeshes + 1) * 8 + 255) & ~size_t(255);
constexpr size_t kStaticBytes = kStaticWorkOff + (size_t)kStaticTiles * 8;
// Descriptors travel as kernel arguments, kDescChunk members per launch.
constexpr int kDescChunk = 8;
struct DescChunk {
    TileArgs d[kDescChunk];
    int64_t toff[kDescChunk + 1];  // first tile of each member, then the first tile after the chunk
    int32_t first = 0;             // index of d[0] among the members
    int32_t count = 0;             // members in this chunk (1 .. kDescChunk)
};
hipError_t static_scratch(char **ptr);
hipError_t launch_put_desc(char *scratch, const DescChunk &c, hipStream_t s);
hipError_t launch_fill_work(char *scratch, int32_t nmesh, int64_t total, hipStream_t s);

// Bandwidth probes (kind 0 read, 1 write, 2 copy) over n doubles on a device of ncu compute units.
hipError_t launch_probe(int kind, const double *src, double *dst, int64_t n, int ncu, hipStream_t s);

// Gather tiles. Tile t owns the contiguous block rows [row[t], row[t+1]) as in the row tiles above,
// with the same node table (owned rows first). Its elements are records rec[eptr[t] .. eptr[t+1])
// holding the four local node ids in the element's own vertex order (uint16 each), sorted by
// element id. Every owned block is a list of contributions (record r, vertices a, b): element r
// adds its 4x4 block (a, b) there. The lists sit in pairs[pptr[t] ..] as uint16 r << 4 | a << 2 | b,
// each list in record order; the tile's blocks are visited in slot order, slot[bptr[row[t]] + s] =
// local block index << 16 | offset of its list in the tile's pairs (a list ends where the next
// slot's begins, the last one at the tile's pair count). Slots run from long lists to short ones so
// that the lanes of one wavefront loop over lists of similar length.
struct GatherArgs {
    int64_t ntiles = 0;
    int64_t lds_bytes = 0;
    const int32_t *tile_row = nullptr;   // [ntiles+1]
    const int64_t *tile_nptr = nullptr;  // [ntiles+1]
    const int32_t *tile_nodes = nullptr;
    const int64_t *tile_eptr = nullptr;  // [ntiles+1]
    const uint2 *rec = nullptr;          // local node ids, 4 x uint16
    const int64_t *tile_pptr = nullptr;  // [ntiles+1]
    const uint16_t *pairs = nullptr;
    const uint32_t *slot = nullptr;      // [nnzb]
    const int64_t *bptr = nullptr;
    const double4 *coord = nullptr;
    const double *vel = nullptr;
    int64_t vel_soa = 0;                 // 0: vel [npoin][3]; npoin: vel [3][npoin]
    double rho = 1, mu = 0, dt = 1;
    int32_t accumulate = 0;
    int32_t threads = 256;
    double *values = nullptr;
    double *rhs = nullptr;
};

// LDS of a gather tile: node table (6 doubles per node), the per-element data (kGatherRecF32 floats
// or kGatherRecF64 doubles per record; odd multiples of 16 bytes so that the records of the lanes of
// one 16-byte read spread over the banks), the records' local node ids (8 bytes each), then the
// tile's contribution lists (2 bytes each).
constexpr int kGatherRecF32 = 44;
constexpr int kGatherRecF64 = 46;
__host__ __device__ constexpr int64_t gather_elem_off(int32_t nnod) { return (48 * (int64_t)nnod + 15) & ~int64_t(15); }
__host__ __device__ constexpr int64_t gather_rec_bytes(bool f64) { return f64 ? 8 * kGatherRecF64 : 4 * kGatherRecF32; }
__host__ __device__ constexpr int64_t gather_loc_off(int32_t nnod, int32_t nrec, bool f64) {
    return gather_elem_off(nnod) + (int64_t)nrec * gather_rec_bytes(f64);
}
__host__ __device__ constexpr int64_t gather_pair_off(int32_t nnod, int32_t nrec, bool f64) {
    return gather_loc_off(nnod, nrec, f64) + 8 * (int64_t)nrec;
}
__host__ __device__ constexpr int64_t gather_lds_bytes(int32_t nnod, int32_t nrec, int32_t npair, bool f64) {
    return gather_pair_off(nnod, nrec, f64) + ((2 * (int64_t)npair + 15) & ~int64_t(15));
}
hipError_t launch_gather(TileKern k, const GatherArgs &a, hipStream_t s);

struct GatherPlan {
    int32_t tile_blocks = 0;
    int32_t threads = 256;
    bool ok = false;
    int64_t lds[2] = {0, 0};      // LDS of the largest tile: [0] FP64 element data, [1] mixed (FP32)
    int32_t cap_blocks = 0, cap_recs = 0, cap_nodes = 0, cap_pairs = 0;
    std::vector<int32_t> row;     // [ntiles+1]
    std::vector<int64_t> nptr, eptr, pptr;
    std::vector<int32_t> nodes, elems;
    std::vector<uint2> recs;
    std::vector<uint16_t> pairs;
    std::vector<uint32_t> slots;  // [nnzb]
    Region r_row, r_nptr, r_nodes, r_eptr, r_recs, r_pptr, r_pairs, r_slots;
    int64_t ntiles() const { return ok ? (int64_t)row.size() - 1 : 0; }
};

// Residual tiles (the explicit-residual outputs): tile t owns the contiguous rows [row[t], row[t+1]);
// its node table is laid out as for the row tiles (owned rows first); its elements are 8-byte
// records rec[eptr[t] .. eptr[t+1]) with the four local node ids, owned nodes first, ordered by
// owned-node count (descending), then so that each group of 16 takes rows distinct mod 16. LDS: node table (6 doubles per node), then 5 accumulators per
// owned row (3 residual components, the tau- and the rho-weighted lumped mass).
struct ResArgs {
    int64_t ntiles = 0;
    int64_t lds_bytes = 0;
    const int32_t *tile_row = nullptr;   // [ntiles+1]
    const int64_t *tile_eptr = nullptr;  // [ntiles+1]
    const uint2 *rec = nullptr;
    const int64_t *tile_nptr = nullptr;  // [ntiles+1]
    const int32_t *tile_nodes = nullptr;
    const double4 *coord = nullptr;
    const double *vel = nullptr;
    int64_t vel_soa = 0;                 // 0: vel [npoin][3]; npoin: vel [3][npoin]
    double rho = 1, mu = 0, dt = 1;
    int32_t accumulate = 0;
    double *rhsid = nullptr;             // [npoin][3]
    double *dt_rho = nullptr;            // [npoin]
    double *mass_rho = nullptr;          // [npoin]
    // precomputed geometry (null: formed from the coordinates): geo[e] = grad N_0..3 (12), V, h, 1/h, 0
    // for element e in its own vertex order; rgel[p] = (element of record p, vertex order: bits 2a..2a+1
    // hold the element vertex at the record's local vertex a)
    const double *geo = nullptr;
    const uint2 *rgel = nullptr;
};
constexpr int kGeoDoubles = 16;
constexpr int kResStride = 5;
__host__ __device__ constexpr int64_t res_lds_bytes(int32_t nnod, int32_t nrows) {
    return 48 * (int64_t)nnod + 8 * (int64_t)kResStride * nrows;
}
hipError_t launch_residual(TileKern k, const ResArgs &a, hipStream_t s);

struct ResPlan {
    int32_t tile_rows = 0;
    bool ok = false;
    int64_t lds = 0;
    std::vector<int32_t> row;     // [ntiles+1]
    std::vector<int64_t> eptr, nptr;
    std::vector<int32_t> nodes, elems;
    std::vector<uint2> recs;
    Region r_row, r_eptr, r_nptr, r_nodes, r_recs;
    Region r_geo, r_rgel;         // precomputed geometry (nsa_mesh_set_residual_geometry)
    int64_t ntiles() const { return ok ? (int64_t)row.size() - 1 : 0; }
};

// ---- 2-D family: bilinear quadrilaterals (four nodes, two dimensions, dofs u v p, 3x3 blocks) ----
// Row tiles as for the tetrahedra: tile t owns the contiguous rows [row[t], row[t+1]) and their blocks
// [b0[t], b0[t+1]); its node table holds the owned rows first (local ids 0 .. nrows-1), then the other
// nodes its elements touch, ascending. One record per (element, tile) with an owned vertex, 48 bytes
// (Q1Rec): the element's four local node ids in its own (counter-clockwise) vertex order, a mask of
// the owned vertices and, for owned vertex a and every vertex b, the tile-local slot of block (a, b).
struct Q1Rec {
    uint16_t loc[4];
    uint16_t own, pad0;
    uint16_t slot[16];   // slot[4a + b]; 0 where vertex a is not owned
    uint16_t pad1[2];
};
static_assert(sizeof(Q1Rec) == 48, "Q1 record layout");

struct Q1Args {
    int64_t ntiles = 0;
    int64_t lds_bytes = 0;
    const int32_t *tile_row = nullptr;   // [ntiles+1]
    const int64_t *tile_b0 = nullptr;    // [ntiles+1] first block of each tile (bptr at its first row)
    const int64_t *tile_nptr = nullptr;  // [ntiles+1]
    const int32_t *tile_nodes = nullptr;
    const int64_t *tile_eptr = nullptr;  // [ntiles+1]
    const uint4 *recs = nullptr;         // Q1Rec as 3 x uint4
    const double2 *coord = nullptr;      // [npoin] (x, y)
    const double *vel = nullptr;         // [npoin][2], or [2][npoin] with vel_soa = npoin
    int64_t vel_soa = 0;
    double rho = 1, mu = 0, dt = 1;
    int32_t accumulate = 0;
    int32_t threads = 256;
    double *values = nullptr;            // [nnzb][3][3]
    double *rhs = nullptr;               // [npoin][3]
};
// LDS of a quadrilateral tile: block image (9 doubles per block), RHS rows (3 doubles), node table
// (x, y, u, v per node) at a 16-byte aligned offset.
__host__ __device__ constexpr int64_t q1_racc_off(int32_t nblk) { return 9 * (int64_t)nblk; }
__host__ __device__ constexpr int64_t q1_nodes_off(int32_t nblk, int32_t nrows) {
    return (q1_racc_off(nblk) + 3 * (int64_t)nrows + 1) & ~int64_t(1);
}
__host__ __device__ constexpr int64_t q1_lds_bytes(int32_t nblk, int32_t nrows, int32_t nnod) {
    return 8 * (q1_nodes_off(nblk, nrows) + 4 * (int64_t)nnod);
}
hipError_t launch_q1(TileKern k, const Q1Args &a, hipStream_t s);

struct Q1Plan {
    int32_t tile_blocks = 0;
    int32_t threads = 256;
    bool ok = false;
    int64_t lds = 0;
    std::vector<int32_t> row;     // [ntiles+1]
    std::vector<int64_t> b0, nptr, eptr;
    std::vector<int32_t> nodes, elems;
    std::vector<Q1Rec> recs;
    Region r_row, r_b0, r_nptr, r_nodes, r_eptr, r_recs;
    int64_t ntiles() const { return ok ? (int64_t)row.size() - 1 : 0; }
};

// A row-tile plan for one scatter mode (host copy, then device regions after upload).
struct TilePlan {
    int32_t tile_blocks = 0;     // requested tile size: LDS budget tile_blocks * 160 bytes
    int32_t threads = 256;       // workgroup size the plan is meant for (runs per tile at most this)
    bool ok = false;             // plan exists (the mesh fits the tiled kernel)
    int32_t cap_blocks = 0, cap_rows = 0, cap_nodes = 0, cap_runs = 0;
    int64_t lds = 0;             // LDS bytes of the largest tile
    int64_t npairs = 0;          // (element, row) pairs over all runs (4 nelem)
    std::vector<int32_t> row;    // [ntiles+1]
    std::vector<int64_t> rptr;   // [ntiles+1]
    std::vector<RunRec> runs;    // [nruns]
    std::vector<int32_t> relems; // [nruns][kRunMax] element of each run position (-1 past the run)
    std::vector<int64_t> nptr;   // [ntiles+1]
    std::vector<int32_t> nodes;
    Region r_row, r_rptr, r_nptr, r_nodes, r_runs, r_b0, r_npad;
    int64_t ntiles() const { return ok ? (int64_t)row.size() - 1 : 0; }
    int64_t nruns() const { return ok ? rptr.back() : 0; }
};

}  // namespace nsa

struct nsa_mesh {
    int32_t family = NSA_TET4;          // NSA_TET4 or NSA_QUAD4
    int64_t npoin = 0, nelem = 0, nnzb = 0;
    int32_t ncolours = 0;
    int64_t max_row_blocks = 0;
    bool host_released = false;
    // host copies
    std::vector<int32_t> lnods;         // [nelem][4]
    std::vector<double> coord;          // [npoin][3] ([npoin][2] for quadrilateral meshes)
    std::vector<int64_t> bptr;          // [npoin+1]
    std::vector<int32_t> bcol;          // [nnzb]
    std::vector<int32_t> emap;          // [nelem][16]
    std::vector<int32_t> colour_ptr;    // [ncolours+1]
    std::vector<int32_t> colour_elems;  // [nelem]
    // row-tile plans: [NSA_ATOMIC] throughput plan, [NSA_COLOUR] deterministic plan; built on first
    // need (info, tiles, upload) from the requested sizes (0 = no plan for that mode)
    nsa::TilePlan plan[2];
    int32_t want_blocks[2] = {0, 0};
    int32_t want_threads = 256;         // workgroup size of the throughput plan
    nsa::GatherPlan gplan;              // gather tiles (both scatter modes, both precisions)
    int32_t want_gather = 0;
    nsa::Q1Plan qplan[2];               // quadrilateral meshes: row tiles per scatter mode
    nsa::Region r_coord2;               // quadrilateral meshes: coordinates (x, y)
    nsa::ResPlan rplan;                 // residual tiles (explicit-residual outputs)
    int32_t want_res = 0;
    bool res_geo_cached = false;        // residual path reads precomputed element geometry
    bool planned = false;
    bool keep_direct = true;            // upload the direct kernel's SoA arrays
    std::mutex plan_mu;
    // device layout (offsets into the caller's workspace)
    nsa::Region r_ln, r_coord, r_emap, r_ln_c, r_emap_c, r_coord4, r_bptr;
    nsa::Region r_esamp;                // err_out sample: node ids of up to NSA_ERR_SAMPLE elements
    size_t ws_bytes = 0;
    char *ws = nullptr;                 // device, caller-owned
    int device = -1;
};
