/*
 * nsa.h -- C ABI of libnsa: P1-tetrahedron incompressible Navier-Stokes element assembly into a
 * global block-CSR matrix plus right-hand side, on AMD Instinct MI355X (gfx950).
 *
 * The operation is the element loop of the paper (Brown, arXiv 2111.05651, Sec. II-A, Listing 1):
 * for every linear tetrahedron, gather the nodal coordinates and velocities through the
 * connectivity (Listing 2, calculate_transients), form the Cartesian shape-function derivatives,
 * the Gauss-point values, the stabilisation parameters and the element operators, build the
 * convective/RHS and viscous terms, and add the element contributions into the global system
 * through the same connectivity (Listing 2, perform_assembly_in_global_system). Here the global
 * system is a fixed-pattern block-CSR matrix with the velocity-velocity, velocity-pressure,
 * pressure-velocity and pressure-pressure couplings (a 16x16 element matrix per tet) and a
 * nodal RHS, rather than the paper's three nodal vectors.
 *
 * Conventions (all calls):
 *   - 0-based node ids; int32 connectivity lnods[nelem][4]; FP64 coordinates coord[npoin][3] and
 *     velocities vel[npoin][3] (dimension fastest, as coord(j, ipoin) / veloc(j, ipoin) in Listing 2).
 *   - Degrees of freedom: 4 per node, dof = 4*node + c with c = 0,1,2 the velocity components and
 *     c = 3 the pressure. Matrix rows are test functions, columns trial functions.
 *   - Matrix layout: BSR with 4x4 blocks. Row i holds the blocks bptr[i] .. bptr[i+1]-1, one per node
 *     that shares an element with node i, columns bcol[] strictly ascending; the diagonal block is
 *     present for every node that belongs to an element (a node in no element has an empty row). values[k][c][c'] (128 bytes per block,
 *     row-major inside the block) is the coupling of dof (row, c) with dof (bcol[k], c').
 *     The scalar CSR view is row_ptr[4i+c] = 16*bptr[i] + 4*c*deg(i), with the 4*deg(i) entries of
 *     that scalar row ordered by (block, c').
 *   - rhs[npoin][4] uses the same dof order.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP device memory of the GPU
 *     that is current when the call is made. All device memory is owned by the caller; libnsa never
 *     frees it. A mesh handle is owned by the caller until nsa_mesh_destroy.
 *   - Device work is enqueued on the caller's stream (hipStream_t passed as void*; NULL = the
 *     default stream) and is asynchronous unless stated otherwise.
 *   - Arguments are checked on the host before anything is launched. On error nothing is launched,
 *     outputs are left untouched, a negative nsa_status is returned and nsa_last_error() describes
 *     the failure (thread-local).
 */
#ifndef NSA_H
#define NSA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nsa_status;
#define NSA_OK 0
#define NSA_EINVAL (-1)        /* bad argument (null pointer, negative size, bad option) */
#define NSA_ERANGE (-2)        /* a connectivity entry outside [0, npoin) */
#define NSA_EDEGENERATE (-3)   /* an element with det J == 0 (or not finite) */
#define NSA_ENOMEM (-4)        /* host allocation failed, or a caller buffer is too small */
#define NSA_EHIP (-5)          /* a HIP runtime call failed */
#define NSA_EUNSUPPORTED (-6)  /* valid request the library cannot serve (e.g. > 128 colours) */
#define NSA_ESTATE (-7)        /* call out of order (e.g. assemble before upload) */

/* precision */
#define NSA_FP64 0             /* everything in FP64 */
#define NSA_MIXED 1            /* Jacobian, inverse, volume and length in FP64; element integration
                                  in FP32; global accumulation in FP64 */
/* scatter: how contributions that target the same block are combined */
#define NSA_ATOMIC 0           /* FP64 atomic adds from concurrent threads (throughput mode; the
                                  order of the additions, hence the last bits, may vary by run) */
#define NSA_COLOUR 1           /* deterministic, bit-reproducible: the tiled kernel processes each
                                  tile's runs in the plan's fixed order inside a single wavefront, so
                                  the adds into each LDS word come in program order; where two lanes
                                  of one add instruction hit the same word (runs of one row in a
                                  tile of fewer rows than lanes), the reproducibility rests on the
                                  LDS applying an instruction's lanes in a fixed order, which the
                                  tests check run to run but AMD does not document. The direct
                                  kernel (NSA_KERNEL_DIRECT) runs one global colour class at a time
                                  with plain load-add-store and needs no such assumption, as does
                                  the gather kernel (NSA_KERNEL_GATHER) */

/* velocity layout (nsa_options.vel_layout) */
#define NSA_VEL_AOS 0          /* vel[node][d], d < the mesh's dimensions: veloc(idime, ipoin) of Listing 2 */
#define NSA_VEL_SOA 1          /* vel[d][node]: one contiguous array of npoin values per component */

/* kernel family */
#define NSA_KERNEL_AUTO 0      /* the row-tiled kernel when the mesh allows it, else the direct one */
#define NSA_KERNEL_TILED 1     /* row tiles: each workgroup owns contiguous block rows, reduces the
                                  contributions to them in LDS and writes every block once */
#define NSA_KERNEL_DIRECT 2    /* element per lane, scattering straight into the global arrays
                                  (zero-fill first unless accumulating); reference implementation */
#define NSA_KERNEL_GATHER 3    /* gather tiles: each block is summed in registers by one lane from a
                                  precomputed list of element contributions (element order) and
                                  stored once; no atomics, bit-reproducible in either scatter mode */

/* element families */
#define NSA_TET4 0             /* linear tetrahedra: 4 nodes, 3 dimensions, dofs u v w p (4x4 blocks) */
#define NSA_QUAD4 1            /* bilinear quadrilaterals: 4 nodes, 2 dimensions, dofs u v p (3x3
                                  blocks); Table 2's two 2-D benchmarks */

/* plan indices of nsa_mesh_set_tiling beside the two scatter modes */
#define NSA_GATHER_PLAN 2
#define NSA_RESIDUAL_PLAN 3

typedef struct nsa_options {
    int32_t precision;         /* NSA_FP64 or NSA_MIXED */
    int32_t scatter;           /* NSA_ATOMIC or NSA_COLOUR */
    int32_t accumulate;        /* 0: values/rhs are overwritten; 1: contributions are added to
                                  what the arrays hold (the inout semantics of Listing 2) */
    int32_t block_threads;     /* threads per workgroup, 0 = default; direct kernel: 64..256 in
                                  steps of 64; tiled atomic mode: 64, 128, 192 or 256 (default:
                                  the plan's, see nsa_mesh_set_tile_threads);
                                  ignored by the tiled colour mode (one wavefront per tile) */
    int32_t kernel;            /* NSA_KERNEL_AUTO, _TILED, _DIRECT or _GATHER */
    int32_t vel_layout;        /* NSA_VEL_AOS (0, the default) or NSA_VEL_SOA: how the velocity array
                                  of nsa_assemble, nsa_assemble_residual and
                                  nsa_assemble_batched_static is laid out; the batch handle
                                  (nsa_assemble_batched) takes NSA_VEL_AOS only */
    double *err_out;           /* optional error report of nsa_assemble (NULL: none; the other
                                  entry points take NULL only). Device pointer to 12 doubles,
                                  8-byte aligned, written in stream order after the assembly:
                                  NSA_ERR_SAMPLE elements spread evenly over the mesh (all of them
                                  in a smaller mesh) are evaluated in the call's precision and in
                                  FP64; per class k of NSA_ERR_UU .. NSA_ERR_RHS_P, err_out[k] =
                                  max |value - FP64 value| and err_out[6 + k] = max |FP64 value|
                                  over every element block entry (RHS entry) of the sample, so
                                  err_out[k] / err_out[6 + k] is the class's relative error of the
                                  mixed form (0 for NSA_FP64). Calls that overlap on one err_out
                                  race. */
} nsa_options;

/* err_out classes: the velocity-velocity, velocity-pressure, pressure-velocity and
 * pressure-pressure parts of the element blocks, then the velocity and pressure rows of the RHS */
#define NSA_ERR_UU 0
#define NSA_ERR_UP 1
#define NSA_ERR_PU 2
#define NSA_ERR_PP 3
#define NSA_ERR_RHS_U 4
#define NSA_ERR_RHS_P 5
#define NSA_ERR_SAMPLE 4096       /* elements of a mesh sampled for err_out */

typedef struct nsa_mesh_info {
    int64_t npoin, nelem, nnzb;
    int32_t ncolours;          /* global greedy element colours (direct colour kernel) */
    int32_t uploaded;          /* 1 once nsa_mesh_upload succeeded */
    size_t ws_bytes;           /* device workspace nsa_mesh_upload needs */
    int64_t max_row_blocks;    /* largest row degree of the block pattern */
    /* row-tile plans of the tiled kernel, indexed by scatter mode (NSA_ATOMIC, NSA_COLOUR) */
    int64_t ntiles[2];         /* number of tiles (0 if the mesh cannot use the tiled kernel) */
    int64_t tile_runs[2];      /* runs over all tiles (see nsa_mesh_get_tiles) */
    int32_t tile_blocks[2];    /* requested tile size (LDS budget tile_blocks * 160 bytes) */
    int32_t tile_threads[2];   /* workgroup size of the plan (a tile holds at most tile_threads - 64
                                  runs, tile_threads for 64, unless one row alone has more) */
    int32_t tile_max_runs[2];  /* largest number of runs in one tile */
    int32_t tile_lds_bytes[2]; /* LDS a workgroup uses (largest tile) */
    /* gather plan (NSA_KERNEL_GATHER) */
    int64_t gather_ntiles;     /* 0 if there is none */
    int64_t gather_records;    /* sum over tiles of the elements each tile evaluates */
    int64_t gather_pairs;      /* element contributions (16 per element) */
    int32_t gather_tile_blocks;/* requested blocks per tile */
    int32_t gather_threads;    /* workgroup size */
    int32_t gather_lds_bytes[2]; /* LDS of the largest tile, [0] FP64, [1] mixed precision */
    /* residual plan (nsa_assemble_residual) */
    int64_t residual_ntiles;   /* 0 if there is none */
    int64_t residual_records;  /* sum over tiles of the elements each tile evaluates */
    int32_t residual_tile_rows;/* requested rows per tile */
    int32_t residual_lds_bytes;/* LDS of the largest tile */
    int32_t family;            /* NSA_TET4 or NSA_QUAD4 */
    int32_t pad0;
} nsa_mesh_info;

typedef struct nsa_mesh nsa_mesh; /* opaque */

/* ---- library ------------------------------------------------------------------------------- */

/* Static description of a status code. Never NULL. */
const char *nsa_status_string(nsa_status st);
/* Detail of the last failure on this thread ("" if none). Valid until the next libnsa call on the
 * same thread. */
const char *nsa_last_error(void);
/* Library version as major*10000 + minor*100 + patch (300 = 0.3.0: the tiled kernel walks runs of
 * elements around an edge, nsa_mesh_get_tiles returns run records). */
int32_t nsa_version(void);

/* ---- block pattern of the node graph (host, standalone) ------------------------------------- */

/* Block-CSR pattern of a tetrahedral mesh (the fixed sparsity into which Listing 2's assembly
 * scatters, one 4x4 block per pair of nodes that share an element).
 *   lnods   host int32 [nelem][4], entries in [0, npoin).
 *   bptr    host int64 [npoin+1], out: row pointers.
 *   nnzb    out: number of blocks (= bptr[npoin]).
 * Errors: NSA_EINVAL (null or negative sizes), NSA_ERANGE (node id out of range), NSA_ENOMEM. */
nsa_status nsa_pattern_count(int64_t npoin, int64_t nelem, const int32_t *lnods, int64_t *bptr,
                             int64_t *nnzb);
/* Second phase: bcol host int32 [nnzb] (ascending per row), emap host int32 [nelem][4][4] with
 * emap[e][a][b] = block index of (lnods[e][a], lnods[e][b]). bptr must be the output of
 * nsa_pattern_count for the same mesh. emap may be NULL. */
nsa_status nsa_pattern_fill(int64_t npoin, int64_t nelem, const int32_t *lnods, const int64_t *bptr,
                            int32_t *bcol, int32_t *emap);

/* ---- meshes ---------------------------------------------------------------------------------- */

/* Register a mesh (host arrays are copied; the caller may free them afterwards). Validates the
 * connectivity (NSA_ERANGE) and every element's Jacobian (NSA_EDEGENERATE, the offending element
 * is named in nsa_last_error), builds the block pattern, the element-to-block map and a greedy
 * element colouring (elements of one colour share no node; first-fit in element order), and the
 * device data layout. nelem may be 0. */
nsa_status nsa_mesh_create(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord,
                           nsa_mesh **out);
/* The 2-D family (Table 2's Cylinder 2D and Venturi 2D: four nodes per element, about one element per
 * nodal point): bilinear quadrilaterals. lnods host int32 [nelem][4] with the vertices of each element
 * in counter-clockwise order (a clockwise element is accepted: the integrals use |det J|), coord host
 * FP64 [npoin][2]. Validates the connectivity (NSA_ERANGE) and every element's Jacobian at the four
 * Gauss points of the 2x2 rule (NSA_EDEGENERATE if it is zero, not finite or changes sign: a crossed
 * or degenerate quadrilateral), builds the block pattern (3x3 blocks, dof 3 node + c, c = 2 pressure)
 * and the element-to-block map. The mesh then takes nsa_mesh_set_tiling (NSA_ATOMIC, NSA_COLOUR),
 * nsa_mesh_get_info, nsa_mesh_get_pattern, nsa_mesh_upload, nsa_mesh_release_host and nsa_assemble
 * with vel FP64 [npoin][2], values FP64 [nnzb][3][3] and rhs FP64 [npoin][3]; the other mesh calls
 * return NSA_EUNSUPPORTED. The element matrix integrates the same terms as for the tetrahedra with the
 * 2x2 Gauss-Legendre rule (the Jacobian varies over a general quadrilateral), element length
 * h = sqrt(area). */
nsa_status nsa_mesh_create_q1(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord,
                              nsa_mesh **out);
/* Row-tile plan of a quadrilateral mesh for one scatter mode (sizes from nsa_mesh_get_info: ntiles[scatter]
 * tiles, tile_runs[scatter] records; any array may be NULL): tile_row int32 [ntiles+1], tile_eptr int64
 * [ntiles+1], elems int32 [records], recs [records] 48-byte records (uint16 local node ids of the four
 * vertices in the element's order, uint16 mask of the owned vertices, uint16 0, uint16 slot[16] with
 * slot[4a+b] the tile-local block of (vertex a, vertex b) for an owned a, 0 otherwise, two uint16 0),
 * tile_nptr int64 [ntiles+1], tile_nodes int32 (owned rows first, then the other nodes ascending).
 * NSA_EUNSUPPORTED for a tetrahedral mesh. */
nsa_status nsa_mesh_get_q1_tiles(const nsa_mesh *m, int32_t scatter, int32_t *tile_row, int64_t *tile_eptr,
                                 int32_t *elems, void *recs, int64_t *tile_nptr, int32_t *tile_nodes);
/* Re-plan the row tiles the tiled kernel uses for one scatter mode. A tile is a contiguous range of
 * block rows whose LDS footprint (136 bytes per block, 40 per row, 48 per touched node) stays within
 * tile_blocks * 160 bytes (64 <= tile_blocks <= 1024; capped at 160 KB) and whose runs (see
 * nsa_mesh_get_tiles) number at most the plan's workgroup size. Defaults: 512 (NSA_ATOMIC, 256-thread
 * workgroups) and 128 (NSA_COLOUR, one wavefront per tile); tile_blocks = 0 drops the plan of that
 * mode (the tiled kernel then refuses the mode and NSA_KERNEL_AUTO falls back to the direct kernel).
 * Plans are built on first need (nsa_mesh_get_info, nsa_mesh_get_tiles, nsa_mesh_upload). Must be
 * called before nsa_mesh_upload (NSA_ESTATE after). */
nsa_status nsa_mesh_set_tiling(nsa_mesh *m, int32_t scatter, int32_t tile_blocks);
/* With scatter = NSA_GATHER_PLAN the call sizes the gather plan instead, which is not built unless
 * asked for: contiguous row ranges of at most tile_blocks blocks (64..4096; 0 drops the plan), 4095
 * elements and 65535 element
 * contributions, whose LDS (48 bytes per touched node, 376 per element with FP64 element data,
 * 184 in mixed precision, 2 per contribution) stays within 80 KB in mixed precision and 160 KB in
 * FP64.
 * With scatter = NSA_RESIDUAL_PLAN it sizes the plan of nsa_assemble_residual, also built only when
 * asked for: contiguous row ranges of at most tile_blocks rows (1..4096; 0 drops the plan) whose LDS
 * (48 bytes per touched node, 40 per row) stays within 64 KB. */
/* Workgroup size of the throughput (NSA_ATOMIC) tile plan: 64, 128, 192 or 256 threads (default 256).
 * A tile then holds at most threads - 64 runs (threads for 64: one run per lane of every wavefront
 * but the last, which only takes part in loading the tile and writing it out), so the size also
 * bounds the tile. Before nsa_mesh_upload (NSA_ESTATE after). The deterministic plan always uses one
 * wavefront per tile. */
nsa_status nsa_mesh_set_tile_threads(nsa_mesh *m, int32_t threads);
/* Whether nsa_mesh_upload also stores the direct kernel's arrays (SoA connectivity, element-to-block
 * map and their colour-ordered copies, ~160 bytes per element; default 1). With 0 the mesh can only
 * be assembled by the tiled kernel (NSA_KERNEL_DIRECT returns NSA_EUNSUPPORTED). Before upload. */
nsa_status nsa_mesh_keep_direct(nsa_mesh *m, int32_t keep);
nsa_status nsa_mesh_destroy(nsa_mesh *m);
nsa_status nsa_mesh_get_info(const nsa_mesh *m, nsa_mesh_info *info);
/* Copy the block pattern out (host arrays of the sizes given by nsa_mesh_get_info: bptr
 * [npoin+1], bcol [nnzb], emap [nelem][4][4]; any of them may be NULL). Requires the host copy
 * (see nsa_mesh_release_host). */
nsa_status nsa_mesh_get_pattern(const nsa_mesh *m, int64_t *bptr, int32_t *bcol, int32_t *emap);
/* Scalar CSR view of the block pattern (Listing 2's scatter target written out per degree of freedom):
 *   row_ptr host int64 [4*npoin+1]: row_ptr[4i+c] = 16*bptr[i] + 4*c*deg(i) (deg(i) = bptr[i+1]-bptr[i]),
 *                                   row_ptr[4*npoin] = 16*nnzb;
 *   col     host int32 [16*nnzb]:   the entries of scalar row 4i+c in (block, c') order,
 *                                   col[row_ptr[4i+c] + 4*(k - bptr[i]) + c'] = 4*bcol[k] + c'.
 * The value of that entry is values[k][c][c'] of nsa_assemble. Either array may be NULL. Requires the
 * host copy (NSA_ESTATE after nsa_mesh_release_host); NSA_EUNSUPPORTED if 16*nnzb or 4*npoin exceeds
 * the int32 column range. */
nsa_status nsa_pattern_scalar_csr(const nsa_mesh *m, int64_t *row_ptr, int32_t *col);
/* Colour classes: colour_ptr host int32 [ncolours+1], colour_elems host int32 [nelem] (element ids
 * grouped by colour, ascending inside a colour). Either may be NULL. */
nsa_status nsa_mesh_get_colouring(const nsa_mesh *m, int32_t *colour_ptr, int32_t *colour_elems);
/* Row-tile plan of one scatter mode (host arrays sized from nsa_mesh_get_info with k = scatter; any
 * may be NULL): tile_row int32 [ntiles+1] (tile t owns rows tile_row[t] .. tile_row[t+1]-1),
 * tile_rptr int64 [ntiles+1] (run offsets), run_elems int32 [tile_runs][4] (the elements of each
 * run in order, -1 past its length), tile_nptr int64 [ntiles+1] and tile_nodes int32
 * [tile_nptr[ntiles]] (the owned rows of tile t first, as local ids 0 .. nrows-1, then the other
 * nodes its elements touch, ascending), runs 32 bytes per run (uint16 fields, local node ids and
 * block slots relative to the tile's first block bptr[tile_row[t]]):
 *   row, hinge, k0, len, diag, jslot, last, 0, knew[4], kslot[4].
 * Every pair (element e, row i) with e containing the node i of a tile's row lies in exactly one run
 * of that tile; the run's element q has the vertices (row, hinge, k_old(q), knew[q]) with
 * k_old(0) = k0 and k_old(q) = knew[q-1]; kslot[q] is the slot of block (row, k_old(q)), diag of
 * (row, row), jslot of (row, hinge), last of (row, knew[len-1]). One lane of the kernel walks a run,
 * integrates row `row` of each of its elements, sums the blocks (row, row), (row, hinge) and the RHS
 * row over the run in registers and carries block (row, knew[q]) to the next element.
 * NSA_EUNSUPPORTED if the mesh has no plan for that mode. */
nsa_status nsa_mesh_get_tiles(const nsa_mesh *m, int32_t scatter, int32_t *tile_row, int64_t *tile_rptr,
                              int32_t *run_elems, int64_t *tile_nptr, int32_t *tile_nodes, uint8_t *runs);
/* Gather plan (sizes from nsa_mesh_get_info; any array may be NULL): tile_row int32 [ntiles+1],
 * tile_nptr int64 [ntiles+1] and tile_nodes int32 (node tables as for the row tiles), tile_eptr
 * int64 [ntiles+1], elems int32 [gather_records] (element of each record, ascending inside a tile),
 * local_nodes uint16 [gather_records][4] (the element's vertices as local node ids, in its own
 * vertex order), tile_pptr int64 [ntiles+1], pairs uint16 [gather_pairs] (record << 4 | a << 2 | b:
 * record adds its block (a, b) to the block being summed), slots uint32 [nnzb] (for tile t the
 * entries at bptr[tile_row[t]] .. : local block index << 16 | offset of its pair list in the tile;
 * a list ends where the next slot's begins, the last at the tile's pair count). NSA_EUNSUPPORTED
 * without a gather plan. */
nsa_status nsa_mesh_get_gather(const nsa_mesh *m, int32_t *tile_row, int64_t *tile_nptr, int32_t *tile_nodes,
                               int64_t *tile_eptr, int32_t *elems, uint16_t *local_nodes, int64_t *tile_pptr,
                               uint16_t *pairs, uint32_t *slots);
/* Make the mesh device-resident: copies the connectivity, coordinates, block maps, colour lists and
 * schedules into ws (device, at least info.ws_bytes bytes, 256-byte aligned, caller-owned and kept
 * alive while the mesh is used). Synchronous: returns after the copies completed on the stream. */
nsa_status nsa_mesh_upload(nsa_mesh *m, void *ws, size_t ws_bytes, void *stream);
/* Drop the host copy of the pattern and element data after upload (saves host memory for large
 * resident sets); nsa_mesh_get_pattern and nsa_mesh_get_colouring then return NSA_ESTATE. */
nsa_status nsa_mesh_release_host(nsa_mesh *m);

/* ---- assembly -------------------------------------------------------------------------------- */

/* Assemble the global matrix and RHS of one uploaded mesh for the given velocity field,
 * density rho > 0, viscosity mu >= 0 and time step dt > 0 (Listing 1's element loop with the
 * block-CSR matrix as the target of perform_assembly_in_global_system).
 *   vel     device FP64 [npoin][3] (the advection field and the previous-step velocity).
 *   values  device FP64 [nnzb][4][4], rhs device FP64 [npoin][4]; 16-byte aligned; not aliased.
 *   opt     may be NULL (FP64, atomic scatter, overwrite).
 * Asynchronous on stream. Errors: NSA_EINVAL, NSA_ESTATE (not uploaded), NSA_EHIP (launch). */
nsa_status nsa_assemble(const nsa_mesh *m, const double *vel, double rho, double mu, double dt,
                        const nsa_options *opt, double *values, double *rhs, void *stream);

/* ---- batched form ------------------------------------------------------------------------------ */

typedef struct nsa_batch nsa_batch; /* opaque */

/* Many uploaded meshes (uneven sizes) assembled by one launch of the tiled kernel over the
 * concatenated tile lists of all meshes (each mesh's tiles contiguous; one workgroup per tile, every
 * XCD taking runs of 16 consecutive items from the whole list, or a persistent grid, every XCD
 * walking a contiguous eighth; see nsa_assemble_batched). Every mesh must be uploaded on the current
 * device and have a tile plan for `scatter` (NSA_EUNSUPPORTED otherwise). The meshes must outlive
 * the batch. */
nsa_status nsa_batch_create(int32_t nmesh, const nsa_mesh *const *meshes, int32_t scatter, nsa_batch **out);
nsa_status nsa_batch_destroy(nsa_batch *b);
/* A reusable batch for continuous batching: room for up to max_meshes members with max_tiles tiles of
 * the plan for `scatter` in total; its members are chosen, and changed between launches, with
 * nsa_batch_reset. Upload it once (the workspace is sized for the capacity). */
nsa_status nsa_batch_reserve(int32_t max_meshes, int64_t max_tiles, int32_t scatter, nsa_batch **out);
/* Replace the members of a batch (same conditions as nsa_batch_create; a mesh may appear more than
 * once, each entry with its own inputs). NSA_ENOMEM if they exceed the capacity. Host only: the new
 * work table reaches the device with the next nsa_batch_set_inputs, which must come before the next
 * launch. Waits until the previous upload has finished reading the host staging buffer. The device
 * copy is rewritten in stream order: a launch of the same batch still running on another stream
 * would race with it. */
nsa_status nsa_batch_reset(nsa_batch *b, int32_t nmesh, const nsa_mesh *const *meshes);
/* Device workspace the batch needs (for its capacity), the current members' total tiles and
 * elements, LDS per workgroup (any may be NULL). */
nsa_status nsa_batch_get_info(const nsa_batch *b, size_t *ws_bytes, int64_t *ntiles, int64_t *nelem,
                              int32_t *lds_bytes);
/* Attach the workspace ws (device, >= ws_bytes, 256-byte aligned, caller-owned, kept alive while the
 * batch is used) and copy the work table into it, ordered on stream. */
nsa_status nsa_batch_upload(nsa_batch *b, void *ws, size_t ws_bytes, void *stream);
/* Per-mesh inputs and outputs (arrays of nmesh entries, in member order): device
 * velocity [npoin][3], rho > 0, mu >= 0, dt > 0, device values [nnzb][4][4] and rhs [npoin][4]
 * (16-byte aligned); accumulate as in nsa_options. Stream-ordered copy of the per-mesh descriptors
 * into the batch workspace (waits for the previous call's copy to finish reading its host staging).
 * Not to be captured in a graph: call it before launching or replaying one. */
nsa_status nsa_batch_set_inputs(nsa_batch *b, const double *const *vel, const double *rho, const double *mu,
                                const double *dt, double *const *values, double *const *rhs, int32_t accumulate,
                                void *stream);
/* One launch over every tile of every mesh of the batch. opt->scatter must equal the batch's mode;
 * opt->kernel must not be NSA_KERNEL_DIRECT; opt->block_threads may pick 128 or 256 threads per
 * workgroup in the atomic mode. grid_wgs = 0: one workgroup per (mesh, tile); grid_wgs > 0: a
 * persistent grid of that many workgroups (rounded down to a multiple of 8, at least 8) walking the
 * tiles, or one workgroup per tile if that is not fewer; NSA_EINVAL if negative.
 * No allocation, no memset, no host synchronisation: the call may be captured in a HIP graph, and a
 * captured graph replays with whatever inputs the last nsa_batch_set_inputs installed. */
nsa_status nsa_assemble_batched(const nsa_batch *b, const nsa_options *opt, int32_t grid_wgs, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops and
 * harnesses that forbid hipMalloc): the batched form without a batch handle or workspace. The member
 * descriptors, tile offsets and work table go into a fixed device array the library holds on each
 * GPU it runs on (about 8.4 MB, kept until the process ends), written by two small kernels in stream
 * order, then one launch of the tiled kernel over every tile of every mesh (one workgroup per
 * tile). Arguments as nsa_batch_set_inputs (arrays of nmesh entries: device velocity [npoin][3],
 * rho > 0, mu >= 0, dt > 0, device values [nnzb][4][4] and rhs [npoin][4], 16-byte aligned) plus the
 * options of nsa_assemble_batched (opt->scatter picks the plan every mesh must have; accumulate as in
 * nsa_options; NULL = FP64, atomic, overwrite). Limits: nmesh <= 256 and at most 2^20 tiles in total,
 * else NSA_EINVAL with nothing launched. No hipMalloc, hipFree, memset, host copy or host
 * synchronisation. Every call on a GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, or other host threads) race and must be ordered by the caller; a call on one stream after
 * another on the same stream is safe. */
nsa_status nsa_assemble_batched_static(int32_t nmesh, const nsa_mesh *const *meshes, const double *const *vel,
                                       const double *rho, const double *mu, const double *dt, double *const *values,
                                       double *const *rhs, const nsa_options *opt, void *stream);

/* ---- explicit residual ---------------------------------------------------------------------- */

/* Residual tiles (sizes from nsa_mesh_get_info; any array may be NULL): tile_row int32 [ntiles+1]
 * (tile t owns rows tile_row[t] .. tile_row[t+1]-1), tile_eptr int64 [ntiles+1], elems int32
 * [residual_records], local_nodes uint16 [residual_records][4] (owned nodes first), tile_nptr int64
 * [ntiles+1], tile_nodes int32 (owned rows first, then the other touched nodes ascending). */
nsa_status nsa_mesh_get_residual_tiles(const nsa_mesh *m, int32_t *tile_row, int64_t *tile_eptr, int32_t *elems,
                                       uint16_t *local_nodes, int64_t *tile_nptr, int32_t *tile_nodes);
/* Precomputed element geometry for the residual path (the paper's multi-engine design moves
 * calculate_cartesian_derivatives off the engine, Sec. III-C): with cached = 1, nsa_mesh_upload also
 * stores every element's FP64 geometry (gradients of the four shape functions, volume, element length
 * and its inverse; 128 bytes per element) and, per residual record, the element id and its vertex
 * order (8 bytes), and nsa_assemble_residual reads the geometry instead of forming it from the
 * coordinates. Same results up to rounding. Default 0. Before nsa_mesh_upload (NSA_ESTATE after). */
nsa_status nsa_mesh_set_residual_geometry(nsa_mesh *m, int32_t cached);
/* The outputs of Listing 2's perform_assembly_in_global_system instead of a matrix: for every node
 * i (sums over the elements that contain it, a = the vertex of the element at i)
 *   rhsid[i][c]  += b_a[c] - sum_b sum_c' A_uu(a c, b c') U_b[c']    (c, c' = 0..2; the momentum
 *                  residual of the element with the nodal velocities as the trial field and zero
 *                  pressure; b and A are the RHS and the element matrix of nsa_assemble),
 *   dt_rho[i]    += tau1 V / 4   and   mass_rho[i] += rho V / 4   (the tau- and rho-weighted
 *                  lumped masses that calculate_tau_and_tim passes to the scatter: a reading, the
 *                  paper does not define them).
 * rhsid device FP64 [npoin][3], dt_rho and mass_rho device FP64 [npoin], 8-byte aligned; overwritten
 * unless opt->accumulate. opt->scatter must be NSA_ATOMIC; the mesh needs a residual plan.
 * Asynchronous on stream. Errors: NSA_EINVAL, NSA_ESTATE, NSA_EUNSUPPORTED, NSA_EHIP. */
nsa_status nsa_assemble_residual(const nsa_mesh *m, const double *vel, double rho, double mu, double dt,
                                 const nsa_options *opt, double *rhsid, double *dt_rho, double *mass_rho,
                                 void *stream);

/* ---- measurement ----------------------------------------------------------------------------- */

#define NSA_PROBE_READ 0
#define NSA_PROBE_WRITE 1
#define NSA_PROBE_COPY 2
/* A plain HBM stream for calibrating the bandwidth the assembly achieves against what this device
 * delivers (not part of the assembly): NSA_PROBE_READ reads src[0 .. n) (dst receives nothing unless
 * the data hold a value no real input has: pass a device double), NSA_PROBE_WRITE writes dst[0 .. n),
 * NSA_PROBE_COPY copies src into dst. n even, src/dst device FP64 arrays, 16-byte aligned, not
 * overlapping. 16-byte accesses, one pass, each stream in the launch shape that measured fastest for
 * it (reads grid-stride with several loads in flight per lane, writes and copies in contiguous 256 KB
 * chunks per workgroup). Asynchronous on stream. Errors: NSA_EINVAL, NSA_EHIP. */
nsa_status nsa_bandwidth_probe(int32_t kind, const double *src, double *dst, int64_t n, void *stream);

/* ---- synthetic inputs ---------------------------------------------------------------------- */

/* Seeded uniform values (a convenience for synthetic inputs such as request velocities; not part
 * of the assembly): out[i] = lo + (hi - lo) * u_i for 0 <= i < n, with u_i = (z_i >> 11) * 2^-53 and
 * z_i = splitmix64 of the counter seed + (i + 1) * 0x9E3779B97F4A7C15 (the mixing function of Steele,
 * Lea and Flood: z ^= z >> 30, z *= 0xBF58476D1CE4E5B9, z ^= z >> 27, z *= 0x94D049BB133111EB,
 * z ^= z >> 31); the product and the sum are rounded separately. out: device FP64, 8-byte aligned.
 * Asynchronous on stream. Errors: NSA_EINVAL, NSA_EHIP. */
nsa_status nsa_fill_uniform(double *out, int64_t n, uint64_t seed, double lo, double hi, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NSA_H */
