// Internal declarations shared by the host library (nsa_host.cpp) and the HIP kernels
// (nsa_kernels.hip). Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nsa.h"

namespace nsa {

// One device region inside a mesh workspace.
struct Region {
    size_t off = 0, bytes = 0;
};

// Arguments of one element-assembly launch. Element data are SoA with leading dimension ld:
// ln[a*ld + e] (a = 0..3) and emap[k*ld + e] (k = 4a+b, 0..15); coordinates are SoA
// coord[d*npoin + node]; the velocity is the caller's AoS vel[3*node + d].
struct AsmArgs {
    int64_t e0 = 0, e1 = 0;      // element range [e0, e1) of the SoA arrays
    int64_t ld = 0;              // leading dimension of ln / emap
    int64_t npoin = 0;
    const int32_t *ln = nullptr;
    const int32_t *emap = nullptr;
    const double *coord = nullptr;
    const double *vel = nullptr;
    double rho = 1, mu = 0, dt = 1;
    double *values = nullptr;
    double *rhs = nullptr;
};

enum class Kern { AtomicF64, AtomicMixed, ColourF64, ColourMixed };

hipError_t launch_fill_zero(double *p, int64_t n, hipStream_t s);
hipError_t launch_assemble(Kern k, const AsmArgs &a, int threads, hipStream_t s);

}  // namespace nsa

struct nsa_mesh {
    int64_t npoin = 0, nelem = 0, nnzb = 0;
    int32_t ncolours = 0;
    int64_t max_row_blocks = 0;
    bool host_released = false;
    // host copies
    std::vector<int32_t> lnods;         // [nelem][4]
    std::vector<double> coord;          // [npoin][3]
    std::vector<int64_t> bptr;          // [npoin+1]
    std::vector<int32_t> bcol;          // [nnzb]
    std::vector<int32_t> emap;          // [nelem][16]
    std::vector<int32_t> colour_ptr;    // [ncolours+1]
    std::vector<int32_t> colour_elems;  // [nelem]
    // device layout (offsets into the caller's workspace)
    nsa::Region r_ln, r_coord, r_emap, r_ln_c, r_emap_c;
    size_t ws_bytes = 0;
    char *ws = nullptr;                 // device, caller-owned
    int device = -1;
};
