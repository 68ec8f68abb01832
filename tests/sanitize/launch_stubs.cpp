// Kernel launchers for the CPU sanitizer build of the host library: the host code links against
// these instead of the HIP kernels; the driver never reaches a launch (it uploads nothing), and a
// call would report the runtime as unsupported.
#include "nsa_internal.h"

namespace nsa {
hipError_t launch_fill_zero(double *, int64_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_fill_uniform(double *, int64_t, uint64_t, double, double, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_assemble(Kern, const AsmArgs &, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_tiled(TileKern, const TileArgs &, hipStream_t) { return hipErrorNotSupported; }
hipError_t prepare_batch(int, size_t) { return hipErrorNotSupported; }
hipError_t launch_tiled_batch(TileKern, const TileArgs *, const int2 *, int64_t, int, int64_t, int, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t ensure_lds(const void *, size_t) { return hipErrorNotSupported; }
hipError_t launch_gather(TileKern, const GatherArgs &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_residual(TileKern, const ResArgs &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_q1(TileKern, const Q1Args &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_err_sample(const int4 *, int, const double4 *, const double *, int64_t, double, double, double, bool,
                             double *, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_probe(int, const double *, double *, int64_t, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t static_scratch(char **) { return hipErrorNotSupported; }
hipError_t launch_put_desc(char *, const DescChunk &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_fill_work(char *, int32_t, int64_t, hipStream_t) { return hipErrorNotSupported; }
}  // namespace nsa
