// Internal declarations of the bandwidth probes beside the march (not public ABI).
#pragma once

#include <hip/hip_runtime.h>

namespace kfp {

// V = U + F / 2 over [rows][nx] FP64 arrays in the tile shape of the
// register march: waves wavefronts of rows_per_wave rows per 64-column tile.
bool tile_probe_supported(int waves, int rows_per_wave);
hipError_t launch_tile_probe(const double *U, const double *F, double *V, long rows, int nx,
                             int waves, int rows_per_wave, hipStream_t s);

}  // namespace kfp
