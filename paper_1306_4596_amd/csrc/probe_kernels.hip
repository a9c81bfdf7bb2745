// Streaming probe in the tile shape of the register march kernel at one time
// step per launch: the same three HBM streams per cell (state and source
// read, state written), the same workgroup of NW wavefronts per 64-column x
// tile with RPW rows per wavefront, each lane one column, all loads of a
// wavefront issued before its stores, and no arithmetic to speak of.  Its
// rate is the streaming ceiling of that access shape on the device, the
// figure a one-step march launch is compared with beside the copy kernel.
#include <hip/hip_runtime.h>

#include "probe_internal.h"

namespace kfp {

template <int NW, int RPW>
__global__ __launch_bounds__(NW * 64) void tile_probe_kernel(const double *__restrict__ U,
                                                             const double *__restrict__ F,
                                                             double *__restrict__ V, long rows,
                                                             int nx) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const long r0 = (long)blockIdx.y * (NW * RPW) + (long)w * RPW;
  const bool col = c < nx;
  double u[RPW], f[RPW];
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const long r = r0 + i;
    u[i] = f[i] = 0.0;
    if (col && r < rows) {
      u[i] = U[r * nx + c];
      f[i] = F[r * nx + c];
    }
  }
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const long r = r0 + i;
    if (col && r < rows) V[r * nx + c] = fma(0.5, f[i], u[i]);
  }
}

#define KFP_TILE_PROBES(X) X(8, 17) X(8, 9) X(4, 1)

bool tile_probe_supported(int waves, int rows_per_wave) {
#define KFP_CHECK(W, R) \
  if (waves == W && rows_per_wave == R) return true;
  KFP_TILE_PROBES(KFP_CHECK)
#undef KFP_CHECK
  return false;
}

hipError_t launch_tile_probe(const double *U, const double *F, double *V, long rows, int nx,
                             int waves, int rows_per_wave, hipStream_t s) {
  if (rows <= 0 || nx <= 0) return hipSuccess;
  const long gy = (rows + (long)waves * rows_per_wave - 1) / ((long)waves * rows_per_wave);
  if (gy > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((nx + 63) / 64), (unsigned)gy);
#define KFP_LAUNCH(W, R)                                                                      \
  if (waves == W && rows_per_wave == R) {                                                    \
    hipLaunchKernelGGL((tile_probe_kernel<W, R>), grid, dim3(W * 64), 0, s, U, F, V, rows, nx); \
    return hipGetLastError();                                                                \
  }
  KFP_TILE_PROBES(KFP_LAUNCH)
#undef KFP_LAUNCH
  return hipErrorInvalidValue;
}

}  // namespace kfp
