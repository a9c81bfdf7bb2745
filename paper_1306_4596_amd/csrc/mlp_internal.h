// Internal declarations of the learned initial-trace network (not public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace kfp {

// C[m][n] = sum_k A[m][k] B[n][k].  Each operand is stored either with K
// contiguous (A[m][k] at A + m*lda + k) or K-major (a_kmajor: A[m][k] at
// A + k*lda + m; likewise B with b_kmajor).  Epilogues:
//   EPI_STORE  + bias[n]; optional FP32 output C and BF16 output Cb (GELU
//              applied to Cb when gelu != 0).  P: split-K partials.
//   EPI_MSE    r = C + bias - T (the squared-error residual): Cb = BF16(scale r),
//              loss_part[4*(column tile*row tiles + row tile) + wavefront] =
//              that wavefront's sum of r^2 in FP64 (summed afterwards by
//              launch_sum_f64: one slot per wavefront, no atomics, a fixed
//              order), PB[2*row tile + w][n] = column sum of scale r over the
//              64 rows of wavefront row w of the tile.
//   EPI_ADAM   C is the gradient of W[M][N] (row stride ldw): one Adam step on
//              W, the moments Mo, Vo and the BF16 copy Wb, in place.
// The fused epilogues need the whole K in one tile (splits == 1), N a
// multiple of 8 and ldt, ldcb, ldw multiples of 4.
enum { EPI_STORE = 0, EPI_MSE = 1, EPI_ADAM = 2 };

struct GemmArgs {
  int M, N, K, kchunk;
  const __bf16 *A;
  long lda;
  const __bf16 *B;
  long ldb;
  int a_kmajor, b_kmajor, epi;
  float *C;
  long ldc;
  __bf16 *Cb;
  long ldcb;
  const float *bias;
  int gelu;
  float *P;
  int splits;  // K chunks (set by the launcher)
  // EPI_MSE
  const float *T;
  long ldt;
  float scale;
  double *loss_part;
  float *PB;
  // EPI_ADAM
  float *W, *Mo, *Vo;
  __bf16 *Wb;
  long ldw;
  float lr, b1, b2, eps, c1, c2;
};

hipError_t launch_gemm(const GemmArgs &g, int splits, hipStream_t s);
hipError_t launch_f32_to_bf16(const float *s_, __bf16 *d, size_t n, hipStream_t s);
hipError_t launch_f32_to_bf16_cols(const float *s_, int rows, int cols, __bf16 *d, long ldd,
                                   hipStream_t s);
hipError_t launch_f64_to_f32(const double *s_, const double *base, float *d, size_t n,
                             hipStream_t s);
hipError_t launch_gelu_back(const float *dA, const float *Z, float *d32, __bf16 *db, size_t n,
                            hipStream_t s);
hipError_t launch_colsum(const float *X, int R, int C, float *out, hipStream_t s);
// out[0] = sum of x[0 .. n) in FP64 (one workgroup of 1024 threads, a fixed order)
hipError_t launch_sum_f64(const double *x, size_t n, double *out, hipStream_t s);
hipError_t launch_adam(float *w, const float *g, float *m, float *v, __bf16 *wb, size_t n,
                       float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_destandardize(const float *y, const float *mean, const float *stdv,
                                const double *base, size_t per, size_t n, double *lam,
                                hipStream_t s);
hipError_t launch_axpy(const float *x, float *y, float alpha, size_t n, hipStream_t s);
hipError_t launch_mul(const float *a, float *y, size_t n, hipStream_t s);
hipError_t launch_colstats(const float *X, int R, size_t C, float *mean, float *stdv, float floor_,
                           hipStream_t s);
hipError_t launch_standardize(float *X, size_t per, size_t n, const float *mean, const float *stdv,
                              hipStream_t s);
// x frequencies of a trace's Fourier coefficients (at most 8)
struct TraceModes {
  int n;
  int m[8];
};
hipError_t launch_trace_modes(const double *lam, long rows, int nx, const TraceModes &md,
                              double *coef, hipStream_t s);
hipError_t launch_trace_synth(const double *coef, int planes, int ntc, int nt, int nx,
                              const TraceModes &md, double *lam, hipStream_t s);
hipError_t launch_init_normal(float *w, size_t n, float stdv, unsigned long long seed,
                              hipStream_t s);

}  // namespace kfp
