// gfx950 kernels of the learned initial-trace network: a BF16 MFMA GEMM
// (FP32 accumulation) with bias / GELU epilogues and split-K, and the
// element-wise pieces of the backward pass and of Adam.
//
// Every product is cast in "NT" form, C[m][n] = sum_k A[m][k] B[n][k], with
// both operands stored K-contiguous, so one tile loader serves the forward
// product (A = activations, B = W[out][in]), the input gradient (B = W^T
// copy) and the weight gradient (A = dZ^T, B = activations^T).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "mlp_internal.h"

namespace kfp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ---------------------------------------------------------------------------
// GEMM: 128 x 128 output tile per workgroup of 4 wavefronts (2 x 2), each
// wavefront 64 x 64 = 4 x 4 blocks of v_mfma_f32_16x16x32_bf16; K step 32.
// One-dimensional grid of tiles_n x tiles_m x splits workgroups; split z
// covers K range [z*kchunk, min(K, (z+1)*kchunk)).  splits > 1 writes FP32
// partials to P[z][M][N] and the reduce kernel applies the epilogue.
// The next K step's tiles are loaded into registers while the current one
// is multiplied (the loads are in flight during the MFMAs).
// Requirements (checked on the host): K, lda, ldb multiples of 8.
// ---------------------------------------------------------------------------
constexpr int BM = 128, BN = 128, BK = 32, LDS_K = BK + 8;

// Workgroups are dealt to the 8 XCDs round-robin (workgroup w runs on XCD
// w mod 8, each with its own L2).  Tiles that read the same operand block
// form a group of G consecutive tile indices (split-K: the tiles of one
// K chunk; otherwise the row tiles of one column tile when there are fewer
// row tiles, else the column tiles of one row tile).  The remap puts each
// group on one XCD, its members one after another there, so the shared
// block comes from HBM once and then from that XCD's L2.  Bijective; the
// tail that does not fill 8 groups keeps the plain order.
__device__ __forceinline__ int xcd_tile(int w, int T, int G) {
  const int T8 = (T / (8 * G)) * (8 * G);
  if (G > 64 || w >= T8) return w;
  const int xcd = w & 7, q = w >> 3;
  return ((q / G) * 8 + xcd) * G + q % G;
}

__global__ __launch_bounds__(256) void gemm_nt_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 sA[BM * LDS_K];
  __shared__ __attribute__((aligned(16))) __bf16 sB[BN * LDS_K];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int tiles_m = (g.M + BM - 1) / BM, tiles_n = (g.N + BN - 1) / BN;
  const int T = tiles_m * tiles_n * g.splits;
  int mt, nt, z;
  if (g.splits > 1) {
    const int G = tiles_m * tiles_n;
    const int t = xcd_tile(blockIdx.x, T, G);
    z = t / G;
    mt = (t % G) % tiles_m;
    nt = (t % G) / tiles_m;
  } else if (tiles_m <= tiles_n) {
    const int t = xcd_tile(blockIdx.x, T, tiles_m);
    z = 0;
    mt = t % tiles_m;
    nt = t / tiles_m;
  } else {
    const int t = xcd_tile(blockIdx.x, T, tiles_n);
    z = 0;
    nt = t % tiles_n;
    mt = t / tiles_n;
  }
  const int m0 = mt * BM, n0 = nt * BN;
  const int kbeg = z * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 zero8;
#pragma unroll
  for (int i = 0; i < 8; ++i) zero8[i] = (__bf16)0.0f;
  // each thread moves two 16-byte pieces of A and of B per K step
  bf16x8 va[2], vb[2];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int idx = tid + r * 256;
      const int row = idx >> 2;
      const int gk = k0 + (idx & 3) * 8;
      const int gm = m0 + row, gn = n0 + row;
      va[r] = zero8;
      vb[r] = zero8;
      if (gm < g.M && gk < kend) va[r] = *(const bf16x8 *)(g.A + (size_t)gm * g.lda + gk);
      if (gn < g.N && gk < kend) vb[r] = *(const bf16x8 *)(g.B + (size_t)gn * g.ldb + gk);
    }
  };
  if (kbeg < kend) load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int idx = tid + r * 256;
      const int row = idx >> 2;
      const int kk = (idx & 3) * 8;
      *(bf16x8 *)(sA + row * LDS_K + kk) = va[r];
      *(bf16x8 *)(sB + row * LDS_K + kk) = vb[r];
    }
    __syncthreads();
    if (k0 + BK < kend) load(k0 + BK);  // in flight during this step's MFMAs
    bf16x8 af[4], bfm[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      af[i] = *(const bf16x8 *)(sA + (wm * 64 + i * 16 + (lane & 15)) * LDS_K + 8 * (lane >> 4));
      bfm[i] = *(const bf16x8 *)(sB + (wn * 64 + i * 16 + (lane & 15)) * LDS_K + 8 * (lane >> 4));
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfm[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // accumulator register r of block (i, j) holds row 4*(lane/16) + r, column lane%16
  const bool partial = g.splits > 1;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        const int n = n0 + wn * 64 + j * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        float v = acc[i][j][r];
        if (partial) {
          g.P[((size_t)z * g.M + m) * g.N + n] = v;
          continue;
        }
        if (g.bias) v += g.bias[n];
        if (g.C) g.C[(size_t)m * g.ldc + n] = v;
        if (g.Cb) g.Cb[(size_t)m * g.ldcb + n] = (__bf16)(g.gelu ? gelu_f(v) : v);
      }
}

__global__ __launch_bounds__(256) void gemm_reduce_kernel(GemmArgs g, int splits) {
  const size_t total = (size_t)g.M * g.N;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    float v = 0.f;
    for (int z = 0; z < splits; ++z) v += g.P[(size_t)z * total + e];
    const int m = (int)(e / g.N), n = (int)(e % g.N);
    if (g.bias) v += g.bias[n];
    if (g.C) g.C[(size_t)m * g.ldc + n] = v;
    if (g.Cb) g.Cb[(size_t)m * g.ldcb + n] = (__bf16)(g.gelu ? gelu_f(v) : v);
  }
}

// ---------------------------------------------------------------------------
// element-wise pieces
// ---------------------------------------------------------------------------
static int egrid(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)(b > 16384 ? 16384 : (b < 1 ? 1 : b));
}

#define GRID_STRIDE(e, n) \
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (n); \
       e += (size_t)gridDim.x * blockDim.x)

__global__ void f32_to_bf16_kernel(const float *__restrict__ s, __bf16 *__restrict__ d, size_t n) {
  GRID_STRIDE(e, n) d[e] = (__bf16)s[e];
}

// [rows][cols] FP32 into the columns of a wider BF16 matrix (row stride ldd)
__global__ void f32_to_bf16_cols_kernel(const float *__restrict__ s, int cols,
                                        __bf16 *__restrict__ d, long ldd, size_t n) {
  GRID_STRIDE(e, n) {
    const size_t r = e / cols, c = e % cols;
    d[r * ldd + c] = (__bf16)s[e];
  }
}

__global__ void f64_to_f32_kernel(const double *__restrict__ s, const double *__restrict__ base,
                                  float *__restrict__ d, size_t n) {
  if (base) {
    GRID_STRIDE(e, n) d[e] = (float)(s[e] - base[e]);
  } else {
    GRID_STRIDE(e, n) d[e] = (float)s[e];
  }
}

// dY = 2 (Y - T) / (B out): FP32 copy (bias gradient) and BF16 copy (products);
// the squared error is accumulated in FP64.
__global__ __launch_bounds__(256) void mse_grad_kernel(const float *__restrict__ Y,
                                                       const float *__restrict__ T,
                                                       float *__restrict__ d32,
                                                       __bf16 *__restrict__ db, size_t n,
                                                       float scale, double *loss) {
  __shared__ double red[4];
  double acc = 0.0;
  GRID_STRIDE(e, n) {
    const float r = Y[e] - T[e];
    acc += (double)r * (double)r;
    const float d = scale * r;
    d32[e] = d;
    db[e] = (__bf16)d;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, red[0] + red[1] + red[2] + red[3]);
}

// dZ = dA * GELU'(Z)
__global__ void gelu_back_kernel(const float *__restrict__ dA, const float *__restrict__ Z,
                                 float *__restrict__ d32, __bf16 *__restrict__ db, size_t n) {
  GRID_STRIDE(e, n) {
    const float d = dA[e] * gelu_grad_f(Z[e]);
    d32[e] = d;
    db[e] = (__bf16)d;
  }
}

// column sums of a row-major [R][C] FP32 matrix (bias gradients), FP64 accumulation
__global__ __launch_bounds__(256) void colsum_kernel(const float *__restrict__ X, int R, int C,
                                                     float *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  double s = 0.0;
  for (int r = 0; r < R; ++r) s += X[(size_t)r * C + c];
  out[c] = (float)s;
}

// tiled transpose of a BF16 matrix: src [R][C] -> dst [C][R]
__global__ __launch_bounds__(256) void transpose_bf16_kernel(const __bf16 *__restrict__ src,
                                                             __bf16 *__restrict__ dst, int R,
                                                             int C) {
  __shared__ __bf16 tile[64][65];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int r = r0 + i, c = c0 + tx;
    if (r < R && c < C) tile[i][tx] = src[(size_t)r * C + c];
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int c = c0 + i, r = r0 + tx;
    if (r < R && c < C) dst[(size_t)c * R + r] = tile[tx][i];
  }
}

// Adam on FP32 masters; refreshes the BF16 copy.
__global__ void adam_kernel(float *__restrict__ w, const float *__restrict__ g,
                            float *__restrict__ m, float *__restrict__ v,
                            __bf16 *__restrict__ wb, size_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  GRID_STRIDE(e, n) {
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    const float wi = w[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[e] = wi;
    if (wb) wb[e] = (__bf16)wi;
  }
}

// lambda = mean + std * y, FP32 -> FP64 (de-standardised network output)
__global__ void destandardize_kernel(const float *__restrict__ y, const float *__restrict__ mean,
                                     const float *__restrict__ stdv,
                                     const double *__restrict__ base, size_t per, size_t n,
                                     double *__restrict__ lam) {
  GRID_STRIDE(e, n) {
    const size_t j = e % per;
    const double v = (double)mean[j] + (double)stdv[j] * (double)y[e];
    lam[e] = base ? base[e] + v : v;
  }
}

// per-column mean and standard deviation of [R][C] FP32 (FP64 accumulation)
__global__ __launch_bounds__(256) void colstats_kernel(const float *__restrict__ X, int R,
                                                       size_t C, float *__restrict__ mean,
                                                       float *__restrict__ stdv, float floor_) {
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  double s = 0.0, s2 = 0.0;
  for (int r = 0; r < R; ++r) {
    const double x = X[(size_t)r * C + c];
    s += x;
    s2 += x * x;
  }
  const double mu = s / R;
  double var = s2 / R - mu * mu;
  if (var < 0) var = 0;
  double sd = sqrt(var);
  mean[c] = (float)mu;
  stdv[c] = (float)(sd > floor_ ? sd : floor_);
}

__global__ void axpy_kernel(const float *__restrict__ x, float *__restrict__ y, float alpha,
                            size_t n) {
  GRID_STRIDE(e, n) y[e] = fmaf(alpha, x[e], y[e]);
}

__global__ void mul_kernel(const float *__restrict__ a, float *__restrict__ y, size_t n) {
  GRID_STRIDE(e, n) y[e] *= a[e];
}

__global__ void standardize_kernel(float *__restrict__ X, size_t per, size_t n,
                                   const float *__restrict__ mean, const float *__restrict__ stdv) {
  GRID_STRIDE(e, n) {
    const size_t j = e % per;
    X[e] = (X[e] - mean[j]) / stdv[j];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_gemm_nt(const GemmArgs &g_in, int splits, hipStream_t s) {
  GemmArgs g = g_in;
  g.splits = splits;
  const long T = (long)((g.N + BN - 1) / BN) * ((g.M + BM - 1) / BM) * splits;
  if (T < 1 || T > 0x7fffffffL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gemm_nt_kernel, dim3((unsigned)T), dim3(256), 0, s, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits <= 1) return e;
  hipLaunchKernelGGL(gemm_reduce_kernel, dim3(egrid((size_t)g.M * g.N)), dim3(256), 0, s, g,
                     splits);
  return hipGetLastError();
}

hipError_t launch_f32_to_bf16(const float *s_, __bf16 *d, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(egrid(n)), dim3(256), 0, s, s_, d, n);
  return hipGetLastError();
}

hipError_t launch_f32_to_bf16_cols(const float *s_, int rows, int cols, __bf16 *d, long ldd,
                                   hipStream_t s) {
  const size_t n = (size_t)rows * cols;
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(f32_to_bf16_cols_kernel, dim3(egrid(n)), dim3(256), 0, s, s_, cols, d, ldd,
                     n);
  return hipGetLastError();
}

hipError_t launch_f64_to_f32(const double *s_, const double *base, float *d, size_t n,
                             hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(egrid(n)), dim3(256), 0, s, s_, base, d, n);
  return hipGetLastError();
}

hipError_t launch_mse_grad(const float *Y, const float *T, float *d32, __bf16 *db, size_t n,
                           float scale, double *loss, hipStream_t s) {
  hipLaunchKernelGGL(mse_grad_kernel, dim3(egrid(n)), dim3(256), 0, s, Y, T, d32, db, n, scale,
                     loss);
  return hipGetLastError();
}

hipError_t launch_gelu_back(const float *dA, const float *Z, float *d32, __bf16 *db, size_t n,
                            hipStream_t s) {
  hipLaunchKernelGGL(gelu_back_kernel, dim3(egrid(n)), dim3(256), 0, s, dA, Z, d32, db, n);
  return hipGetLastError();
}

hipError_t launch_colsum(const float *X, int R, int C, float *out, hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel, dim3((C + 255) / 256), dim3(256), 0, s, X, R, C, out);
  return hipGetLastError();
}

hipError_t launch_transpose_bf16(const __bf16 *src, __bf16 *dst, int R, int C, hipStream_t s) {
  dim3 grid((C + 63) / 64, (R + 63) / 64);
  hipLaunchKernelGGL(transpose_bf16_kernel, grid, dim3(256), 0, s, src, dst, R, C);
  return hipGetLastError();
}

hipError_t launch_adam(float *w, const float *g, float *m, float *v, __bf16 *wb, size_t n,
                       float lr, float b1, float b2, float eps, float c1, float c2,
                       hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(egrid(n)), dim3(256), 0, s, w, g, m, v, wb, n, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_destandardize(const float *y, const float *mean, const float *stdv,
                                const double *base, size_t per, size_t n, double *lam,
                                hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(destandardize_kernel, dim3(egrid(n)), dim3(256), 0, s, y, mean, stdv, base,
                     per, n, lam);
  return hipGetLastError();
}

hipError_t launch_axpy(const float *x, float *y, float alpha, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(axpy_kernel, dim3(egrid(n)), dim3(256), 0, s, x, y, alpha, n);
  return hipGetLastError();
}

hipError_t launch_mul(const float *a, float *y, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(mul_kernel, dim3(egrid(n)), dim3(256), 0, s, a, y, n);
  return hipGetLastError();
}

hipError_t launch_colstats(const float *X, int R, size_t C, float *mean, float *stdv, float floor_,
                           hipStream_t s) {
  hipLaunchKernelGGL(colstats_kernel, dim3((unsigned)((C + 255) / 256)), dim3(256), 0, s, X, R, C,
                     mean, stdv, floor_);
  return hipGetLastError();
}

hipError_t launch_standardize(float *X, size_t per, size_t n, const float *mean, const float *stdv,
                              hipStream_t s) {
  hipLaunchKernelGGL(standardize_kernel, dim3(egrid(n)), dim3(256), 0, s, X, per, n, mean, stdv);
  return hipGetLastError();
}

}  // namespace kfp

namespace kfp {

// Weight initialisation: N(0, stdv^2) from a counter-based generator
// (splitmix64 of seed and index, two uniforms, Box-Muller).
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void init_normal_kernel(float *w, size_t n, float stdv, unsigned long long seed) {
  GRID_STRIDE(e, n) {
    const unsigned long long h1 = splitmix64(seed ^ (2 * e));
    const unsigned long long h2 = splitmix64(seed ^ (2 * e + 1));
    const double u1 = ((h1 >> 11) + 1.0) * (1.0 / 9007199254740993.0);
    const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
    w[e] = (float)(stdv * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
  }
}

hipError_t launch_init_normal(float *w, size_t n, float stdv, unsigned long long seed,
                              hipStream_t s) {
  hipLaunchKernelGGL(init_normal_kernel, dim3(egrid(n)), dim3(256), 0, s, w, n, stdv, seed);
  return hipGetLastError();
}

}  // namespace kfp
