// gfx950 kernels of the learned initial-trace network: a BF16 MFMA GEMM
// (FP32 accumulation) with bias / GELU epilogues and split-K, and the
// element-wise pieces of the backward pass and of Adam.
//
// Every product is cast as C[m][n] = sum_k A[m][k] B[n][k] with each operand
// either K-contiguous or K-major, so the stored layouts serve all three
// products without transposes: the forward product (A = activations, B =
// W[out][in], both K-contiguous), the input gradient (A = dZ[batch][out],
// B = W[out][in] read K-major) and the weight gradient (A = dZ and B = the
// activations, both K-major with K = batch).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "mlp_internal.h"

namespace kfp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// One Adam step (bias-corrected moments) on one FP32 master weight; the
// same arithmetic in the stand-alone update and in the fused GEMM epilogue.
__device__ __forceinline__ float adam_update(float &w, float gi, float &m, float &v, float lr,
                                             float b1, float b2, float eps, float c1, float c2) {
  const float mi = fmaf(b1, m, (1.f - b1) * gi);
  const float vi = fmaf(b2, v, ((1.f - b2) * gi) * gi);
  m = mi;
  v = vi;
  const float step = (lr * (mi / c1)) / (sqrtf(vi / c2) + eps);
  w = w - step;
  return w;
}

// ---------------------------------------------------------------------------
// GEMM: 128 x 128 output tile per workgroup of 4 wavefronts (2 x 2), each
// wavefront 64 x 64 = 4 x 4 blocks of v_mfma_f32_16x16x32_bf16; K step 64.
// One-dimensional grid of tiles_n x tiles_m x splits workgroups; split z
// covers K range [z*kchunk, min(K, (z+1)*kchunk)).  splits > 1 writes FP32
// partials to P[z][M][N] and the reduce kernel applies the epilogue.
// The next K step's tiles are loaded into registers while the current one
// is multiplied (the loads are in flight during the MFMAs).  The products
// here are HBM-bound with little arithmetic per byte, so a step's wait on
// its loads is close to a whole memory latency: the K step is 64 (16 KiB
// of operand tiles per workgroup in flight) to halve the number of waits.
//
// Both operand tiles sit in LDS as [row][k] (row pitch LDS_K), the layout
// the MFMA fragments read: for the 32-wide k half h, lane l takes the 8
// consecutive k of group 4h + l/16 for row l%16.  A K-contiguous operand is
// copied in 16-byte pieces.  A K-major operand is read from HBM along its
// rows (16 lanes cover 128 consecutive rows of one k) and transposed on the
// way into LDS: each thread loads rows k and k+1 for 8 consecutive tile rows
// and writes the 8 (k, k+1) pairs as 32-bit words.  Within each 32-wide half
// the four 8-wide k groups of a row are XOR-permuted by bits 4-5 of the row
// index: the fragment reads and the
// K-contiguous copies see a permutation that is uniform across each
// wavefront (no change in bank use), while the pair writes of one
// wavefront, 8 rows apart, spread over the banks.
// Requirements (checked on the host): K, lda, ldb multiples of 8; M (N) a
// multiple of 8 for a K-major A (B).
// ---------------------------------------------------------------------------
constexpr int BM = 128, BN = 128, BK = 64, LDS_K = BK + 8;
// 16-byte pieces of one operand tile per thread
constexpr int NP = BM * BK / 8 / 256;
// The fused epilogues stage each wavefront's 64 x 64 FP32 block in LDS, 32
// rows at a time (row pitch EP_PITCH floats: 16-byte aligned rows, and the
// accumulator writes of one wavefront, rows 4 apart, fall in distinct
// banks), and walk it row-major, 16 lanes per row with 4 columns each, so
// every HBM access of the epilogue covers whole 128-byte lines.
constexpr int EP_PITCH = 68;
constexpr int SMEM_AB = 2 * BM * LDS_K * 2;
constexpr int SMEM_EPI = 4 * 32 * EP_PITCH * 4;

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

__device__ __forceinline__ int kswz(int row) { return (row >> 4) & 3; }

// global -> registers: the two pieces of one operand tile this thread moves
template <bool KM>
__device__ __forceinline__ void tile_load(bf16x8 (&v)[NP], const __bf16 *__restrict__ p, long ld,
                                          int r0, int R, int k0, int kend, int tid,
                                          const bf16x8 &zero8) {
  if constexpr (!KM) {
#pragma unroll
    for (int r = 0; r < NP; ++r) {
      const int idx = tid + r * 256;
      const int row = r0 + idx / (BK / 8);
      const int gk = k0 + (idx % (BK / 8)) * 8;
      v[r] = zero8;
      if (row < R && gk < kend) v[r] = *(const bf16x8 *)(p + (size_t)row * ld + gk);
    }
  } else {
    // pieces 2q and 2q + 1: rows k and k + 1 of k pair (tid / 16) + 16 q
    const int row = r0 + 8 * (tid & 15);
#pragma unroll
    for (int r = 0; r < NP; ++r) {
      const int gk = k0 + 2 * ((tid >> 4) + 16 * (r >> 1)) + (r & 1);
      v[r] = zero8;
      if (row < R && gk < kend) v[r] = *(const bf16x8 *)(p + (size_t)gk * ld + row);
    }
  }
}

// registers -> LDS tile [row][k]
template <bool KM>
__device__ __forceinline__ void tile_store(__bf16 *__restrict__ s, const bf16x8 (&v)[NP],
                                           int tid) {
  if constexpr (!KM) {
#pragma unroll
    for (int r = 0; r < NP; ++r) {
      const int idx = tid + r * 256;
      const int row = idx / (BK / 8);
      *(bf16x8 *)(s + row * LDS_K + (((idx % (BK / 8)) ^ kswz(row)) * 8)) = v[r];
    }
  } else {
    const int row0 = 8 * (tid & 15);
#pragma unroll
    for (int q = 0; q < NP / 2; ++q) {
      const int kp = (tid >> 4) + 16 * q;
      const int grp = kp >> 2, off = 2 * (kp & 3);
      // the pieces as raw 16-bit patterns (whole-vector casts: element-wise
      // casts of a BF16 vector are not relied on)
      const u16x8 lo = __builtin_bit_cast(u16x8, v[2 * q]);
      const u16x8 hi = __builtin_bit_cast(u16x8, v[2 * q + 1]);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int row = row0 + j;
        *(uint32_t *)(s + row * LDS_K + ((grp ^ kswz(row)) * 8) + off) =
            (uint32_t)lo[j] | ((uint32_t)hi[j] << 16);
      }
    }
  }
}

template <int EPI, bool AK, bool BKM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void gemm_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16)))
  unsigned char smem[EPI == EPI_STORE ? SMEM_AB : (SMEM_EPI > SMEM_AB ? SMEM_EPI : SMEM_AB)];
  __bf16 *sA = (__bf16 *)smem;
  __bf16 *sB = sA + BM * LDS_K;
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
  bf16x8 va[NP], vb[NP];
  auto load = [&](int k0) {
    tile_load<AK>(va, g.A, g.lda, m0, g.M, k0, kend, tid, zero8);
    tile_load<BKM>(vb, g.B, g.ldb, n0, g.N, k0, kend, tid, zero8);
  };
  if (kbeg < kend) load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    tile_store<AK>(sA, va, tid);
    tile_store<BKM>(sB, vb, tid);
    __syncthreads();
    if (k0 + BK < kend) load(k0 + BK);  // in flight during this step's MFMAs
#pragma unroll
    for (int h = 0; h < BK / 32; ++h) {
      bf16x8 af[4], bfm[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int ra = wm * 64 + i * 16 + (lane & 15);
        const int rb = wn * 64 + i * 16 + (lane & 15);
        af[i] = *(const bf16x8 *)(sA + ra * LDS_K + ((4 * h + ((lane >> 4) ^ kswz(ra))) * 8));
        bfm[i] = *(const bf16x8 *)(sB + rb * LDS_K + ((4 * h + ((lane >> 4) ^ kswz(rb))) * 8));
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfm[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator register r of block (i, j) holds row 4*(lane/16) + r, column lane%16
  if (g.splits > 1) {
    // split-K partials; the reduce kernel applies the epilogue
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
          const int n = n0 + wn * 64 + j * 16 + (lane & 15);
          if (m < g.M && n < g.N) g.P[((size_t)z * g.M + m) * g.N + n] = acc[i][j][r];
        }
    return;
  }
  if constexpr (EPI == EPI_STORE) {
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
          if (g.bias) v += g.bias[n];
          if (g.C) g.C[(size_t)m * g.ldc + n] = v;
          if (g.Cb) g.Cb[(size_t)m * g.ldcb + n] = (__bf16)(g.gelu ? gelu_f(v) : v);
        }
  } else {
    // row (4 it + lane/16) of a staged half, columns cq .. cq + 3 (N is a
    // multiple of 8, so the four are valid together)
    float *sE = (float *)smem + wv * 32 * EP_PITCH;
    const int cq = 4 * (lane & 15);
    const int n = n0 + wn * 64 + cq;
    const bool ncol = n < g.N;
    double lsum = 0.0;
    f32x4 cs = {0.f, 0.f, 0.f, 0.f};
    f32x4 bias4 = {0.f, 0.f, 0.f, 0.f};
    if (EPI == EPI_MSE && g.bias && ncol) bias4 = *(const f32x4 *)(g.bias + n);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      // stage rows 32h .. 32h + 31 of this wavefront's block (the previous
      // barrier has retired every read of the operand tiles or of the
      // previous half)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            sE[(i * 16 + 4 * (lane >> 4) + r) * EP_PITCH + j * 16 + (lane & 15)] =
                acc[2 * h + i][j][r];
      __syncthreads();
      const int mrow = m0 + wm * 64 + 32 * h + (lane >> 4);
#pragma unroll
      for (int it0 = 0; it0 < 8; it0 += 4) {
        if constexpr (EPI == EPI_MSE) {
          f32x4 t[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int m = mrow + 4 * (it0 + u);
            t[u] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (ncol && m < g.M) t[u] = *(const f32x4 *)(g.T + (size_t)m * g.ldt + n);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int m = mrow + 4 * (it0 + u);
            if (!ncol || m >= g.M) continue;
            const int rl = 4 * (it0 + u) + (lane >> 4);
            const f32x4 res = (*(const f32x4 *)(sE + rl * EP_PITCH + cq) + bias4) - t[u];
            bf16x4 db;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              lsum += (double)res[c] * (double)res[c];
              const float d = g.scale * res[c];
              db[c] = (__bf16)d;
              cs[c] += d;
            }
            *(bf16x4 *)(g.Cb + (size_t)m * g.ldcb + n) = db;
          }
        } else {
          f32x4 w4[4], m4[4], v4[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int m = mrow + 4 * (it0 + u);
            if (!ncol || m >= g.M) continue;
            const size_t e = (size_t)m * g.ldw + n;
            w4[u] = *(const f32x4 *)(g.W + e);
            m4[u] = *(const f32x4 *)(g.Mo + e);
            v4[u] = *(const f32x4 *)(g.Vo + e);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int m = mrow + 4 * (it0 + u);
            if (!ncol || m >= g.M) continue;
            const int rl = 4 * (it0 + u) + (lane >> 4);
            const f32x4 gr = *(const f32x4 *)(sE + rl * EP_PITCH + cq);
            bf16x4 wb;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              float w = w4[u][c], mo = m4[u][c], vo = v4[u][c];
              adam_update(w, gr[c], mo, vo, g.lr, g.b1, g.b2, g.eps, g.c1, g.c2);
              w4[u][c] = w;
              m4[u][c] = mo;
              v4[u][c] = vo;
              wb[c] = (__bf16)w;
            }
            const size_t e = (size_t)m * g.ldw + n;
            *(f32x4 *)(g.W + e) = w4[u];
            *(f32x4 *)(g.Mo + e) = m4[u];
            *(f32x4 *)(g.Vo + e) = v4[u];
            *(bf16x4 *)(g.Wb + e) = wb;
          }
        }
      }
      if (h == 0) __syncthreads();
    }
    if constexpr (EPI == EPI_MSE) {
      // lanes l, l^16, l^32, l^48 hold the same columns: sum the 64 rows
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        cs[c] += __shfl_xor(cs[c], 16, 64);
        cs[c] += __shfl_xor(cs[c], 32, 64);
      }
      if (lane < 16 && ncol) *(f32x4 *)(g.PB + (size_t)(mt * 2 + wm) * g.N + n) = cs;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
      // one slot per wavefront: an atomic sum into one address serialises
      // every wavefront of the launch on one L2 channel
      if (lane == 0) g.loss_part[((size_t)nt * tiles_m + mt) * 4 + wv] = lsum;
    }
  }
}

__global__ __launch_bounds__(256) void gemm_reduce_kernel(GemmArgs g, int splits) {
  const size_t total = (size_t)g.M * g.N;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    float v = 0.f;
#pragma unroll 8
    for (int z = 0; z < splits; ++z) v += g.P[(size_t)z * total + e];
    const int m = (int)(e / g.N), n = (int)(e % g.N);
    if (g.epi == EPI_ADAM) {
      const size_t o = (size_t)m * g.ldw + n;
      float w = g.W[o], mo = g.Mo[o], vo = g.Vo[o];
      adam_update(w, v, mo, vo, g.lr, g.b1, g.b2, g.eps, g.c1, g.c2);
      g.W[o] = w;
      g.Mo[o] = mo;
      g.Vo[o] = vo;
      g.Wb[o] = (__bf16)w;
      continue;
    }
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

// One workgroup of 1024 threads; each thread keeps 16 independent loads in
// flight per pass, then the wavefront and workgroup sums in a fixed order.
__global__ __launch_bounds__(1024) void sum_f64_kernel(const double *__restrict__ x, size_t n,
                                                       double *__restrict__ out) {
  __shared__ double part[16];
  const int tid = threadIdx.x;
  double v = 0.0;
  for (size_t base = 0; base < n; base += 16 * 1024) {
    double t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const size_t e = base + (size_t)u * 1024 + tid;
      t[u] = e < n ? x[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) v += t[u];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((tid & 63) == 0) part[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < 16; ++w) s += part[w];
    out[0] = s;
  }
}

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

// dZ = dA * GELU'(Z)
__global__ void gelu_back_kernel(const float *__restrict__ dA, const float *__restrict__ Z,
                                 float *__restrict__ d32, __bf16 *__restrict__ db, size_t n) {
  GRID_STRIDE(e, n) {
    const float d = dA[e] * gelu_grad_f(Z[e]);
    d32[e] = d;
    db[e] = (__bf16)d;
  }
}

// column sums of a row-major [R][C] FP32 matrix (bias gradients), FP64
// accumulation: 64 columns per workgroup, each wavefront summing every
// fourth row, the four partial sums added in wavefront order
__global__ __launch_bounds__(256) void colsum_kernel(const float *__restrict__ X, int R, int C,
                                                     float *__restrict__ out) {
  __shared__ double part[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int w = threadIdx.x >> 6;
  double s = 0.0;
  if (c < C) {
#pragma unroll 8
    for (int r = w; r < R; r += 4) s += X[(size_t)r * C + c];
  }
  part[w][threadIdx.x & 63] = s;
  __syncthreads();
  if (w == 0 && c < C)
    out[c] = (float)(((part[0][threadIdx.x] + part[1][threadIdx.x]) + part[2][threadIdx.x]) +
                     part[3][threadIdx.x]);
}

// Adam on FP32 masters; refreshes the BF16 copy.
__global__ void adam_kernel(float *__restrict__ w, const float *__restrict__ g,
                            float *__restrict__ m, float *__restrict__ v,
                            __bf16 *__restrict__ wb, size_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  GRID_STRIDE(e, n) {
    float wi = w[e], mi = m[e], vi = v[e];
    adam_update(wi, g[e], mi, vi, lr, b1, b2, eps, c1, c2);
    m[e] = mi;
    v[e] = vi;
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
template <int EPI>
static void *gemm_entry(int ak, int bk) {
  if (ak && bk) return (void *)gemm_kernel<EPI, true, true>;
  if (ak) return (void *)gemm_kernel<EPI, true, false>;
  if (bk) return (void *)gemm_kernel<EPI, false, true>;
  return (void *)gemm_kernel<EPI, false, false>;
}

hipError_t launch_gemm(const GemmArgs &g_in, int splits, hipStream_t s) {
  GemmArgs g = g_in;
  g.splits = splits;
  if (g.epi == EPI_MSE && splits != 1) return hipErrorInvalidValue;
  const long T = (long)((g.N + BN - 1) / BN) * ((g.M + BM - 1) / BM) * splits;
  if (T < 1 || T > 0x7fffffffL) return hipErrorInvalidValue;
  void *fn = g.epi == EPI_MSE    ? gemm_entry<EPI_MSE>(g.a_kmajor, g.b_kmajor)
             : g.epi == EPI_ADAM ? gemm_entry<EPI_ADAM>(g.a_kmajor, g.b_kmajor)
                                 : gemm_entry<EPI_STORE>(g.a_kmajor, g.b_kmajor);
  void *args[] = {&g};
  hipError_t e = hipLaunchKernel(fn, dim3((unsigned)T), dim3(256), args, 0, s);
  if (e != hipSuccess) return e;
  e = hipGetLastError();
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

hipError_t launch_gelu_back(const float *dA, const float *Z, float *d32, __bf16 *db, size_t n,
                            hipStream_t s) {
  hipLaunchKernelGGL(gelu_back_kernel, dim3(egrid(n)), dim3(256), 0, s, dA, Z, d32, db, n);
  return hipGetLastError();
}

hipError_t launch_colsum(const float *X, int R, int C, float *out, hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel, dim3((C + 63) / 64), dim3(256), 0, s, X, R, C, out);
  return hipGetLastError();
}

hipError_t launch_sum_f64(const double *x, size_t n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(sum_f64_kernel, dim3(1), dim3(1024), 0, s, x, n, out);
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

// ---------------------------------------------------------------------------
// Trace planes as x-Fourier coefficients.  Every operator of the scheme is
// circulant in the periodic x direction, so a field made of the discrete
// modes cos/sin(2 pi m x_i), x_i = i/nx, keeps exactly those modes in every
// trace; a trace row is then its 2 NM coefficients.  The angle 2 pi m i/nx
// is reduced to the exact integer residue (m i) mod nx before sincospi.
// ---------------------------------------------------------------------------
template <int NM>
__global__ __launch_bounds__(256) void trace_modes_kernel(const double *__restrict__ lam,
                                                          long rows, int nx, TraceModes md,
                                                          double *__restrict__ coef) {
  __shared__ double part[4][2 * NM];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (long r = blockIdx.x; r < rows; r += gridDim.x) {
    const double *row = lam + r * nx;
    double acc[2 * NM];
#pragma unroll
    for (int j = 0; j < 2 * NM; ++j) acc[j] = 0.0;
    for (int i = threadIdx.x; i < nx; i += 256) {
      const double x = row[i];
#pragma unroll
      for (int k = 0; k < NM; ++k) {
        const long q = ((long)md.m[k] * i) % nx;
        double sn, cs;
        sincospi(2.0 * (double)q / (double)nx, &sn, &cs);
        acc[2 * k] += x * cs;
        acc[2 * k + 1] += x * sn;
      }
    }
#pragma unroll
    for (int j = 0; j < 2 * NM; ++j) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc[j] += __shfl_xor(acc[j], off, 64);
    }
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < 2 * NM; ++j) part[w][j] = acc[j];
    }
    __syncthreads();
    if (threadIdx.x < 2 * NM) {
      const int j = threadIdx.x;
      coef[r * 2 * NM + j] =
          (2.0 / nx) * (((part[0][j] + part[1][j]) + part[2][j]) + part[3][j]);
    }
    __syncthreads();
  }
}

// lam[p][n][i] from coef[p][ntc][2 NM]: the coefficients of fine level n
// (time (n+1)/nt of the window) interpolated linearly between coarse levels
// (level kc at time (kc+1)/ntc), held at the first and last coarse level
// outside them.  Workgroup: 256 columns x 16 plane-levels per pass.
template <int NM>
__global__ __launch_bounds__(256) void trace_synth_kernel(const double *__restrict__ coef,
                                                          int planes, int ntc, int nt, int nx,
                                                          TraceModes md,
                                                          double *__restrict__ lam) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  double cs[NM], sn[NM];
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    const long q = ((long)md.m[k] * (i < nx ? i : 0)) % nx;
    sincospi(2.0 * (double)q / (double)nx, &sn[k], &cs[k]);
  }
  const long rows = (long)planes * nt;
  for (long r0 = (long)blockIdx.y * 16; r0 < rows; r0 += (long)gridDim.y * 16) {
    const int rend = (int)(rows - r0 < 16 ? rows - r0 : 16);
    for (int rr = 0; rr < rend; ++rr) {
      const long r = r0 + rr;
      const int p = (int)(r / nt), n = (int)(r % nt);
      const double sc = (double)(n + 1) * ntc / nt - 1.0;
      int k0, k1;
      double wt;
      if (sc <= 0.0) {
        k0 = k1 = 0;
        wt = 0.0;
      } else if (sc >= ntc - 1) {
        k0 = k1 = ntc - 1;
        wt = 0.0;
      } else {
        k0 = (int)sc;
        k1 = k0 + 1;
        wt = sc - k0;
      }
      const double *c0 = coef + ((long)p * ntc + k0) * 2 * NM;
      const double *c1 = coef + ((long)p * ntc + k1) * 2 * NM;
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < NM; ++k) {
        const double a = c0[2 * k] + wt * (c1[2 * k] - c0[2 * k]);
        const double b = c0[2 * k + 1] + wt * (c1[2 * k + 1] - c0[2 * k + 1]);
        v += a * cs[k] + b * sn[k];
      }
      if (i < nx) lam[r * nx + i] = v;
    }
  }
}

hipError_t launch_trace_modes(const double *lam, long rows, int nx, const TraceModes &md,
                              double *coef, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const unsigned grid = (unsigned)(rows < 65536 ? rows : 65536);
#define KFP_TM(N)                                                                       \
  case N:                                                                               \
    hipLaunchKernelGGL(trace_modes_kernel<N>, dim3(grid), dim3(256), 0, s, lam, rows, nx, \
                       md, coef);                                                       \
    break;
  switch (md.n) {
    KFP_TM(1) KFP_TM(2) KFP_TM(3) KFP_TM(4) KFP_TM(5) KFP_TM(6) KFP_TM(7) KFP_TM(8)
    default:
      return hipErrorInvalidValue;
  }
#undef KFP_TM
  return hipGetLastError();
}

hipError_t launch_trace_synth(const double *coef, int planes, int ntc, int nt, int nx,
                              const TraceModes &md, double *lam, hipStream_t s) {
  const long rows = (long)planes * nt;
  if (rows <= 0 || nx <= 0) return hipSuccess;
  const long ychunks = (rows + 15) / 16;
  dim3 grid((unsigned)((nx + 255) / 256), (unsigned)(ychunks < 65535 ? ychunks : 65535));
#define KFP_TS(N)                                                                          \
  case N:                                                                                  \
    hipLaunchKernelGGL(trace_synth_kernel<N>, grid, dim3(256), 0, s, coef, planes, ntc, nt, \
                       nx, md, lam);                                                       \
    break;
  switch (md.n) {
    KFP_TS(1) KFP_TS(2) KFP_TS(3) KFP_TS(4) KFP_TS(5) KFP_TS(6) KFP_TS(7) KFP_TS(8)
    default:
      return hipErrorInvalidValue;
  }
#undef KFP_TS
  return hipGetLastError();
}

}  // namespace kfp
