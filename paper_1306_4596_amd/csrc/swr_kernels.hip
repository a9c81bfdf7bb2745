// gfx950 kernels of libkfpswr: the fused SWR time-step kernel and its helpers.
//
// The fused step kernel advances one subdomain's x-tile (64 columns, one per
// lane) by one time step of Section 6.2:
//   1. upwind x-transport (eqs. (6.4)/(6.5)) and the source term,
//   2. the implicit v-diffusion solve of eq. (6.2): one tridiagonal system per
//      column.  The unknown rows are split into P contiguous segments, one per
//      wavefront; each segment is eliminated locally (Thomas, precomputed
//      factors), the P-1 separator rows form a small tridiagonal system that
//      every lane solves from LDS, and two precomputed spike vectors correct
//      the segment values (a SPIKE-type partition of the same matrix).
// Before the step, the kernel also produces the interface data of the level
// it reads (eqs. (6.9)/(6.11)) and folds the level's mismatch (6.12) into the
// instance's residual, one step behind the march, so exchange and residual
// need no extra pass over the state.
//
// Memory layout: every field is [row][x] with x contiguous, so a wavefront's
// 64 lanes read 512 contiguous bytes per row.  All arithmetic is FP64.
#include <hip/hip_runtime.h>

#include "kfp_internal.h"

namespace kfp {

// ---------------------------------------------------------------------------
// interface traces and residual of time level n (1 <= n <= nt), from U^n
// ---------------------------------------------------------------------------
__device__ __forceinline__ void traces_and_residual(const StepTables &t, const SubDev &sd,
                                                    const InstDev &I, int n, int par, int lane,
                                                    int m, int mc, bool valid) {
  const int nx = I.nx;
  const size_t plane = (size_t)I.nt * nx;
  const size_t lvl = (size_t)(n - 1) * nx;
  const double *S = I.U[n & 1];
  const double *self = S + (size_t)sd.row_off * nx;
  double *lout = I.lam[par ^ 1];
  const double *lin = I.lam[par];
  const bool robin = I.tr == 1;
  if (sd.out_hi_plane >= 0) {  // Q_2 u_j at a_{j+1}, eq. (6.9)
    const double ua = self[(size_t)sd.out_hi_row * nx + mc];
    double v = ua;
    if (robin) {
      const double ua1 = self[(size_t)(sd.out_hi_row + 1) * nx + mc];
      v = I.q * ua - (ua1 - ua) / I.hv;
    }
    if (valid) lout[(size_t)sd.out_hi_plane * plane + lvl + m] = v;
  }
  if (sd.out_lo_plane >= 0) {  // Q_1 u_j at b_{j-1}, eq. (6.11)
    const double ub = self[(size_t)sd.out_lo_row * nx + mc];
    double v = ub;
    if (robin) {
      const double ub1 = self[(size_t)(sd.out_lo_row - 1) * nx + mc];
      v = I.p * ub + (ub - ub1) / I.hv;
    }
    if (valid) lout[(size_t)sd.out_lo_plane * plane + lvl + m] = v;
  }
  if (sd.res_nb >= 0) {  // (6.12) at the two end nodes of the overlap
    const SubDev nb = t.subs[sd.res_nb];
    const double *oth = S + (size_t)nb.row_off * nx;
    const double sa = self[(size_t)sd.out_hi_row * nx + mc];
    const double na = sd.res_row_a_nb >= 0 ? oth[(size_t)sd.res_row_a_nb * nx + mc]
                                           : lin[(size_t)sd.res_plane_a * plane + lvl + mc];
    const double sb = sd.res_row_b_self >= 0 ? self[(size_t)sd.res_row_b_self * nx + mc]
                                             : lin[(size_t)sd.res_plane_b * plane + lvl + mc];
    const double nbb = oth[(size_t)sd.res_row_b_nb * nx + mc];
    // non-negative doubles order like their bit patterns; NaN sorts above +inf
    unsigned long long ra = (unsigned long long)__double_as_longlong(fabs(sa - na));
    unsigned long long rb = (unsigned long long)__double_as_longlong(fabs(sb - nbb));
    unsigned long long r = valid ? (ra > rb ? ra : rb) : 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      unsigned long long o = __shfl_xor(r, off, 64);
      r = o > r ? o : r;
    }
    if (lane == 0) atomicMax(I.res, r);
  }
}

// Right-hand side of local row i for step n -> n+1.
__device__ __forceinline__ double row_rhs(const SubDev &sd, const InstDev &I, const RowCoef &c,
                                          int i, const double *src, const double *fr,
                                          const double *lin, size_t plane, int n, int mc,
                                          double gn) {
  const int nx = I.nx;
  if (i == 0 && sd.lo_kind == END_ROBIN)
    return lin[(size_t)sd.lam_lo * plane + (size_t)n * nx + mc];
  if (i == sd.n - 1 && sd.hi_kind == END_ROBIN)
    return lin[(size_t)sd.lam_hi * plane + (size_t)n * nx + mc];
  const double nu = c.nu;
  int mn = mc + (nu > 0.0 ? -1 : (nu < 0.0 ? 1 : 0));
  mn = mn < 0 ? mn + nx : (mn >= nx ? mn - nx : mn);
  const double w = fabs(nu);
  const double u = src[(size_t)i * nx + mc];
  const double un = src[(size_t)i * nx + mn];
  double val = (1.0 - w) * u + w * un + gn * fr[(size_t)i * nx + mc];
  if (i == 0 && sd.lo_kind == END_DIRI)
    val += I.r * lin[(size_t)sd.lam_lo * plane + (size_t)n * nx + mc];
  if (i == sd.n - 1 && sd.hi_kind == END_DIRI)
    val += I.r * lin[(size_t)sd.lam_hi * plane + (size_t)n * nx + mc];
  return val;
}

// Reduced (separator) system of one column, solved from LDS by each lane.
// Returns the separators below and above segment w.
template <int NW>
__device__ __forceinline__ void reduced_solve(const RedCoef *__restrict__ rc, int P, int w,
                                              int lane, const double (*sh_first)[64],
                                              const double (*sh_last)[64],
                                              const double (*sh_sep)[64], double &xlo,
                                              double &xhi) {
  double z[NW > 1 ? NW - 1 : 1];
  double prev = 0.0;
#pragma unroll
  for (int s = 0; s < NW - 1; ++s) {
    if (s < P - 1) {
      const RedCoef c = rc[s];
      const double D = sh_sep[s][lane] - c.ra * sh_last[s][lane] - c.rc * sh_first[s + 1][lane];
      prev = (s == 0) ? D * c.g1 : fma(c.g2, prev, D * c.g1);
      z[s] = prev;
    }
  }
  double nxt = 0.0;
#pragma unroll
  for (int s = NW - 2; s >= 0; --s) {
    if (s < P - 1) {
      nxt = (s == P - 2) ? z[s] : fma(rc[s].h, nxt, z[s]);
      z[s] = nxt;
    }
  }
  xlo = 0.0;
  xhi = 0.0;
#pragma unroll
  for (int s = 0; s < NW - 1; ++s) {
    if (s < P - 1) {
      if (s == w - 1) xlo = z[s];
      if (s == w) xhi = z[s];
    }
  }
}

// ---------------------------------------------------------------------------
// fused step kernel.  SEGMAX > 0: a segment lives in registers (<= SEGMAX
// rows); SEGMAX == 0: any segment length, intermediates staged in the output
// rows (global memory, cache-resident).
// ---------------------------------------------------------------------------
template <int SEGMAX, int NW>
__global__ __launch_bounds__(NW * 64) void step_kernel(StepTables t, int n, int par) {
  __shared__ double sh_first[NW][64];
  __shared__ double sh_last[NW][64];
  __shared__ double sh_sep[NW][64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int it = blockIdx.x; it < t.n_items; it += gridDim.x) {
    const Item item = t.items[it];
    const SubDev sd = t.subs[item.sub];
    const InstDev &I = t.inst[sd.inst];
    if (!I.active) continue;
    const int nx = I.nx;
    const int nt = I.nt;
    const int m = item.x0 + lane;
    const bool valid = m < nx;
    const int mc = valid ? m : nx - 1;
    if (w == 0 && n >= 1 && n <= nt) traces_and_residual(t, sd, I, n, par, lane, m, mc, valid);
    if (n >= nt) continue;

    const size_t plane = (size_t)nt * nx;
    const double *src = (n == 0) ? I.u0 + (size_t)sd.g_lo * nx : I.U[n & 1] + (size_t)sd.row_off * nx;
    double *dst = I.U[(n + 1) & 1] + (size_t)sd.row_off * nx;
    const double *fr = I.f + (size_t)sd.g_lo * nx;
    const double *lin = I.lam[par];
    const double gn = I.g[n];
    const RowCoef *__restrict__ rows = t.rows + sd.tab;
    const int P = sd.P;
    int s0 = 0, len = 0, blk = 0;
    if (w < P) {
      s0 = t.segs[sd.seg + w];
      len = t.segs[sd.seg + w + 1] - s0;
      blk = (w < P - 1) ? len - 1 : len;
    }
    double xlo = 0.0, xhi = 0.0;
    if constexpr (SEGMAX > 0) {
      double d[SEGMAX];
      if (w < P) {
#pragma unroll
        for (int k = 0; k < SEGMAX; ++k) {
          if (k < len) {
            const RowCoef c = rows[s0 + k];
            d[k] = row_rhs(sd, I, c, s0 + k, src, fr, lin, plane, n, mc, gn);
          }
        }
        // local forward elimination
        double y = 0.0;
#pragma unroll
        for (int k = 0; k < SEGMAX; ++k) {
          if (k < blk) {
            const RowCoef c = rows[s0 + k];
            y = (k == 0) ? d[k] * c.fa : fma(c.fb, y, d[k] * c.fa);
            d[k] = y;
          }
        }
        // local back substitution
        double x = 0.0;
#pragma unroll
        for (int k = SEGMAX - 1; k >= 0; --k) {
          if (k < blk) {
            x = (k == blk - 1) ? d[k] : fma(rows[s0 + k].bc, x, d[k]);
            d[k] = x;
          }
        }
        if (P > 1) {
          double last = 0.0, sep = 0.0;
#pragma unroll
          for (int k = 0; k < SEGMAX; ++k) {
            if (k == blk - 1) last = d[k];
            if (k == blk && k < len) sep = d[k];
          }
          sh_first[w][lane] = d[0];
          sh_last[w][lane] = last;
          sh_sep[w][lane] = sep;
        }
      }
      if (P > 1) {
        __syncthreads();
        if (w < P) reduced_solve<NW>(t.reds + sd.red, P, w, lane, sh_first, sh_last, sh_sep, xlo, xhi);
      }
      if (w < P && valid) {
#pragma unroll
        for (int k = 0; k < SEGMAX; ++k) {
          if (k < blk) {
            const RowCoef c = rows[s0 + k];
            const double v = fma(-c.sl, xlo, fma(-c.sr, xhi, d[k]));
            dst[(size_t)(s0 + k) * nx + m] = v;
          }
        }
        if (w < P - 1) dst[(size_t)(s0 + blk) * nx + m] = xhi;
      }
    } else {
      // global-staged variant for long segments
      if (w < P) {
        double y = 0.0, sep = 0.0;
        for (int k = 0; k < len; ++k) {
          const RowCoef c = rows[s0 + k];
          const double dk = row_rhs(sd, I, c, s0 + k, src, fr, lin, plane, n, mc, gn);
          if (k < blk) {
            y = (k == 0) ? dk * c.fa : fma(c.fb, y, dk * c.fa);
            dst[(size_t)(s0 + k) * nx + mc] = y;
          } else {
            sep = dk;
          }
        }
        double x = 0.0, first = 0.0, last = 0.0;
        for (int k = blk - 1; k >= 0; --k) {
          const double yk = dst[(size_t)(s0 + k) * nx + mc];
          x = (k == blk - 1) ? yk : fma(rows[s0 + k].bc, x, yk);
          dst[(size_t)(s0 + k) * nx + mc] = x;
          if (k == blk - 1) last = x;
        }
        first = x;
        if (P > 1) {
          sh_first[w][lane] = first;
          sh_last[w][lane] = last;
          sh_sep[w][lane] = sep;
        }
      }
      if (P > 1) {
        __syncthreads();
        if (w < P) {
          reduced_solve<NW>(t.reds + sd.red, P, w, lane, sh_first, sh_last, sh_sep, xlo, xhi);
          for (int k = 0; k < blk; ++k) {
            const RowCoef c = rows[s0 + k];
            const size_t o = (size_t)(s0 + k) * nx + mc;
            dst[o] = fma(-c.sl, xlo, fma(-c.sr, xhi, dst[o]));
          }
          if (w < P - 1) dst[(size_t)(s0 + blk) * nx + mc] = xhi;
        }
      }
      // Lanes past nx wrote duplicates of column nx-1 with identical values;
      // the clamp keeps every access inside the row.
    }
    __syncthreads();  // LDS is reused by the next item
  }
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__global__ void reset_res_kernel(const InstDev *inst, int n_inst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_inst && inst[i].active) *inst[i].res = 0ull;
}

__global__ void assemble_kernel(const double *__restrict__ U, const int *__restrict__ rowmap,
                                double *__restrict__ uT, int nv, int nx) {
  const size_t total = (size_t)(nv + 1) * nx;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / nx);
    const int m = (int)(e - (size_t)i * nx);
    const int r = rowmap[i];
    uT[e] = r >= 0 ? U[(size_t)r * nx + m] : 0.0;
  }
}

__global__ void fill_kernel(double *p, size_t n, double v) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    p[e] = v;
}

__global__ void copy_kernel(const double *__restrict__ s, double *__restrict__ d, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    d[e] = s[e];
}

__global__ void count_nonfinite_kernel(const double *__restrict__ p, size_t n, unsigned int *cnt) {
  unsigned int c = 0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    c += isfinite(p[e]) ? 0u : 1u;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(cnt, c);
}

// lambda^0(n) = Q(u0) at every interface node, for all time levels.
__global__ void u0_guess_kernel(const double *__restrict__ u0, int nx, int nt, int J,
                                const int *__restrict__ ab, int tr, double p, double hv,
                                double *__restrict__ lam) {
  const size_t plane = (size_t)nt * nx;
  const size_t total = (size_t)(J - 1) * plane;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / plane);
    const int m = (int)(e % nx);
    const size_t off = e - (size_t)j * plane;
    const int al = ab[2 * j], be = ab[2 * j + 1];
    const double ua = u0[(size_t)al * nx + m];
    const double ub = u0[(size_t)be * nx + m];
    double toR = ua, toL = ub;
    if (tr == 1) {
      const double ua1 = u0[(size_t)(al + 1) * nx + m];
      const double ub1 = u0[(size_t)(be - 1) * nx + m];
      toR = p * ua - (ua1 - ua) / hv;
      toL = p * ub + (ub - ub1) / hv;
    }
    lam[(size_t)(2 * j) * plane + off] = toR;
    lam[(size_t)(2 * j + 1) * plane + off] = toL;
  }
}

// Streaming copy, 16 B per lane per iteration (bandwidth probe).
__global__ void bw_probe_kernel(const double2 *__restrict__ s, double2 *__restrict__ d, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    d[e] = s[e];
}

static int grid_for(size_t n, int block) {
  size_t g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_reset_res(const InstDev *inst, int n_inst, hipStream_t s) {
  hipLaunchKernelGGL(reset_res_kernel, dim3((n_inst + 255) / 256), dim3(256), 0, s, inst, n_inst);
  return hipGetLastError();
}

hipError_t launch_assemble(const double *U, const int *rowmap, double *uT, int nv, int nx,
                           hipStream_t s) {
  const size_t n = (size_t)(nv + 1) * nx;
  hipLaunchKernelGGL(assemble_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, U, rowmap, uT, nv,
                     nx);
  return hipGetLastError();
}

hipError_t launch_fill(double *p, size_t n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_copy(const double *src, double *dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_count_nonfinite(const double *p, size_t n, unsigned int *count, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(count_nonfinite_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, count);
  return hipGetLastError();
}

hipError_t launch_u0_guess(const double *u0, int nx, int nt, int J, const int *ab, int tr,
                           double p, double hv, double *lam, hipStream_t s) {
  const size_t n = (size_t)(J - 1) * nt * nx;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(u0_guess_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, u0, nx, nt, J, ab,
                     tr, p, hv, lam);
  return hipGetLastError();
}

hipError_t launch_bw_probe(const void *src, void *dst, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 16;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(bw_probe_kernel, dim3(grid_for(n, 256) < 8192 ? grid_for(n, 256) : 8192),
                     dim3(256), 0, s, (const double2 *)src, (double2 *)dst, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dispatch over the compiled (waves, seg_max) configurations
// ---------------------------------------------------------------------------
#define KFP_STEP_CONFIGS(X) \
  X(1, 0) X(1, 8) X(1, 16) X(1, 24) X(1, 32) X(1, 48) X(1, 64) \
  X(2, 0) X(2, 8) X(2, 16) X(2, 24) X(2, 32) X(2, 48) X(2, 64) \
  X(4, 0) X(4, 8) X(4, 16) X(4, 24) X(4, 32) X(4, 48) X(4, 64) \
  X(8, 0) X(8, 8) X(8, 16) X(8, 24) X(8, 32) X(8, 48) \
  X(16, 0) X(16, 8) X(16, 16) X(16, 24) X(16, 32)

bool step_config_supported(int waves, int seg_max) {
#define KFP_CHECK(W, S) \
  if (waves == W && seg_max == S) return true;
  KFP_STEP_CONFIGS(KFP_CHECK)
#undef KFP_CHECK
  return false;
}

hipError_t launch_step(const StepTables &t, int waves, int seg_max, int n, int par, int grid,
                       hipStream_t s) {
#define KFP_LAUNCH(W, S)                                                                  \
  if (waves == W && seg_max == S) {                                                      \
    hipLaunchKernelGGL((step_kernel<S, W>), dim3(grid), dim3(W * 64), 0, s, t, n, par); \
    return hipGetLastError();                                                            \
  }
  KFP_STEP_CONFIGS(KFP_LAUNCH)
#undef KFP_LAUNCH
  return hipErrorInvalidValue;
}

}  // namespace kfp
