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

#include <cfloat>
#include <type_traits>

#include "kfp_internal.h"

namespace kfp {

template <class T>
using KConst = __attribute__((address_space(4))) const T;
template <class T>
__device__ __forceinline__ KConst<T> *as_const(const T *p) {
  return (KConst<T> *)p;
}

template <class T>
using KGlob = __attribute__((address_space(1))) T;
template <class T>
__device__ __forceinline__ KGlob<T> *as_glob(T *p) {
  return (KGlob<T> *)p;
}

// Copy of a descriptor from the constant address space (scalar loads), in
// words as wide as its alignment so that pointers stay whole.
template <class W, int N>
struct Words {
  W w[N];
};
template <class T>
__device__ __forceinline__ T load_const(KConst<T> *p) {
  using W = typename std::conditional<alignof(T) >= 8 && sizeof(T) % 8 == 0,
                                      unsigned long long, unsigned>::type;
  static_assert(sizeof(T) % sizeof(W) == 0, "descriptor size");
  constexpr int N = sizeof(T) / sizeof(W);
  Words<W, N> v;
  KConst<W> *q = reinterpret_cast<KConst<W> *>(p);
#pragma unroll
  for (int i = 0; i < N; ++i) v.w[i] = q[i];
  return __builtin_bit_cast(T, v);
}

// The instance descriptor holds pointers: copy it field by field, so that
// every pointer is loaded with its own type and the copy stays in registers.
__device__ __forceinline__ InstDev load_inst(KConst<InstDev> *p) {
  InstDev I;
  I.U[0] = p->U[0];
  I.U[1] = p->U[1];
  I.u0 = p->u0;
  I.f = p->f;
  I.g = p->g;
  I.lam[0] = p->lam[0];
  I.lam[1] = p->lam[1];
  I.res = p->res;
  I.V = p->V;
  I.r = p->r;
  I.p = p->p;
  I.q = p->q;
  I.hv = p->hv;
  I.nx = p->nx;
  I.nv = p->nv;
  I.nt = p->nt;
  I.tr = p->tr;
  I.active = p->active;
  I.nonovl = p->nonovl;
  I.xmode = p->xmode;
  I.scheme = p->scheme;
  I.gconst = p->gconst;
  return I;
}

// ---------------------------------------------------------------------------
// interface traces and residual of time level n (1 <= n <= nt), from U^n
// ---------------------------------------------------------------------------
// S: state U^n of the instance; lin / lout: trace windows read / written.
__device__ __forceinline__ void traces_and_residual(const StepTables &t, const SubDev &sd,
                                                    const InstDev &I, const double *S,
                                                    const double *lin, double *lout, int n,
                                                    int lane, int m, int mc, bool valid) {
  const int nx = I.nx;
  const size_t plane = (size_t)I.nt * nx;
  const size_t lvl = (size_t)(n - 1) * nx;
  const double *self = S + (size_t)sd.row_off * nx;
  const bool robin = I.tr == 1;
  // without overlap the derivative in Q comes from the subdomain's own Robin
  // condition at the shared node: Q_2 u_j = (p+q) u_j - lambda_1 and
  // Q_1 u_{j+1} = (p+q) u_{j+1} - lambda_2, with the traces it was solved with
  if (sd.out_hi_plane >= 0) {  // Q_2 u_j at a_{j+1}, eq. (6.9)
    const double ua = self[(size_t)sd.out_hi_row * nx + mc];
    double v = ua;
    if (I.nonovl) {
      v = (I.p + I.q) * ua - lin[(size_t)sd.lam_hi * plane + lvl + mc];
    } else if (robin) {
      const double ua1 = self[(size_t)(sd.out_hi_row + 1) * nx + mc];
      v = I.q * ua - (ua1 - ua) / I.hv;
    }
    if (valid) lout[(size_t)sd.out_hi_plane * plane + lvl + m] = v;
  }
  if (sd.out_lo_plane >= 0) {  // Q_1 u_j at b_{j-1}, eq. (6.11)
    const double ub = self[(size_t)sd.out_lo_row * nx + mc];
    double v = ub;
    if (I.nonovl) {
      v = (I.p + I.q) * ub - lin[(size_t)sd.lam_lo * plane + lvl + mc];
    } else if (robin) {
      const double ub1 = self[(size_t)(sd.out_lo_row - 1) * nx + mc];
      v = I.p * ub + (ub - ub1) / I.hv;
    }
    if (valid) lout[(size_t)sd.out_lo_plane * plane + lvl + m] = v;
  }
  if (sd.res_nb >= 0) {  // (6.12) at the two end nodes of the overlap
    const SubDev nb = load_const(as_const(t.subs) + sd.res_nb);
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

// Weight of the incoming trace in the right-hand side of an end row taking
// boundary data: a Robin row is the trace itself; a row next to a classical
// interface node moves r times that node's value over; a half-cell row
// (no overlap) gains the flux 2 dt / h_v times the trace.
__device__ __forceinline__ double end_scale(int kind, const InstDev &I) {
  return kind == END_ROBIN ? 1.0 : (kind == END_RFV ? 2.0 * I.r * I.hv : I.r);
}

// Right-hand side of local row i for step n -> n+1.
__device__ __forceinline__ double row_rhs(const SubDev &sd, const InstDev &I, const RowCoef &c,
                                          int i, KGlob<const double> *src,
                                          KGlob<const double> *fr, KGlob<const double> *lin,
                                          size_t plane, int n, int mc, double gn) {
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
  if (i == 0 && (sd.lo_kind == END_DIRI || sd.lo_kind == END_RFV))
    val += end_scale(sd.lo_kind, I) * lin[(size_t)sd.lam_lo * plane + (size_t)n * nx + mc];
  if (i == sd.n - 1 && (sd.hi_kind == END_DIRI || sd.hi_kind == END_RFV))
    val += end_scale(sd.hi_kind, I) * lin[(size_t)sd.lam_hi * plane + (size_t)n * nx + mc];
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
    const Item item = load_const(as_const(t.items) + it);
    const SubDev sd = load_const(as_const(t.subs) + item.sub);
    KConst<InstDev> *ip = as_const(t.inst) + sd.inst;
    const InstDev I = load_inst(ip);
    if (!I.active) continue;
    // ping-pong buffers picked in constant memory (n and par are uniform)
    const double *Ucur = ip->U[n & 1];
    double *Unext = ip->U[(n + 1) & 1];
    const double *lam_in = ip->lam[par];
    double *lam_out = ip->lam[par ^ 1];
    const int nx = I.nx;
    const int nt = I.nt;
    const int m = item.x0 + lane;
    const bool valid = m < nx;
    const int mc = valid ? m : nx - 1;
    if (w == 0 && n >= 1 && n <= nt)
      traces_and_residual(t, sd, I, Ucur, lam_in, lam_out, n, lane, m, mc, valid);
    if (n >= nt) continue;

    const size_t plane = (size_t)nt * nx;
    KGlob<const double> *src = as_glob((n == 0) ? I.u0 + (size_t)sd.g_lo * nx
                                                : Ucur + (size_t)sd.row_off * nx);
    KGlob<double> *dst = as_glob(Unext + (size_t)sd.row_off * nx);
    KGlob<const double> *fr = as_glob(I.f + (size_t)sd.g_lo * nx);
    KGlob<const double> *lin = as_glob(lam_in);
    const double gn = as_const(I.g)[n];  // scalar load: no vector-memory wait
    KConst<RowCoef> *rows = as_const(t.rows) + sd.tab;
    KConst<int> *segs = as_const(t.segs);
    const int P = sd.P;
    int s0 = 0, len = 0, blk = 0;
    if (w < P) {
      s0 = segs[sd.seg + w];
      len = segs[sd.seg + w + 1] - s0;
      blk = (w < P - 1) ? len - 1 : len;
    }
    double xlo = 0.0, xhi = 0.0;
    if constexpr (SEGMAX > 0) {
      double d[SEGMAX];
      if (w < P) {
        // rows past the segment re-read its last row, so every load is
        // unconditional and the whole segment's loads are in flight at once
#pragma unroll
        for (int k = 0; k < SEGMAX; ++k) {
          const int i = s0 + (k < len ? k : len - 1);
          const double nu = rows[i].nu;
          int mn = mc + (nu > 0.0 ? -1 : (nu < 0.0 ? 1 : 0));
          mn = mn < 0 ? mn + nx : (mn >= nx ? mn - nx : mn);
          const double wgt = fabs(nu);
          const double u = src[(size_t)i * nx + mc];
          const double un = src[(size_t)i * nx + mn];
          d[k] = (1.0 - wgt) * u + wgt * un + gn * fr[(size_t)i * nx + mc];
        }
        if (w == 0 && sd.lo_kind != END_PHYS) {
          const double l = lin[(size_t)sd.lam_lo * plane + (size_t)n * nx + mc];
          d[0] = sd.lo_kind == END_ROBIN ? l : d[0] + end_scale(sd.lo_kind, I) * l;
        }
        if (w == P - 1 && sd.hi_kind != END_PHYS) {
          const double l = lin[(size_t)sd.lam_hi * plane + (size_t)n * nx + mc];
          const double sc = end_scale(sd.hi_kind, I);
#pragma unroll
          for (int k = 0; k < SEGMAX; ++k)
            if (k == len - 1) d[k] = sd.hi_kind == END_ROBIN ? l : d[k] + sc * l;
        }
        // local forward elimination
        double y = 0.0;
#pragma unroll
        for (int k = 0; k < SEGMAX; ++k) {
          if (k < blk) {
            const RowCoef c = load_const(rows + s0 + k);
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
            const RowCoef c = load_const(rows + s0 + k);
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
          const RowCoef c = load_const(rows + s0 + k);
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
            const RowCoef c = load_const(rows + s0 + k);
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
// multi-step (temporally blocked) march kernel.  A workgroup owns one
// subdomain's tile of 64 x-columns (one per lane) including a halo of H
// columns on each side, keeps its column segments and the source rows in
// registers, and advances S <= H steps without leaving the chip: the upwind
// neighbour comes from the adjacent lane, and every step the valid lanes
// shrink by one on each side, so lanes H .. 63-H are exact after S steps.
// Interface-node values of every level go to value planes; the exchange
// pass turns them into traces and the residual.
// ---------------------------------------------------------------------------
// Upwind neighbour of every lane: lane i receives lane i-1 (v > 0, the cell
// at m-1) or lane i+1 (v < 0, the cell at m+1) through a wave-wide DPP shift;
// the edge lane, which has no neighbour in the wave, reads 0 (it is halo).
__device__ __forceinline__ double from_lower_lane(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_upper_lane(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

// A wave-uniform double moved to scalar registers (FP64 vector instructions
// take it as a scalar operand, so it holds no vector register).
__device__ __forceinline__ double wave_uniform(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// A wave's column segment of SEG <= 48 rows held in registers.  Up to three
// vectors of at most 16 doubles, so that a wave-uniform run-time index
// compiles to relative register addressing (longer vectors would be spilled
// to scratch).
template <int SEG>
struct SegRegs {
  static constexpr int NA = SEG < 16 ? SEG : 16;
  static constexpr int NB = SEG > 32 ? 16 : (SEG > 16 ? SEG - 16 : 1);
  static constexpr int NC = SEG > 32 ? SEG - 32 : 1;
  typedef double va __attribute__((ext_vector_type(NA)));
  typedef double vb __attribute__((ext_vector_type(NB)));
  typedef double vc __attribute__((ext_vector_type(NC)));
  va a;
  vb b;
  vc c;
  template <int K>
  __device__ __forceinline__ double ld() const {
    if constexpr (K < 16) return a[K];
    else if constexpr (K < 32) return b[K - 16];
    else return c[K - 32];
  }
  template <int K>
  __device__ __forceinline__ void st(double v) {
    if constexpr (K < 16) a[K] = v;
    else if constexpr (K < 32) b[K - 16] = v;
    else c[K - 32] = v;
  }
  __device__ __forceinline__ double get(int k) const {
    if (SEG <= 16 || k < 16) return a[k];
    if (SEG <= 32 || k < 32) return b[k - 16];
    return c[k - 32];
  }
};

template <int K, int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (K < N) {
    f(std::integral_constant<int, K>{});
    static_for<K + 1, N>(f);
  }
}

// Upwind direction of a wave's rows: all v < 0 (neighbour at m+1), all
// v >= 0 (neighbour at m-1), or mixed (the wave holding v = 0).
enum Dir : int { DIR_UP = 0, DIR_LO = 1, DIR_MIX = 2 };

// Segments longer than this keep only the state in registers and re-read
// the (cache-resident) source rows every step.
constexpr int kFRegMax = 33;

// Upper bound of the steps one multi-step launch takes (checked by the host).
constexpr int kMaxStepsPerLaunch = 24;

// Transport, source and forward elimination of one step.  The elimination
// starts from y = blo, the boundary data of row 0 of the subdomain (zero in
// every other wave): the first real row of each segment has multiplier 1,
// and the padding rows in front of it pass y on unchanged, so the data
// lands on that row without a per-row test.  mc: the wave's coefficient
// rows in LDS (wave-uniform addresses: broadcast reads).
template <int SEG, int NW, int DIR>
__device__ __forceinline__ void march_forward(SegRegs<SEG> &d, const SegRegs<SEG> &fs,
                                              const MarchCoef *mc, double gn, double blo,
                                              double bhi, int vsplit,
                                              KGlob<const double> *fr, int base, int nx,
                                              int col) {
  double y = blo;
  static_for<0, SEG>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const double u = d.template ld<k>();
    double nb;
    if constexpr (DIR == DIR_LO) {
      nb = from_lower_lane(u);
    } else if constexpr (DIR == DIR_UP) {
      nb = from_upper_lane(u);
    } else {
      const double a = from_lower_lane(u), c = from_upper_lane(u);
      nb = (k >= vsplit) ? a : c;
    }
    double fk;
    if constexpr (SEG <= kFRegMax) {
      fk = fs.template ld<k>();
    } else {
      fk = mc[k].fa * fr[(size_t)max(base + k, 0) * nx + col];
    }
    double tk = fma(mc[k].alpha, u, fma(mc[k].beta, nb, gn * fk));
    if constexpr (k == SEG - 1) tk += bhi;
    y = fma(mc[k].fb, y, tk);
    d.template st<k>(y);
  });
}

// Finite elements, first half of a step: G_k = T W^n + dt s f in every
// register (DIR_NONE at the first step of a solve: nothing transported yet).
// The Courant number of register k is nu0 + k dnu (no table read: the pass
// issues no LDS loads and waits on none).
constexpr int DIR_NONE = 3;
template <int SEG, int DIR>
__device__ __forceinline__ void fem_stage(SegRegs<SEG> &d, const SegRegs<SEG> &fs, double nu0,
                                          double dnu, double gn, int vsplit,
                                          KGlob<const double> *fr, int base, int nx, int col) {
  static_for<0, SEG>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const double u = d.template ld<k>();
    double fk;
    if constexpr (SEG <= kFRegMax)
      fk = fs.template ld<k>();
    else
      fk = fr[(size_t)max(base + k, 0) * nx + col];
    double g;
    if constexpr (DIR == DIR_NONE) {
      g = fma(gn, fk, u);
    } else {
      double nb;
      if constexpr (DIR == DIR_LO) {
        nb = from_lower_lane(u);
      } else if constexpr (DIR == DIR_UP) {
        nb = from_upper_lane(u);
      } else {
        const double a = from_lower_lane(u), c = from_upper_lane(u);
        nb = (k >= vsplit) ? a : c;
      }
      const double w = fabs(fma((double)k, dnu, nu0));
      g = fma(w, nb - u, fma(gn, fk, u));
    }
    d.template st<k>(g);
  });
}

// G of one node outside the segment (its state u in every lane): signed
// Courant number nu, source value fv.
__device__ __forceinline__ double fem_edge_g(double u, double nu, double gn, double fv,
                                             bool first) {
  const double lo = from_lower_lane(u), up = from_upper_lane(u);
  if (first) return fma(gn, fv, u);
  const double w = fabs(nu);
  const double nb = nu > 0.0 ? lo : (nu < 0.0 ? up : u);
  return fma(1.0 - w, u, fma(w, nb, gn * fv));
}

// Finite elements, second half: forward elimination with the mass-matrix
// right-hand side.  ylo: the starting value (boundary data and the G of the
// node below, already weighted); bhi: the same for the last register.
// The coefficients of row k+2 are loaded before row k is computed (LDS
// reads return in order, so the wait for a row's coefficients overlaps two
// rows of arithmetic); the scheduling barrier keeps the loads in that
// order.  (The same in the finite-difference pass made it slower: there the
// compiler's own placement already hides most of the latency.)
struct FemRow {
  double wl, wm, wu, fb;
};
__device__ __forceinline__ FemRow fem_row(const FemCoef *mc, int k) {
  return FemRow{mc[k].wl, mc[k].wm, mc[k].wu, mc[k].fb};
}
template <int SEG, bool AHEAD = true>
__device__ __forceinline__ void fem_forward(SegRegs<SEG> &d, const FemCoef *mc, double ylo,
                                            double bhi) {
  double y = ylo;
  double gprev = 0.0;
  FemRow c0 = fem_row(mc, 0);
  FemRow c1 = fem_row(mc, SEG > 1 ? 1 : 0);
  static_for<0, SEG>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    FemRow c;
    if constexpr (AHEAD) {
      c = c0;
      c0 = c1;
      if constexpr (k + 2 < SEG) c1 = fem_row(mc, k + 2);
      __builtin_amdgcn_sched_barrier(0x1);  // arithmetic may cross, memory operations not
    } else {
      c = fem_row(mc, k);
    }
    const double gk = d.template ld<k>();
    double t = c.wm * gk;
    if constexpr (k > 0) t = fma(c.wl, gprev, t);
    if constexpr (k < SEG - 1)
      t = fma(c.wu, d.template ld<k + 1>(), t);
    else
      t += bhi;
    gprev = gk;
    y = fma(c.fb, y, t);
    d.template st<k>(y);
  });
}

// G lane groups per wavefront: a wavefront holds G segments of a subdomain,
// each for a tile of 64/G x-columns (lanes g*64/G .. (g+1)*64/G - 1 hold
// segment w*G + g).  G = 1 is one segment per wavefront over 64 columns;
// G > 1 lets a workgroup hold G times the rows of one whose wavefronts each
// hold a single segment, for subdomains too tall for the register file of
// one 64-column tile, at the cost of a narrower tile.  The upwind shift runs
// across the whole wavefront: the edge lane of a group then receives a
// value of the neighbouring group, which is halo like the zero the edge
// lane of the wavefront receives, and the valid lanes never see it.
// OCC: wavefronts per SIMD the register allocation must allow (1: no limit
// beyond one workgroup).  A build of the same code for more resident
// workgroups, for launches with several work items per compute unit.
// FEM: the finite-element scheme (FemCoef tables; the step forms G in every
// register first, then eliminates with the mass-matrix right-hand side; the
// G of the node below a segment comes from that node's state, which the
// lane holds: the separator value the reduced system gave it, or the fixed
// node's trace; the separator's G of the node above enters the reduced
// system from LDS).
template <int SEG, int NW, int G, int OCC = 1, bool FEM = false>
__global__ __launch_bounds__(NW * 64, OCC) void march_kernel(StepTables t, int n0_in, int S,
                                                             int H, int src_in, int par) {
  static_assert(G == 1 || G == 2 || G == 4, "lane groups");
  using MC = typename std::conditional<FEM, FemCoef, MarchCoef>::type;
  constexpr int NV = NW * G;  // segments per workgroup
  constexpr int TW = 64 / G;  // tile columns
  // The reduced (separator) system.  Finite elements in workgroups of at
  // most 8 segments (RR):
  // each segment forms its own parts of the reduced right-hand sides before
  // the barrier, E_v = sep_v - ra_v last_v and F_v = -rc_{v-1} first_v (with
  // finite elements + rg_{v-1} G(first_v)), and each lane keeps the two rows
  // of the reduced inverse it needs in registers for the whole item, so the
  // sum after the barrier reads two LDS values per separator and no
  // coefficient, with no branch (per launch 64.9 -> 51.8 us on 1024 x 1024,
  // J = 8).  Otherwise the segment end values and the inverse are staged in
  // LDS: wider workgroups, longer segments and the builds limited in
  // registers would spill, and the finite-difference kernel measured no
  // gain (44.8 against 44.2 us).  Either way the values are double-buffered by step parity: a step's
  // writes never meet the previous step's reads, so one barrier per step
  // suffices.
  constexpr bool RR = FEM && NV <= 8 && OCC == 1 && SEG <= 17;
  constexpr int NB = RR ? 1 : 2, NS = RR ? 1 : NV, NT = RR ? 1 : TW;
  constexpr int EB = RR ? 2 : 1, ES = RR ? NV : 1, ET = RR ? TW : 1;
  __shared__ double sh_first[NB][NS][NT];
  __shared__ double sh_last[NB][NS][NT];
  __shared__ double sh_sep[NB][NS][NT];
  __shared__ double sh_E[EB][ES][ET];
  __shared__ double sh_F[EB][ES][ET];
  // boundary data of the launch's steps (low end, high end), staged once so
  // that the step loop issues no vector loads: its stores then never hold a
  // step up, since nothing in the loop waits on vector memory
  __shared__ double sh_bd[2][kMaxStepsPerLaunch][TW];
  // the work item's coefficient rows (per segment), reduced system and
  // source factors, staged once per item: the step loop then issues no
  // scalar loads either, and LDS reads (returned in order) can be waited on
  // one by one, so they are issued well ahead of their use
  __shared__ MC sh_mc[NV][SEG];
  __shared__ RedCoef sh_rc[RR ? 1 : NV];
  // finite elements, wider workgroups: G of every segment's first real row,
  // for the separator below it (double-buffered like the values above)
  constexpr bool GF = FEM && !RR;
  __shared__ double sh_gf[GF ? 2 : 1][GF ? NV : 1][GF ? TW : 1];
  __shared__ double sh_rinv[RR ? 1 : (NV - 1) * (NV - 1) + 1];
  __shared__ double sh_g[NW][kMaxStepsPerLaunch];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gh = G == 1 ? 0 : lane / TW;  // lane group
  const int tl = G == 1 ? lane : lane % TW;  // column within the tile
  const int v = w * G + gh;               // this lane's segment
  KConst<Item> *items = as_const(t.items);
  KConst<SubDev> *subs = as_const(t.subs);
  KConst<InstDev> *insts = as_const(t.inst);
  for (int it = blockIdx.x; it < t.n_items; it += gridDim.x) {
    const int sub = items[it].sub;
    const int x0 = items[it].x0;
    KConst<SubDev> *sd = subs + sub;
    KConst<InstDev> *I = insts + sd->inst;
    if (!I->active) continue;
    int n0 = n0_in, src_par = src_in;
    if (t.blk) {  // pipelined iterations: this instance's block of this launch
      const int b = as_const(t.blk)[sd->inst];
      if (b < 0) continue;
      n0 = b * S;
      src_par = b & 1;
    }
    const int nx = I->nx;
    const int nt = I->nt;
    if (n0 >= nt) continue;
    const int steps = min(min(S, kMaxStepsPerLaunch), nt - n0);  // S is checked by the host
    const int rel = tl - H;
    int col = (x0 + rel) % nx;
    if (col < 0) col += nx;
    const bool out = rel >= 0 && rel < TW - 2 * H && x0 + rel < nx;
    const size_t plane = (size_t)nt * nx;
    const int n_rows = sd->n;
    const int row_off = sd->row_off;
    const int g_lo = sd->g_lo;
    KGlob<const double> *src = as_glob((n0 == 0) ? I->u0 + (size_t)g_lo * nx
                                                 : I->U[src_par] + (size_t)row_off * nx);
    KGlob<double> *dst = as_glob(I->U[src_par ^ 1] + (size_t)row_off * nx);
    KGlob<const double> *fr = as_glob(I->f + (size_t)g_lo * nx);
    KGlob<const double> *lin = as_glob((const double *)I->lam[par]);
    KGlob<double> *Vbase = as_glob(I->V);
    const double rr = I->r;
    const bool robin = I->tr == 1;
    const int P = sd->P;
    const int pad = sd->pad;
    // segments of this wavefront that hold rows: w*G .. w*G + nseg - 1
    const int nseg = min(G, P - w * G);
    const bool wave_active = nseg > 0;
    const bool active = v < P;
    const bool last = v == P - 1;
    // the last segment ends on the subdomain's last row: its first `pad`
    // registers repeat rows of the segment before it
    auto first_reg = [&](int vv) { return vv == P - 1 ? pad : 0; };
    auto seg_base = [&](int vv) { return vv * SEG - first_reg(vv); };
    const int k0 = first_reg(v);  // first real row in this lane's registers
    const int base = seg_base(v);  // local row of register k is base + k
    // rows with local index >= vsplit have v >= 0: upwind neighbour at m-1
    const int vsplit = sd->vsplit - base;
    // one direction for the whole wavefront when all its segments agree
    const int vs_first = sd->vsplit - seg_base(w * G);
    const int vs_last = sd->vsplit - seg_base(w * G + (nseg > 0 ? nseg - 1 : 0));
    const int dir = vs_first <= 0 ? DIR_LO : (vs_last >= SEG ? DIR_UP : DIR_MIX);
    const int lo_kind = sd->lo_kind, hi_kind = sd->hi_kind;
    const int lam_lo = sd->lam_lo, lam_hi = sd->lam_hi;
    const int out_hi_plane = sd->out_hi_plane, out_hi_row = sd->out_hi_row;
    const int out_lo_plane = sd->out_lo_plane, out_lo_row = sd->out_lo_row;
    // end rows taking boundary data: row 0 in segment 0, row n-1 in the last
    const bool lo_end = active && v == 0 && lo_kind != END_PHYS;
    const bool hi_end = active && last && hi_kind != END_PHYS;
    KGlob<const double> *lin_lo = lin + (size_t)(lam_lo > 0 ? lam_lo : 0) * plane + col;
    KGlob<const double> *lin_hi = lin + (size_t)(lam_hi > 0 ? lam_hi : 0) * plane + col;
    // staging: each wave copies its own segments' rows, factors and boundary
    // data (written and read by the same wave: no barrier); the reduced
    // system is copied by wave 0 and first read after the step's first
    // barrier (the previous item's last reads ended at its last step's
    // second barrier)
    const MC *mc = sh_mc[v];
    if (wave_active) {
      const MC *tab = FEM ? (const MC *)t.frows : (const MC *)t.mrows;
      KGlob<const double> *ct = as_glob((const double *)(tab + sd->tab + w * G * SEG));
      double *cs = reinterpret_cast<double *>(sh_mc[w * G]);
      constexpr int NDB = (int)(sizeof(MC) / sizeof(double));
      const int ncw = nseg * SEG * NDB;  // rows past the table's end are not read
#pragma unroll
      for (int e0 = 0; e0 < G * SEG * NDB; e0 += 64)
        if (e0 + lane < ncw) cs[e0 + lane] = ct[e0 + lane];
      KGlob<const double> *gt = as_glob(I->g);
      if (lane < steps) sh_g[w][lane] = gt[n0 + lane];
      if (!RR && w == 0 && P > 1) {
        constexpr int NRW = (int)(sizeof(RedCoef) / sizeof(double));
        KGlob<const double> *rt = as_glob((const double *)(t.reds + sd->red));
        double *rs = reinterpret_cast<double *>(sh_rc);
        for (int e = lane; e < (P - 1) * NRW; e += 64) rs[e] = rt[e];
        KGlob<const double> *rv = as_glob(t.rinv + sd->rinv);
        for (int e = lane; e < (P - 1) * (P - 1); e += 64) sh_rinv[e] = rv[e];
      }
      if (lo_end)
        for (int s = 0; s < steps; ++s) sh_bd[0][s][tl] = lin_lo[(size_t)(n0 + s) * nx];
      if (hi_end)
        for (int s = 0; s < steps; ++s) sh_bd[1][s][tl] = lin_hi[(size_t)(n0 + s) * nx];
    }
    // RR: rows v-1 and v of the reduced inverse (zero past the subdomain's
    // separators), this segment's separator coefficient ra_v and the
    // coefficients rc_{v-1}, rg_{v-1} of the separator below; the slots of
    // segments the subdomain does not use are zeroed, so the branch-free sum
    // only adds zeros for them
    constexpr int NR1 = RR && NV > 1 ? NV - 1 : 1;
    double RL[NR1], RH[NR1];
    double ra_s = 0.0, rc_s = 0.0, rg_s = 0.0;
    if constexpr (RR) {
#pragma unroll
      for (int q = 0; q < NR1; ++q) RL[q] = RH[q] = 0.0;
      if (P > 1) {
        if (active) {
          const int m = P - 1;
          KGlob<const double> *rv = as_glob(t.rinv + sd->rinv);
#pragma unroll
          for (int q = 0; q < NV - 1; ++q) {
            if (q < m) {
              if (v > 0) RL[q] = rv[(size_t)(v - 1) * m + q];
              if (v < m) RH[q] = rv[(size_t)v * m + q];
            }
          }
          KGlob<const double> *rt = as_glob((const double *)(t.reds + sd->red));
          constexpr int NRW = (int)(sizeof(RedCoef) / sizeof(double));
          if (v < m) ra_s = rt[(size_t)v * NRW + 0];
          if (v > 0) {
            rc_s = rt[(size_t)(v - 1) * NRW + 1];
            rg_s = rt[(size_t)(v - 1) * NRW + 5];
          }
        } else if (v < NV) {
          sh_E[0][v][tl] = sh_E[1][v][tl] = 0.0;
          sh_F[0][v][tl] = sh_F[1][v][tl] = 0.0;
        }
      }
    }
    double gf1 = 0.0;  // finite elements, RR: G of the first real row
    SegRegs<SEG> d, fs;
    if (active) {
      static_for<0, SEG>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const int r = max(base + k, 0);
        d.template st<k>(src[(size_t)r * nx + col]);
        if constexpr (SEG <= kFRegMax) {
          if constexpr (FEM)
            fs.template st<k>(fr[(size_t)r * nx + col]);
          else
            fs.template st<k>(mc[k].fa * fr[(size_t)r * nx + col]);
        }
      });
    }
    // weight of the incoming trace in an end row: finite differences: 1 (a
    // Robin row), 2 dt / h_v (half-cell row), r (next to a fixed node);
    // finite elements (rows times dt / h_v): dt / h_v for a Robin row with or
    // without overlap (a natural condition), r - 1/6 next to a fixed node
    const double rfv = 2.0 * rr * I->hv;
    auto end_w = [&](int kind) {
      if constexpr (FEM)
        return kind == END_DIRI ? rr - 1.0 / 6.0 : rr * I->hv;
      else
        return kind == END_ROBIN ? 1.0 : (kind == END_RFV ? rfv : rr);
    };
    const double lo_scale = lo_end ? mc[k0].fab * end_w(lo_kind) : 0.0;
    const double hi_scale = hi_end ? mc[SEG - 1].fab * end_w(hi_kind) : 0.0;
    // finite elements: the nodes next to the segment (below its first real
    // row; above the subdomain's last row), their source values and states
    double nul = 0.0, wol = 0.0, nua = 0.0, woa = 0.0;
    double fbelow = 0.0, ubelow = 0.0, fabove = 0.0, uabove = 0.0;
    // Courant number of register k: nu0 + k dnu, v_i = -1 + i h_v, dt/h_x = r h_v^2 nx
    const double dtx = rr * I->hv * I->hv * nx;
    const double dnu = I->hv * dtx;
    const double nu0_item = (-1.0 + (g_lo + base) * I->hv) * dtx;
    if constexpr (FEM) {
      if (active) {
        KGlob<const double> *fsg = as_glob((const double *)(t.fsegs + sd->seg + v));
        nul = fsg[0];
        wol = fsg[1];
        nua = fsg[2];
        woa = fsg[3];
        const int rb = base + k0 - 1;  // local row below the first real row
        KGlob<const double> *f0 = as_glob(I->f);
        KGlob<const double> *u00 = as_glob(I->u0);
        if (wol != 0.0) {
          fbelow = f0[(size_t)(g_lo + rb) * nx + col];
          if (rb >= 0)
            ubelow = src[(size_t)rb * nx + col];
          else
            ubelow = n0 == 0 ? u00[(size_t)(g_lo - 1) * nx + col] : lin_lo[(size_t)(n0 - 1) * nx];
        }
        if (woa != 0.0) {
          fabove = f0[(size_t)(g_lo + n_rows) * nx + col];
          uabove = n0 == 0 ? u00[(size_t)(g_lo + n_rows) * nx + col]
                           : lin_hi[(size_t)(n0 - 1) * nx];
        }
      }
    }
    // register `pad` of every lane (a wave-uniform index): the first real row
    // of the last segment
    auto first_value = [&](const SegRegs<SEG> &dd) {
      // finite differences: the back substitution copies the first real row
      // into the padding registers below it (their bc is 1), so after it
      // register 0 holds that row in every segment
      if constexpr (!FEM) return dd.template ld<0>();
      if constexpr (G == 1) {
        return dd.get(k0);
      } else {
        const double a = dd.get(pad);
        return k0 != 0 ? a : dd.template ld<0>();
      }
    };
    // value of local row R to *p from the lanes holding it: the segments of
    // this wave are walked with wave-uniform register indices
    auto put_row = [&](int R, KGlob<double> *p) {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int vv = w * G + g;
        if (vv < P) {
          const int kg = first_reg(vv);
          const int r = R - seg_base(vv);
          if (r >= kg && r < SEG) {
            const double val = d.get(r);
            if (gh == g && out) *p = val;
          }
        }
      }
    };
    for (int s = 0; s < steps; ++s) {
      const int n = n0 + s;
      double xlo = 0.0, xhi = 0.0;
      // the direction split, segment count and segment index are re-derived
      // each step, so that tests built on them are not kept as per-row
      // masks across the loop (they would not fit in scalar registers)
      int vs = vsplit, Pq = P, wq = v;
      if constexpr (G == 1)
        asm volatile("" : "+s"(vs), "+s"(Pq), "+s"(wq));
      else
        asm volatile("" : "+v"(vs), "+s"(Pq), "+v"(wq));
      if (active) {
        const double gn = sh_g[w][s];
        const double blo = lo_end ? lo_scale * sh_bd[0][s][tl] : 0.0;
        const double bhi = hi_end ? hi_scale * sh_bd[1][s][tl] : 0.0;
        if constexpr (FEM) {
          // G in every register, then the elimination with the mass matrix.
          // Builds with longer or more segments recompute the Courant numbers
          // each step (kept across the loop, one per register, they spill);
          // 8 wavefronts of at most 17 rows keep them (51.8 against 53.3 us
          // per launch on 1024 x 1024, J = 8)
          double nu0 = nu0_item;
          if constexpr (NW > 8 || SEG > 17) asm volatile("" : "+v"(nu0));
          const bool first = n == 0;
          if (first)
            fem_stage<SEG, DIR_NONE>(d, fs, nu0, dnu, gn, vs, fr, base, nx, col);
          else if (dir == DIR_LO)
            fem_stage<SEG, DIR_LO>(d, fs, nu0, dnu, gn, vs, fr, base, nx, col);
          else if (dir == DIR_UP)
            fem_stage<SEG, DIR_UP>(d, fs, nu0, dnu, gn, vs, fr, base, nx, col);
          else
            fem_stage<SEG, DIR_MIX>(d, fs, nu0, dnu, gn, vs, fr, base, nx, col);
          const double gb = fem_edge_g(ubelow, nul, gn, fbelow, first);
          const double ga = fem_edge_g(uabove, nua, gn, fabove, first);
          if (Pq > 1) {
            if constexpr (RR)
              gf1 = first_value(d);
            else
              sh_gf[s & 1][v][tl] = first_value(d);
          }
          // (no loads ahead in 16-wave builds, 128 registers, or for segments
          // longer than 20 rows: the extra registers would spill)
          fem_forward<SEG, (NW <= 8 && SEG <= 20)>(d, mc, fma(wol, gb, blo), fma(woa, ga, bhi));
        } else {
          // transport + source + forward elimination, one pass
          if (dir == DIR_LO)
            march_forward<SEG, NW, DIR_LO>(d, fs, mc, gn, blo, bhi, vs, fr, base, nx, col);
          else if (dir == DIR_UP)
            march_forward<SEG, NW, DIR_UP>(d, fs, mc, gn, blo, bhi, vs, fr, base, nx, col);
          else
            march_forward<SEG, NW, DIR_MIX>(d, fs, mc, gn, blo, bhi, vs, fr, base, nx, col);
        }
        // back substitution
        double x = d.template ld<SEG - 1>();
        static_for<0, SEG - 1>([&](auto kc) {
          constexpr int k = SEG - 2 - decltype(kc)::value;
          x = fma(mc[k].bc, x, d.template ld<k>());
          d.template st<k>(x);
        });
        if (Pq > 1) {
          if constexpr (RR) {
            const double Ev =
                last ? 0.0 : fma(-ra_s, d.template ld<SEG - 2>(), d.template ld<SEG - 1>());
            double Fv = -rc_s * first_value(d);
            if constexpr (FEM) Fv = fma(rg_s, gf1, Fv);
            sh_E[s & 1][v][tl] = Ev;
            sh_F[s & 1][v][tl] = Fv;
          } else {
            sh_first[s & 1][v][tl] = first_value(d);
            sh_last[s & 1][v][tl] = d.template ld<SEG - 2>();
            sh_sep[s & 1][v][tl] = d.template ld<SEG - 1>();
          }
        }
      }
      if (Pq > 1) {
        __syncthreads();
        if constexpr (RR) {
          if (active) {
            double xl = 0.0, xh = 0.0;
#pragma unroll
            for (int q = 0; q < NV - 1; ++q) {
              const double D = sh_E[s & 1][q][tl] + sh_F[s & 1][q + 1][tl];
              xl = fma(RL[q], D, xl);
              xh = fma(RH[q], D, xh);
            }
            xlo = xl;
            xhi = xh;
          }
        } else if (active) {
          // reduced separator system, per column: right-hand sides D_r from
          // LDS, then the two separators this segment borders (r = v-1, v)
          // as dot products with rows of the precomputed inverse
          const int m = Pq - 1;
          const double *Rl = sh_rinv + (wq > 0 ? wq - 1 : 0) * m;
          const double *Rh = sh_rinv + (wq < m ? wq : 0) * m;
          double xl = 0.0, xh = 0.0;
#pragma unroll
          for (int q = 0; q < NV - 1; ++q) {
            if (q < m) {
              const RedCoef &rq = sh_rc[q];
              double D = sh_sep[s & 1][q][tl] - rq.ra * sh_last[s & 1][q][tl] -
                         rq.rc * sh_first[s & 1][q + 1][tl];
              if constexpr (FEM) D = fma(rq.rg, sh_gf[s & 1][q + 1][tl], D);
              xl = fma(Rl[q], D, xl);
              xh = fma(Rh[q], D, xh);
            }
          }
          xlo = wq > 0 ? xl : 0.0;
          xhi = wq < m ? xh : 0.0;
        }
      }
      if (active) {
        static_for<0, SEG>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          d.template st<k>(fma(-mc[k].sl, xlo, fma(-mc[k].sr, xhi, d.template ld<k>())));
        });
        if (!last) d.template st<SEG - 1>(xhi);
      }
      if constexpr (FEM) {
        // states of the outside nodes at level n+1: the separator below (from
        // the reduced system), or the fixed nodes' traces
        if (v > 0)
          ubelow = xlo;
        else if (lo_end)
          ubelow = sh_bd[0][s][tl];
        if (hi_end) uabove = sh_bd[1][s][tl];
      }
      // interface-node values of level n+1
      if (wave_active) {
        const size_t lvl = (size_t)n * nx + col;
        if (out_hi_plane >= 0) {
          KGlob<double> *Vj = Vbase + (size_t)(out_hi_plane >> 1) * 6 * plane + lvl;
          put_row(out_hi_row, Vj + V_A_LO * plane);
          if (robin) {
            put_row(out_hi_row + (FEM ? -1 : 1), Vj + V_A1_LO * plane);
            put_row(n_rows - 1, Vj + V_B_LO * plane);
          }
        }
        if (out_lo_plane >= 0) {
          KGlob<double> *Vj = Vbase + (size_t)((out_lo_plane - 1) >> 1) * 6 * plane + lvl;
          put_row(out_lo_row, Vj + V_B_HI * plane);
          if (robin) {
            put_row(out_lo_row + (FEM ? 1 : -1), Vj + V_B1_HI * plane);
            put_row(0, Vj + V_A_HI * plane);
          }
        }
      }
    }
    // the next item restages the reduced system and reuses the slots
    if (P > 1) __syncthreads();
    if (active && out) {
      static_for<0, SEG>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        if (k >= k0) dst[(size_t)(base + k) * nx + col] = d.template ld<k>();
      });
    }
  }
}

// ---------------------------------------------------------------------------
// Finite-difference march over TPW x-tiles per wavefront (the default for
// finite differences when one workgroup of NW wavefronts holds a subdomain).
// The arithmetic of a step is that of march_kernel (transport, source and
// forward elimination in one pass, back substitution, reduced separator
// system, spike correction), organised for fewer instructions per cell:
//  * every wavefront holds its segment for TPW tiles of 64 columns: the
//    coefficient reads (wave-uniform LDS broadcasts), the loop and the
//    barrier are shared by TPW independent columns per lane, which also
//    gives the dependent elimination chains TPW-fold instruction-level
//    parallelism;
//  * a subdomain whose rows all move the same way in x (all v >= 0 or all
//    v <= 0) needs its halo only on the upwind side: the tile then yields
//    64 - S columns instead of 64 - 2S (SubDev::hsides);
//  * the back substitution copies the first real row of the last segment into
//    its padding registers (their bc is 1), so every segment's first row is
//    register 0 (no run-time register index);
//  * the reduced system: each segment forms its own parts of the separator
//    right-hand sides before the barrier, E_v = sep_v - ra_v last_v and
//    F_v = -rc_{v-1} first_v, and each lane keeps the two rows of the reduced
//    inverse it needs in registers, so after the barrier a separator costs two
//    LDS reads and two FMAs per tile.
// Items: (sub, x0) with x0 the first output column of tile 0; tile t outputs
// columns x0 + t W .. x0 + (t+1) W - 1 (W = 64 - halo sides), lane l holds
// column x0 + t W - HL + l.
constexpr int kMaxStepsFd = 16;
#define KFP_FD_SCHED 1


// A column segment in registers, indexed at compile time only: each row is
// its own value, so a step's results take the registers of its inputs (a
// vector type would be rebuilt and copied back every step).
template <int N>
struct ColRegs {
  double r[N];
  template <int K>
  __device__ __forceinline__ double ld() const {
    return r[K];
  }
  template <int K>
  __device__ __forceinline__ void st(double v) {
    r[K] = v;
  }
};

template <int SEG, int NW, int TPW, int OCC>
__global__ __launch_bounds__(NW * 64, OCC) void march_fd_kernel(StepTables t, int n0_in, int S,
                                                                int H, int src_in, int par) {
  static_assert(TPW == 1 || TPW == 2, "tiles per wavefront");
  static_assert(SEG <= kFRegMax, "the source segment is held in registers");
  constexpr int NR = NW > 1 ? NW - 1 : 1;  // separators of a full workgroup
  // separator v's right-hand side parts, side by side: E_v (from segment v)
  // and F_{v+1} (from segment v+1), read as one 16-byte value
  __shared__ double2 sh_EF[2][NW][TPW][64];
  __shared__ double sh_bd[2][kMaxStepsFd][TPW][64];
  __shared__ MarchCoef sh_mc[NW][SEG];
  __shared__ double sh_g[NW][kMaxStepsFd];
  // the reduced inverse of the item's subdomain, transposed: sh_ri[q][v + 1]
  // is row v, column q (zero past the subdomain's separators; column 0 and
  // columns past the last separator zero), so that a segment's two rows are
  // adjacent
  __shared__ double sh_ri[NR][NW + 1];
  const int lane = threadIdx.x & 63;
  const int v = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // this wave's segment
  KConst<Item> *items = as_const(t.items);
  KConst<SubDev> *subs = as_const(t.subs);
  KConst<InstDev> *insts = as_const(t.inst);
  for (int it = blockIdx.x; it < t.n_items; it += gridDim.x) {
    const int sub = items[it].sub;
    const int x0 = items[it].x0;
    KConst<SubDev> *sd = subs + sub;
    KConst<InstDev> *I = insts + sd->inst;
    if (!I->active) continue;
    int n0 = n0_in, src_par = src_in;
    if (t.blk) {  // pipelined iterations: this instance's block of this launch
      const int b = as_const(t.blk)[sd->inst];
      if (b < 0) continue;
      n0 = b * S;
      src_par = b & 1;
    }
    const int nx = I->nx;
    const int nt = I->nt;
    if (n0 >= nt) continue;
    const int steps = min(min(S, kMaxStepsFd), nt - n0);  // S is checked by the host
    const int hs = sd->hsides;
    const int HL = (hs & 1) ? H : 0, HR = (hs & 2) ? H : 0;
    const int W = 64 - HL - HR;
    const int rel = lane - HL;
    int col[TPW];
    bool out[TPW];
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
      const int xo = x0 + tt * W;  // first output column of the tile
      int c = (xo + rel) % nx;
      if (c < 0) c += nx;
      col[tt] = c;
      out[tt] = rel >= 0 && rel < W && xo + rel < nx;
    }
    const size_t plane = (size_t)nt * nx;
    const int n_rows = sd->n;
    const int row_off = sd->row_off;
    const int g_lo = sd->g_lo;
    KGlob<const double> *src = as_glob((n0 == 0) ? I->u0 + (size_t)g_lo * nx
                                                 : I->U[src_par] + (size_t)row_off * nx);
    KGlob<double> *dst = as_glob(I->U[src_par ^ 1] + (size_t)row_off * nx);
    KGlob<const double> *fr = as_glob(I->f + (size_t)g_lo * nx);
    KGlob<const double> *lin = as_glob((const double *)I->lam[par]);
    KGlob<double> *Vbase = as_glob(I->V);
    const double rr = I->r;
    const bool robin = I->tr == 1;
    const int P = sd->P;
    const int pad = sd->pad;
    const bool active = v < P;
    const bool last = v == P - 1;
    const int k0 = last ? pad : 0;             // first real row in this wave's registers
    const int base = v * SEG - (last ? pad : 0);  // local row of register 0
    const int vsplit = sd->vsplit - base;      // registers >= vsplit have v >= 0
    const int dir = vsplit <= 0 ? DIR_LO : (vsplit >= SEG ? DIR_UP : DIR_MIX);
    const int lo_kind = sd->lo_kind, hi_kind = sd->hi_kind;
    const int lam_lo = sd->lam_lo, lam_hi = sd->lam_hi;
    const int out_hi_plane = sd->out_hi_plane, out_hi_row = sd->out_hi_row;
    const int out_lo_plane = sd->out_lo_plane, out_lo_row = sd->out_lo_row;
    const bool lo_end = active && v == 0 && lo_kind != END_PHYS;
    const bool hi_end = active && last && hi_kind != END_PHYS;
    // staging (each wave its own rows, factors and boundary data: written and
    // read by the same wave; the zeroed reduced-system slots of unused
    // segments are first read after the first step's barrier)
    const MarchCoef *mc = sh_mc[v];
    {
      // a wave without rows (v >= P) runs the same steps on zero rows and
      // zero state: its results stay zero and are never stored
      KGlob<const double> *ct = as_glob((const double *)(t.mrows + sd->tab + v * SEG));
      double *cs = reinterpret_cast<double *>(sh_mc[v]);
      constexpr int NDB = (int)(sizeof(MarchCoef) / sizeof(double));
#pragma unroll
      for (int e0 = 0; e0 < SEG * NDB; e0 += 64) {
        if (e0 + lane < SEG * NDB) {
          double c = 0.0;
          if (active) c = ct[e0 + lane];  // rows past the subdomain's table are not read
          cs[e0 + lane] = c;
        }
      }
      KGlob<const double> *gt = as_glob(I->g);
      if (lane < steps) sh_g[v][lane] = gt[n0 + lane];
    }
    if (active) {
#pragma unroll
      for (int tt = 0; tt < TPW; ++tt) {
        if (lo_end) {
          KGlob<const double> *p = lin + (size_t)lam_lo * plane + col[tt];
          for (int s = 0; s < steps; ++s) sh_bd[0][s][tt][lane] = p[(size_t)(n0 + s) * nx];
        }
        if (hi_end) {
          KGlob<const double> *p = lin + (size_t)lam_hi * plane + col[tt];
          for (int s = 0; s < steps; ++s) sh_bd[1][s][tt][lane] = p[(size_t)(n0 + s) * nx];
        }
      }
    }
    // the reduced inverse, row v staged by the wave of segment v (the wave
    // of segment v reads rows v - 1 and v: separators v - 1 and v); the
    // separator coefficient ra_v and rc_{v-1}
    double ra_s = 0.0, rc_s = 0.0;
    if (P > 1) {
      const int m = P - 1;
      KGlob<const double> *rv = as_glob(t.rinv + sd->rinv);
      if (lane < NR) {
        double e = 0.0;
        if (v < m && lane < m) e = rv[(size_t)v * m + lane];
        sh_ri[lane][v + 1] = e;
        if (v == 0) sh_ri[lane][0] = 0.0;
      }
    }
    if (P > 1 && active) {
      const int m = P - 1;
      KGlob<const double> *rt = as_glob((const double *)(t.reds + sd->red));
      constexpr int NRW = (int)(sizeof(RedCoef) / sizeof(double));
      if (v < m) ra_s = rt[(size_t)v * NRW + 0];
      if (v > 0) rc_s = rt[(size_t)(v - 1) * NRW + 1];
    }
    ra_s = wave_uniform(ra_s);
    rc_s = wave_uniform(rc_s);
    // weight of the incoming trace in an end row: 1 (a Robin row), 2 dt / h_v
    // (half-cell row), r (next to a fixed node)
    const double rfv = 2.0 * rr * I->hv;
    auto end_w = [&](int kind) {
      return kind == END_ROBIN ? 1.0 : (kind == END_RFV ? rfv : rr);
    };
    const double lo_scale = wave_uniform(lo_end ? mc[k0].fab * end_w(lo_kind) : 0.0);
    const double hi_scale = wave_uniform(hi_end ? mc[SEG - 1].fab * end_w(hi_kind) : 0.0);
    // the item's march, one copy per upwind direction of the wave's rows
    // (loads, steps, stores: the state's registers are assigned within one
    // copy), with no branch on the wave's rows in the step loop (a wave
    // without rows steps zeros)
    // CG: the source factor g is the same at every level (s constant in
    // time): the source rows are scaled by it once, at load, and the step
    // adds them as they are (the same products, rounded the same way)
    auto march_steps = [&](auto dirc, auto cgc) {
      constexpr int DIR = decltype(dirc)::value;
      constexpr bool CG = decltype(cgc)::value;
      // (row pointers are wave-uniform: each load is a scalar base plus the
      // lane's 32-bit column offset, so no 64-bit address per row is held)
      ColRegs<SEG> d[TPW], fs[TPW];
      static_for<0, SEG>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const int r = max(base + k, 0);
        const double fa = mc[k].fa;
        KGlob<const double> *srow = src + (size_t)r * nx;
        KGlob<const double> *frow = fr + (size_t)r * nx;
  #pragma unroll
        for (int tt = 0; tt < TPW; ++tt) {
          double u = 0.0, fv = 0.0;
          if (active) {  // a wave without rows reads nothing
            u = srow[(unsigned)col[tt]];
            fv = fa * frow[(unsigned)col[tt]];
          if constexpr (CG) fv = sh_g[v][0] * fv;
          }
          d[tt].template st<k>(u);
          fs[tt].template st<k>(fv);
        }
      });
        // value of local row R of every tile to p[tt]: the register is selected
      // with wave-uniform branches (no run-time register index), searched in
      // a window of six registers (interface rows lie near a segment's ends)
      auto put_reg = [&](auto lo, auto hi, int r, KGlob<double> *p) {
        static_for<decltype(lo)::value, decltype(hi)::value>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          if (r == k) {
#pragma unroll
            for (int tt = 0; tt < TPW; ++tt)
              if (out[tt]) p[(unsigned)col[tt]] = d[tt].template ld<k>();
          }
        });
      };
      auto put_row = [&](int R, KGlob<double> *p) {
        const int r = R - base;
        constexpr int WL = SEG < 6 ? SEG : 6, WH = SEG - 6 > WL ? SEG - 6 : WL;
        if (r < k0 || r >= SEG) return;
        if (r < WL)
          put_reg(std::integral_constant<int, 0>{}, std::integral_constant<int, WL>{}, r, p);
        else if (r >= WH)
          put_reg(std::integral_constant<int, WH>{}, std::integral_constant<int, SEG>{}, r, p);
        else
          put_reg(std::integral_constant<int, WL>{}, std::integral_constant<int, WH>{}, r, p);
      };
      for (int s = 0; s < steps; ++s) {
        const int n = n0 + s;
        // re-derived each step, so that tests built on them are not kept as
        // per-row masks across the loop
        int vs = vsplit, Pq = P;
        asm volatile("" : "+s"(vs), "+s"(Pq));
        const double gn = wave_uniform(sh_g[v][s]);
        double y[TPW], bh[TPW];
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt) {
          y[tt] = lo_end ? lo_scale * sh_bd[0][s][tt][lane] : 0.0;
          bh[tt] = hi_end ? hi_scale * sh_bd[1][s][tt][lane] : 0.0;
        }
        // transport + source + forward elimination, one pass.  The
        // coefficients of row k+2 are read before row k is computed, and the
        // scheduling barrier keeps the reads in that order (LDS reads return
        // in order: each wait overlaps two rows of arithmetic, and no more
        // rows' coefficients than that are held in registers)
        double2 ab0 = *(const double2 *)&mc[0].alpha, ab1 = *(const double2 *)&mc[1].alpha;
        double fb0 = mc[0].fb, fb1 = mc[1].fb;
        static_for<0, SEG>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          const double al = ab0.x, be = ab0.y, fb = fb0;
          ab0 = ab1;
          fb0 = fb1;
          if constexpr (k + 2 < SEG) {
            ab1 = *(const double2 *)&mc[k + 2].alpha;
            fb1 = mc[k + 2].fb;
          }
          __builtin_amdgcn_sched_barrier(KFP_FD_SCHED);
#pragma unroll
          for (int tt = 0; tt < TPW; ++tt) {
            const double u = d[tt].template ld<k>();
            double nb;
            if constexpr (DIR == DIR_LO) {
              nb = from_lower_lane(u);
            } else if constexpr (DIR == DIR_UP) {
              nb = from_upper_lane(u);
            } else {
              const double a = from_lower_lane(u), c = from_upper_lane(u);
              nb = (k >= vs) ? a : c;
            }
            const double sk = CG ? fs[tt].template ld<k>() : gn * fs[tt].template ld<k>();
            double tk = fma(al, u, fma(be, nb, sk));
            if constexpr (k == SEG - 1) tk += bh[tt];
            y[tt] = fma(fb, y[tt], tk);
            d[tt].template st<k>(y[tt]);
          }
        });
        // back substitution
        double x[TPW];
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt) x[tt] = d[tt].template ld<SEG - 1>();
        double bc0 = mc[SEG - 2].bc, bc1 = mc[SEG > 2 ? SEG - 3 : 0].bc;
        static_for<0, SEG - 1>([&](auto kc) {
          constexpr int k = SEG - 2 - decltype(kc)::value;
          const double bc = bc0;
          bc0 = bc1;
          if constexpr (k - 2 >= 0) bc1 = mc[k - 2].bc;
          __builtin_amdgcn_sched_barrier(KFP_FD_SCHED);
#pragma unroll
          for (int tt = 0; tt < TPW; ++tt) {
            x[tt] = fma(bc, x[tt], d[tt].template ld<k>());
            d[tt].template st<k>(x[tt]);
          }
        });
        // reduced separator system
        double xlo[TPW], xhi[TPW];
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt) xlo[tt] = xhi[tt] = 0.0;
        if (Pq > 1) {
#pragma unroll
          for (int tt = 0; tt < TPW; ++tt) {
            sh_EF[s & 1][v][tt][lane].x =
                last ? 0.0
                     : fma(-ra_s, d[tt].template ld<SEG - 2>(), d[tt].template ld<SEG - 1>());
            if (v > 0) sh_EF[s & 1][v - 1][tt][lane].y = -rc_s * d[tt].template ld<0>();
          }
          __syncthreads();
#pragma unroll
          for (int q = 0; q < NR; ++q) {
            const double rl = sh_ri[q][v], rh = sh_ri[q][v + 1];
#pragma unroll
            for (int tt = 0; tt < TPW; ++tt) {
              const double2 ef = sh_EF[s & 1][q][tt][lane];
              const double D = ef.x + ef.y;
              xlo[tt] = fma(rl, D, xlo[tt]);
              xhi[tt] = fma(rh, D, xhi[tt]);
            }
          }
        }
        // spike correction; a non-final segment's last register is its separator
        double2 sp0 = *(const double2 *)&mc[0].sl, sp1 = *(const double2 *)&mc[1].sl;
        static_for<0, SEG>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          const double sl = sp0.x, sr = sp0.y;
          sp0 = sp1;
          if constexpr (k + 2 < SEG) sp1 = *(const double2 *)&mc[k + 2].sl;
          __builtin_amdgcn_sched_barrier(KFP_FD_SCHED);
#pragma unroll
          for (int tt = 0; tt < TPW; ++tt)
            d[tt].template st<k>(fma(-sl, xlo[tt], fma(-sr, xhi[tt], d[tt].template ld<k>())));
        });
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt)
          d[tt].template st<SEG - 1>(last ? d[tt].template ld<SEG - 1>() : xhi[tt]);
        // interface-node values of level n+1
        const size_t lvl = (size_t)n * nx;
        if (out_hi_plane >= 0) {
          KGlob<double> *Vj = Vbase + (size_t)(out_hi_plane >> 1) * 6 * plane + lvl;
          put_row(out_hi_row, Vj + V_A_LO * plane);
          if (robin) {
            put_row(out_hi_row + 1, Vj + V_A1_LO * plane);
            put_row(n_rows - 1, Vj + V_B_LO * plane);
          }
        }
        if (out_lo_plane >= 0) {
          KGlob<double> *Vj = Vbase + (size_t)((out_lo_plane - 1) >> 1) * 6 * plane + lvl;
          put_row(out_lo_row, Vj + V_B_HI * plane);
          if (robin) {
            put_row(out_lo_row - 1, Vj + V_B1_HI * plane);
            put_row(0, Vj + V_A_HI * plane);
          }
        }
      }
      // the next item restages the tables and reuses the slots
      if (P > 1) __syncthreads();
      if (active) {
        // addresses formed anew: offsets kept from the loads before the loop
        // would hold registers across it
        int nxs = nx;
        asm volatile("" : "+s"(nxs));
  #pragma unroll
        for (int tt = 0; tt < TPW; ++tt) asm volatile("" : "+v"(col[tt]));
        static_for<0, SEG>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          if (k >= k0) {
            KGlob<double> *drow = dst + (size_t)(base + k) * nxs;
  #pragma unroll
            for (int tt = 0; tt < TPW; ++tt)
              if (out[tt]) drow[(unsigned)col[tt]] = d[tt].template ld<k>();
          }
        });
      }
    };
    using CGT = std::true_type;
    using CGF = std::false_type;
    const bool cg = I->gconst != 0;
    if (dir == DIR_LO) {
      if (cg)
        march_steps(std::integral_constant<int, DIR_LO>{}, CGT{});
      else
        march_steps(std::integral_constant<int, DIR_LO>{}, CGF{});
    } else if (dir == DIR_UP) {
      if (cg)
        march_steps(std::integral_constant<int, DIR_UP>{}, CGT{});
      else
        march_steps(std::integral_constant<int, DIR_UP>{}, CGF{});
    } else {
      if (cg)
        march_steps(std::integral_constant<int, DIR_MIX>{}, CGT{});
      else
        march_steps(std::integral_constant<int, DIR_MIX>{}, CGF{});
    }
  }
}

// Traces of every level and the residual of one interface, from the value
// planes: lambda_{j->j+1} = Q_2 u_j at a_{j+1}, lambda_{j+1->j} = Q_1 u_{j+1}
// at b_j, and max |u_j - u_{j+1}| at the two end nodes of the overlap.
// mode 0: both planes of every interface and the residual (parallel order);
// 1: only the planes sent by even subdomains (plane 2j when j is even, plane
// 2j+1 when j+1 is even); 2: only those sent by odd subdomains, and the
// residual (red-black order: run after the even, then the odd half-sweep).
// A launch with mode 0 takes each instance's own mode (InstDev::xmode).
// nodes per thread and chunk in the exchange's common case
constexpr int kExU = 4;

__global__ __launch_bounds__(256) void exchange_kernel(StepTables t, int par, int S, int mode_in) {
  __shared__ unsigned long long red[4];
  const ExItem ex = load_const(as_const(t.ex) + blockIdx.y);
  const InstDev I = load_inst(as_const(t.inst) + ex.inst);
  if (!I.active) return;
  // mode 0 at launch: the instance's own (red-black half-sweep slots)
  const int mode = mode_in != 0 ? mode_in : I.xmode;
  const size_t plane = (size_t)I.nt * I.nx;
  // levels covered: the whole window, or (pipelined) the instance's block
  size_t e_begin = 0, e_end = plane;
  if (t.blk) {
    const int b = as_const(t.blk)[ex.inst];
    if (b < 0) return;
    const int n0 = b * S;
    if (n0 >= I.nt) return;
    e_begin = (size_t)n0 * I.nx;
    e_end = (size_t)min(n0 + S, I.nt) * I.nx;
  }
  const int j = ex.j;
  const double *V = I.V + (size_t)j * 6 * plane;
  const double *lin = par ? I.lam[1] : I.lam[0];
  double *lout = par ? I.lam[0] : I.lam[1];
  const bool robin = I.tr == 1;
  unsigned long long r = 0ull;
  if (robin && !I.nonovl && I.scheme != SCHEME_FEM) {
    // overlapping Robin with finite differences (the common case): chunks of
    // kExU x 256 nodes, all six value-plane reads of a chunk issued before
    // any trace store (the stores may alias nothing here, but the compiler
    // cannot know that, and would otherwise wait on each node's loads in
    // turn); the arithmetic per node is the one of the general loop below
    for (size_t c0 = e_begin + (size_t)blockIdx.x * (256 * kExU); c0 < e_end;
         c0 += (size_t)gridDim.x * (256 * kExU)) {
      double ua[kExU], ubh[kExU], ua1[kExU], ub1h[kExU], ublo[kExU], uahi[kExU];
#pragma unroll
      for (int u = 0; u < kExU; ++u) {
        const size_t e = c0 + (size_t)u * 256 + threadIdx.x;
        const size_t ee = e < e_end ? e : e_begin;  // past the end: a node read, not used
        ua[u] = V[V_A_LO * plane + ee];
        ubh[u] = V[V_B_HI * plane + ee];
        ua1[u] = V[V_A1_LO * plane + ee];
        ub1h[u] = V[V_B1_HI * plane + ee];
        ublo[u] = V[V_B_LO * plane + ee];
        uahi[u] = V[V_A_HI * plane + ee];
      }
#pragma unroll
      for (int u = 0; u < kExU; ++u) {
        const size_t e = c0 + (size_t)u * 256 + threadIdx.x;
        if (e >= e_end) continue;
        const double toR = I.q * ua[u] - (ua1[u] - ua[u]) / I.hv;
        const double toL = I.p * ubh[u] + (ubh[u] - ub1h[u]) / I.hv;
        if (mode == 0 || (j & 1) == mode - 1) lout[(size_t)(2 * j) * plane + e] = toR;
        if (mode == 0 || ((j + 1) & 1) == mode - 1) lout[(size_t)(2 * j + 1) * plane + e] = toL;
        if (mode == 1 && lout != lin) {
          const size_t other = (size_t)(2 * j + ((j & 1) ? 0 : 1)) * plane + e;
          lout[other] = lin[other];
        }
        const unsigned long long ra =
            (unsigned long long)__double_as_longlong(fabs(ua[u] - uahi[u]));
        const unsigned long long rb =
            (unsigned long long)__double_as_longlong(fabs(ublo[u] - ubh[u]));
        r = ra > r ? ra : r;
        r = rb > r ? rb : r;
      }
    }
  } else
  for (size_t e = e_begin + (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < e_end;
       e += (size_t)gridDim.x * blockDim.x) {
    const double ua = V[V_A_LO * plane + e];
    const double ubh = V[V_B_HI * plane + e];
    double toR = ua, toL = ubh, ub_lo, ua_hi;
    if (I.nonovl) {  // shared node: Q from the Robin condition each side was solved with
      toR = (I.p + I.q) * ua - lin[(size_t)(2 * j + 1) * plane + e];
      toL = (I.p + I.q) * ubh - lin[(size_t)(2 * j) * plane + e];
      ub_lo = ua;
      ua_hi = ubh;
    } else if (robin && I.scheme == SCHEME_FEM) {
      // finite elements: the derivative in Q is the flux the sender's element
      // next to the node carries (weak form of the diffusion stage):
      //   below a: F = h/(6dt) [(W_{a-1} - G_{a-1}) + 2 (W_a - G_a)] + (W_a - W_{a-1})/h,
      //   above b: F = h/(6dt) [2 (W_b - G_b) + (W_{b+1} - G_{b+1})] + (W_b - W_{b+1})/h,
      // Q_2 u_j = q W_a - F(a), Q_1 u_{j+1} = p W_b - F(b); G = T W^n + dt s f
      // from the previous level of the same value plane (u0 at the first)
      const int nx = I.nx;
      const int lv = (int)(e / nx), m = (int)(e - (size_t)lv * nx);
      const double dt = I.r * I.hv * I.hv;
      const double gn = I.g[lv];
      const double cm = I.hv / (6.0 * dt);
      auto stage = [&](int slot, int node) {
        double u;
        if (lv == 0) {
          u = I.u0[(size_t)node * nx + m];
        } else {
          const double nu = (-1.0 + node * I.hv) * dt * nx;
          const double *row = V + (size_t)slot * plane + (size_t)(lv - 1) * nx;
          int mn = m + (nu > 0.0 ? -1 : (nu < 0.0 ? 1 : 0));
          mn = mn < 0 ? mn + nx : (mn >= nx ? mn - nx : mn);
          const double w = fabs(nu);
          u = fma(1.0 - w, row[m], w * row[mn]);
        }
        return fma(gn, I.f[(size_t)node * nx + m], u);
      };
      const double ua1 = V[V_A1_LO * plane + e];   // W_j(a-1)
      const double ub1h = V[V_B1_HI * plane + e];  // W_{j+1}(b+1)
      const double ga = stage(V_A_LO, ex.a), ga1 = stage(V_A1_LO, ex.a - 1);
      const double gb = stage(V_B_HI, ex.b), gb1 = stage(V_B1_HI, ex.b + 1);
      toR = I.q * ua - (cm * ((ua1 - ga1) + 2.0 * (ua - ga)) + (ua - ua1) / I.hv);
      toL = I.p * ubh - (cm * (2.0 * (ubh - gb) + (ub1h - gb1)) + (ubh - ub1h) / I.hv);
      ub_lo = V[V_B_LO * plane + e];
      ua_hi = V[V_A_HI * plane + e];
    } else if (robin) {
      const double ua1 = V[V_A1_LO * plane + e];
      const double ub1h = V[V_B1_HI * plane + e];
      toR = I.q * ua - (ua1 - ua) / I.hv;
      toL = I.p * ubh + (ubh - ub1h) / I.hv;
      ub_lo = V[V_B_LO * plane + e];
      ua_hi = V[V_A_HI * plane + e];
    } else {
      ub_lo = lin[(size_t)(2 * j + 1) * plane + e];
      ua_hi = lin[(size_t)(2 * j) * plane + e];
    }
    if (mode == 0 || (j & 1) == mode - 1) lout[(size_t)(2 * j) * plane + e] = toR;
    if (mode == 0 || ((j + 1) & 1) == mode - 1) lout[(size_t)(2 * j + 1) * plane + e] = toL;
    // overlapped red-black half-sweeps write a window of their own: the even
    // half-sweep also carries over the odd subdomains' traces it was solved
    // with, which the odd half-sweep's residual needs (Dirichlet: the fixed
    // node values of the even subdomains)
    if (mode == 1 && lout != lin) {
      const size_t other = (size_t)(2 * j + ((j & 1) ? 0 : 1)) * plane + e;
      lout[other] = lin[other];
    }
    const unsigned long long ra = (unsigned long long)__double_as_longlong(fabs(ua - ua_hi));
    const unsigned long long rb = (unsigned long long)__double_as_longlong(fabs(ub_lo - ubh));
    r = ra > r ? ra : r;
    r = rb > r ? rb : r;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(r, off, 64);
    r = o > r ? o : r;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = red[0];
    for (int i = 1; i < 4; ++i) m = red[i] > m ? red[i] : m;
    if (m && mode != 1) atomicMax(I.res, m);
  }
}

// Scheduler of pipelined iterations, run by one lane after every launch:
// records the iterations whose last block just ran (residual history,
// convergence, the first non-finite residual), then assigns each slot its
// block of the next launch (slot i: the unit k = i mod M, if any, with
// 0 <= t - d (k-1) < L), clearing the residual of units that start.  A unit
// is an iteration, or in red-black order a half-sweep (unit 2k-1 marches the
// even subdomains of iteration k, unit 2k the odd ones and closes it).
__global__ void pipe_tick_kernel(PipeCtl *c, int *blk, int *iter, unsigned long long *res,
                                 double *hist) {
  if (threadIdx.x != 0) return;
  const int M = c->M, d = c->d, L = c->L;
  // red-black: the units are half-sweeps, unit 2k closing iteration k
  const int rb = c->rb;
  for (int i = 0; i < M; ++i) {
    if (blk[i] != L - 1) continue;
    const int u = iter[i];
    if (rb && (u & 1)) continue;  // an even-subdomain half-sweep: no residual yet
    const int k = rb ? u / 2 : u;
    const double r = __longlong_as_double((long long)res[i]);
    hist[k - 1] = r;
    c->done = k;
    if (c->stop == 0) {
      if (k == 1 && c->restart_on_nonfinite && !(r <= DBL_MAX))
        c->stop = -1;
      else if (r < c->tol || k >= c->kmax)
        c->stop = k;
    }
  }
  const int t1 = c->t + 1;
  c->t = t1;
  const int khi = t1 / d + 1;
  const int umax = rb ? 2 * c->kmax : c->kmax;
  bool any = false;
  for (int i = 0; i < M; ++i) {
    int b = -1;
    const int k = khi - (((khi - i) % M) + M) % M;
    if (c->stop == 0 && k >= 1 && k <= umax) {
      const int bb = t1 - d * (k - 1);
      if (bb >= 0 && bb < L) b = bb;
    }
    if (b == 0) res[i] = 0ull;
    if (b >= 0) {
      iter[i] = k;
      any = true;
    }
    blk[i] = b;
  }
  if (any) c->last_busy = t1;
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__global__ void reset_res_kernel(const InstDev *inst, int n_inst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_inst && inst[i].active) *inst[i].res = 0ull;
}

// Glued output.  nudt > 0 (finite elements): the transport stage of the last
// step, row i with Courant number (-1 + i hv) nudt.
__global__ void assemble_kernel(const double *__restrict__ U, const int *__restrict__ rowmap,
                                double *__restrict__ uT, int nv, int nx, double nudt,
                                double hv) {
  const size_t total = (size_t)(nv + 1) * nx;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / nx);
    const int m = (int)(e - (size_t)i * nx);
    const int r = rowmap[i];
    if (r == -2) continue;  // node taken from another state
    if (r < 0) {
      uT[e] = 0.0;
      continue;
    }
    const double *row = U + (size_t)r * nx;
    const double nu = (-1.0 + i * hv) * nudt;
    if (nudt == 0.0 || nu == 0.0) {
      uT[e] = row[m];
      continue;
    }
    int mn = m + (nu > 0.0 ? -1 : 1);
    mn = mn < 0 ? mn + nx : (mn >= nx ? mn - nx : mn);
    const double w = fabs(nu);
    uT[e] = fma(1.0 - w, row[m], w * row[mn]);
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
                                const int *__restrict__ ab, int tr, double p, double q,
                                double hv, double *__restrict__ lam) {
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
      toR = q * ua - (ua1 - ua) / hv;  // Q_2 = q - d/dv at a_{j+1}
      toL = p * ub + (ub - ub1) / hv;  // Q_1 = p + d/dv at b_j
    }
    lam[(size_t)(2 * j) * plane + off] = toR;
    lam[(size_t)(2 * j + 1) * plane + off] = toL;
  }
}

// Streaming copy, 16 B per lane (bandwidth probe).  One element per lane
// with a workgroup per 4 KiB: on gfx950 this streams about 6.2 TB/s, where a
// grid-stride copy over a fixed 8192-workgroup grid (each lane striding the
// whole grid's 32 MiB) stays near 4.6 TB/s.
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
                           hipStream_t s, double nudt, double hv) {
  const size_t n = (size_t)(nv + 1) * nx;
  hipLaunchKernelGGL(assemble_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, U, rowmap, uT, nv,
                     nx, nudt, hv);
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
                           double p, double q, double hv, double *lam, hipStream_t s) {
  const size_t n = (size_t)(J - 1) * nt * nx;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(u0_guess_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, u0, nx, nt, J, ab,
                     tr, p, q, hv, lam);
  return hipGetLastError();
}

hipError_t launch_bw_probe(const void *src, void *dst, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 16;
  if (n == 0) return hipSuccess;
  size_t g = (n + 255) / 256;
  if (g > (1u << 22)) g = 1u << 22;  // beyond 16 GiB the grid-stride loop takes over
  hipLaunchKernelGGL(bw_probe_kernel, dim3((unsigned)g), dim3(256), 0, s, (const double2 *)src,
                     (double2 *)dst, n);
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

// (waves, seg_max, lane groups)
#define KFP_MARCH_CONFIGS(X) \
  X(1, 4, 1) X(1, 8, 1) X(1, 12, 1) X(1, 16, 1) X(1, 24, 1) X(1, 32, 1) \
  X(2, 4, 1) X(2, 8, 1) X(2, 12, 1) X(2, 16, 1) X(2, 24, 1) X(2, 32, 1) \
  X(4, 4, 1) X(4, 6, 1) X(4, 8, 1) X(4, 12, 1) X(4, 16, 1) X(4, 20, 1) X(4, 24, 1) X(4, 32, 1) \
  X(8, 4, 1) X(8, 6, 1) X(8, 8, 1) X(8, 10, 1) X(8, 12, 1) X(8, 14, 1) X(8, 17, 1) X(8, 20, 1) \
  X(8, 24, 1) X(8, 33, 1) \
  X(16, 4, 1) X(16, 6, 1) X(16, 8, 1) X(16, 9, 1) X(16, 10, 1) X(16, 12, 1) \
  X(4, 8, 2) X(8, 17, 2) X(8, 24, 2) X(8, 33, 2) X(8, 33, 4)

bool march_config_supported(int waves, int groups, int seg_max) {
#define KFP_CHECK(W, S, G) \
  if (waves == W && seg_max == S && groups == G) return true;
  KFP_MARCH_CONFIGS(KFP_CHECK)
#undef KFP_CHECK
  return false;
}

static int device_cus();
int device_cu_count() { return device_cus(); }

static int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        n > 0)
      cus = n;
    else
      cus = 256;
  }
  return cus;
}

// (waves, seg_max, tiles per wavefront) of the multi-tile finite-difference
// march, built for up to 256 registers (one 8-wave workgroup per compute
// unit); the one-tile builds of at most 17 rows also for 128 registers (two
// workgroups per compute unit), which launches with two or more work items
// per compute unit run
#define KFP_FD_CONFIGS(X) \
  X(8, 17, 2) X(8, 17, 1) X(8, 12, 2) X(8, 12, 1) X(8, 24, 1) X(8, 33, 1) \
  X(4, 20, 2) X(4, 20, 1) X(4, 12, 2) X(4, 8, 2)

bool fd_config_supported(int waves, int seg_max, int tiles) {
#define KFP_CHECK(W, S, T) \
  if (waves == W && seg_max == S && tiles == T) return true;
  KFP_FD_CONFIGS(KFP_CHECK)
#undef KFP_CHECK
  return false;
}

static hipError_t launch_march_fd(const StepTables &t, int waves, int seg_max, int tiles, int n0,
                                  int S, int H, int src, int par, int grid, hipStream_t s) {
  if (t.fem || S < 1 || S > kMaxStepsFd || H < 1 || 2 * H >= 64) return hipErrorInvalidValue;
  if (tiles == 1 && waves == 8 && (seg_max == 17 || seg_max == 12) && grid >= 2 * device_cus()) {
    if (seg_max == 17)
      hipLaunchKernelGGL((march_fd_kernel<17, 8, 1, 4>), dim3(grid), dim3(512), 0, s, t, n0, S, H,
                         src, par);
    else
      hipLaunchKernelGGL((march_fd_kernel<12, 8, 1, 4>), dim3(grid), dim3(512), 0, s, t, n0, S, H,
                         src, par);
    return hipGetLastError();
  }
#define KFP_LAUNCH(W, SM, T)                                                               \
  if (waves == W && seg_max == SM && tiles == T) {                                        \
    hipLaunchKernelGGL((march_fd_kernel<SM, W, T, 2>), dim3(grid), dim3(W * 64), 0, s, t, n0, \
                       S, H, src, par);                                                   \
    return hipGetLastError();                                                             \
  }
  KFP_FD_CONFIGS(KFP_LAUNCH)
#undef KFP_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_march(const StepTables &t, int waves, int groups, int seg_max, int tiles,
                        int n0, int S, int H, int src, int par, int grid, hipStream_t s) {
  if (tiles > 0)
    return groups == 1 ? launch_march_fd(t, waves, seg_max, tiles, n0, S, H, src, par, grid, s)
                       : hipErrorInvalidValue;
  if (groups < 1 || S < 1 || S > kMaxStepsPerLaunch || H < 1 || 2 * H * groups >= 64)
    return hipErrorInvalidValue;
  // 8 wavefronts of 17 rows (the 131-row subdomains of J = 8 on 1024 and
  // J = 32 on 4096 v-cells): with two or more work items per compute unit,
  // the build limited to 128 registers (two resident workgroups per compute
  // unit, a few spilled values) is the faster one; with one item per
  // compute unit the unlimited build is.  Same arithmetic, same results.
  if (t.fem) {
#define KFP_LAUNCH_FEM(W, SM, G)                                                           \
  if (waves == W && seg_max == SM && groups == G) {                                       \
    hipLaunchKernelGGL((march_kernel<SM, W, G, 1, true>), dim3(grid), dim3(W * 64), 0, s, t, \
                       n0, S, H, src, par);                                               \
    return hipGetLastError();                                                             \
  }
    KFP_MARCH_CONFIGS(KFP_LAUNCH_FEM)
#undef KFP_LAUNCH_FEM
    return hipErrorInvalidValue;
  }
  if (waves == 8 && seg_max == 17 && groups == 1 && grid >= 2 * device_cus()) {
    hipLaunchKernelGGL((march_kernel<17, 8, 1, 4>), dim3(grid), dim3(8 * 64), 0, s, t, n0, S, H,
                       src, par);
    return hipGetLastError();
  }
#define KFP_LAUNCH(W, SM, G)                                                                \
  if (waves == W && seg_max == SM && groups == G) {                                        \
    hipLaunchKernelGGL((march_kernel<SM, W, G>), dim3(grid), dim3(W * 64), 0, s, t, n0, S, \
                       H, src, par);                                                       \
    return hipGetLastError();                                                              \
  }
  KFP_MARCH_CONFIGS(KFP_LAUNCH)
#undef KFP_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_exchange(const StepTables &t, int par, int S, hipStream_t s, int mode) {
  if (t.n_ex == 0) return hipSuccess;
  if (mode < 0 || mode > 2) return hipErrorInvalidValue;
  // a block of S levels is S * nx nodes per interface: fewer workgroups then.
  // A whole window: 1024 workgroups per interface (at 4096 x 8192 nodes per
  // interface, 8 chunks of 1024 nodes per workgroup; measured against 256
  // and 2048 workgroups, and 2 or 8 nodes per thread)
  const unsigned gx = t.blk ? 32u : 1024u;
  hipLaunchKernelGGL(exchange_kernel, dim3(gx, t.n_ex), dim3(256), 0, s, t, par, S, mode);
  return hipGetLastError();
}

hipError_t launch_pipe_tick(PipeCtl *c, int *blk, int *iter, unsigned long long *res,
                            double *hist, hipStream_t s) {
  hipLaunchKernelGGL(pipe_tick_kernel, dim3(1), dim3(64), 0, s, c, blk, iter, res, hist);
  return hipGetLastError();
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
