/*
 * kfp_oracle.c -- CPU FP64 oracle for the Schwarz waveform relaxation (SWR)
 * method for the Kolmogorov equation  u_t + v u_x - u_vv = f  on
 * [0,T] x [0,1)_periodic x [-1,1]  (Section 6.1, eq. (6.1)).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously correct
 * restatement of the discrete method.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the GPU library, and it never calls it.
 *
 * Discretisation (Section 6.2, read as an IMEX Euler step; see readings R2-R6
 * in the design notes):
 *   grid:       h_x = 1/Nx, x_m = m h_x (m = 0..Nx-1, periodic)
 *               h_v = 2/Nv, v_i = -1 + i h_v (i = 0..Nv)
 *               dt = T/Nt, nu_i = v_i dt / h_x, r = dt / h_v^2
 *   transport:  first-order upwind interpolation in x, eqs. (6.4)/(6.5):
 *               (T U)_{i,m} = (1-|nu_i|) U_{i,m} + |nu_i| U_{i,m-sgn(v_i)}
 *   source:     rhs = T U^n + dt * s(t_{n+1}) * f
 *   diffusion:  implicit Euler in v, one tridiagonal system per x-column,
 *               eq. (6.2) with finite differences:
 *               -r U_{i-1} + (1+2r) U_i - r U_{i+1} = rhs_i
 *   boundary:   U = 0 at v = -1 and v = +1.
 *
 * SWR (Section 6.3): overlapping split in v, interface variables (6.7),
 * subdomain solves (6.8)/(6.10), trace updates (6.9)/(6.11), the stopping
 * test (6.12), and the parallel (Jacobi) variant of the Remark that follows
 * (6.12): every subdomain of iteration k reads only the traces of k-1.
 * Transmission operators: Q = I (classical, Dirichlet) or
 * Q_1 = p + d/dv at beta, Q_2 = q - d/dv at alpha (optimized, Robin), with
 * q = p (one-sided OSWR(p), Section 6.4.1).  Derivatives at the interface
 * node are one-sided first-order differences taken inside the subdomain that
 * owns the condition.
 *
 * Without overlap (L = beta - alpha = 0, Section 6.3 allows it for OSWR) the
 * two neighbours share the interface node.  Each one's row there is the
 * balance of the half cell it owns next to the node, with the flux through
 * the interface given by its Robin condition (the row linear finite elements
 * with a lumped mass give for the natural Robin condition):
 *   subdomain below, Q_1 u = (p + d/dv) u = lambda_1, flux d/dv u = lambda_1 - p u:
 *     (h/2)(u^{n+1} - T u^n)/dt - (lambda_1 - p u) + (u_b - u_{b-1})/h = (h/2) s f
 *   subdomain above, Q_2 u = (q - d/dv) u = lambda_2, flux d/dv u = q u - lambda_2.
 * The neighbour's trace then needs no difference across the node: its
 * derivative follows from its own Robin condition, so
 *   Q_2 u_j = (p + q) u_j - lambda_1,   Q_1 u_{j+1} = (p + q) u_{j+1} - lambda_2
 * (with p = q, lambda_new = 2p u - lambda_old).  At a fixed point the two
 * half-cell rows add up to the monodomain row of the shared node.
 *
 * A second discretisation, Section 6.2 as printed (linear finite elements
 * with the consistent mass matrix, Neumann ends, diffusion then transport),
 * is selected by scheme KFP_O_FEM; its definition is given with its code
 * below (fem_solve_subdomain, fem_emit_trace).
 *
 * Every linear system is solved by plain Thomas elimination, written out here
 * with divisions, rebuilt for every column and every step.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define KFP_O_DIRICHLET 0
#define KFP_O_ROBIN 1
#define KFP_O_FD 0  /* finite differences, IMEX step (the default discretisation) */
#define KFP_O_FEM 1 /* linear finite elements, diffusion then transport (Section 6.2) */

/* ------------------------------------------------------------------ */
/* Thomas elimination for a tridiagonal system.                        */
/* Row i:  lo[i] x[i-1] + di[i] x[i] + up[i] x[i+1] = rhs[i]           */
/* (lo[0] and up[n-1] are ignored).  Work arrays cp, dp of length n.  */
/* ------------------------------------------------------------------ */
static void thomas(int n, const double *lo, const double *di, const double *up,
                   const double *rhs, double *x, double *cp, double *dp) {
  double den = di[0];
  cp[0] = (n > 1) ? up[0] / den : 0.0;
  dp[0] = rhs[0] / den;
  for (int i = 1; i < n; ++i) {
    den = di[i] - lo[i] * cp[i - 1];
    cp[i] = (i < n - 1) ? up[i] / den : 0.0;
    dp[i] = (rhs[i] - lo[i] * dp[i - 1]) / den;
  }
  x[n - 1] = dp[n - 1];
  for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
}

int oracle_thomas(int n, const double *lo, const double *di, const double *up,
                  const double *rhs, double *x) {
  if (n < 1) return 1;
  double *cp = (double *)malloc(sizeof(double) * n);
  double *dp = (double *)malloc(sizeof(double) * n);
  thomas(n, lo, di, up, rhs, x, cp, dp);
  free(cp);
  free(dp);
  return 0;
}

/* Upwind transport of one v-row, eqs. (6.4)/(6.5):  v < 0 takes the
 * neighbour at m+1, v > 0 the neighbour at m-1, periodic in x. */
static void transport_row(int nx, double nu, const double *in, double *out) {
  double w = fabs(nu);
  for (int m = 0; m < nx; ++m) {
    int nb;
    if (nu > 0.0)
      nb = (m - 1 + nx) % nx;
    else if (nu < 0.0)
      nb = (m + 1) % nx;
    else
      nb = m;
    out[m] = (1.0 - w) * in[m] + w * in[nb];
  }
}

/* Exposed for the transport pins: applies the x-transport of one time step
 * to every interior v-row of a full [nv+1][nx] field. */
int oracle_transport(int nx, int nv, int nt, double T, const double *U, double *out) {
  if (nx < 1 || nv < 2 || nt < 1 || !(T > 0)) return 1;
  double hx = 1.0 / nx, hv = 2.0 / nv, dt = T / nt;
  for (int i = 0; i <= nv; ++i) {
    double v = -1.0 + i * hv;
    transport_row(nx, v * dt / hx, U + (size_t)i * nx, out + (size_t)i * nx);
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Monodomain reference: the discrete solution on the whole v-range.   */
/* u0, f: [nv+1][nx]; s: [nt+1] or NULL (s == 1); uT: [nv+1][nx].      */
/* ------------------------------------------------------------------ */
int oracle_mono_solve(int nx, int nv, int nt, double T, const double *u0,
                      const double *f, const double *s, double *uT) {
  if (nx < 1 || nv < 2 || nt < 1 || !(T > 0)) return 1;
  const double hx = 1.0 / nx, hv = 2.0 / nv, dt = T / nt, r = dt / (hv * hv);
  const size_t N = (size_t)(nv + 1) * nx;
  double *U = (double *)malloc(sizeof(double) * N);
  double *V = (double *)malloc(sizeof(double) * N);
  memcpy(U, u0, sizeof(double) * N);
  for (int m = 0; m < nx; ++m) U[m] = U[(size_t)nv * nx + m] = 0.0;
  const int nu_ = nv - 1; /* unknown rows 1..nv-1 */
  for (int n = 0; n < nt; ++n) {
    const double g = dt * (s ? s[n + 1] : 1.0);
    /* transport + source, row by row */
    for (int i = 1; i < nv; ++i) {
      double v = -1.0 + i * hv;
      transport_row(nx, v * dt / hx, U + (size_t)i * nx, V + (size_t)i * nx);
      for (int m = 0; m < nx; ++m) V[(size_t)i * nx + m] += g * f[(size_t)i * nx + m];
    }
    /* implicit diffusion, column by column */
#pragma omp parallel
    {
      double *lo = (double *)malloc(sizeof(double) * nu_ * 6);
      double *di = lo + nu_, *up = di + nu_, *rhs = up + nu_, *cp = rhs + nu_, *dp = cp + nu_;
      double *x = (double *)malloc(sizeof(double) * nu_);
#pragma omp for schedule(static)
      for (int m = 0; m < nx; ++m) {
        for (int k = 0; k < nu_; ++k) {
          lo[k] = -r;
          di[k] = 1.0 + 2.0 * r;
          up[k] = -r;
          rhs[k] = V[(size_t)(k + 1) * nx + m];
        }
        /* neighbours v = -1 and v = +1 are zero: nothing moves to the rhs */
        thomas(nu_, lo, di, up, rhs, x, cp, dp);
        for (int k = 0; k < nu_; ++k) U[(size_t)(k + 1) * nx + m] = x[k];
      }
      free(lo);
      free(x);
    }
  }
  memcpy(uT, U, sizeof(double) * N);
  free(U);
  free(V);
  return 0;
}

/* ------------------------------------------------------------------ */
/* SWR                                                                  */
/* ------------------------------------------------------------------ */

/* Overlapping partition of the v-nodes into J subdomains [a_j, b_j]
 * (eq. (6.6) generalised to J pieces): the core cuts are c_j = j nv / J, and
 * an overlap of o cells is placed ceil(o/2) above and floor(o/2) below each
 * cut.  Returns nonzero for an invalid request. */
int oracle_partition(int nv, int J, int o, int *a, int *b) {
  if (J < 1 || o < 0 || nv % J != 0 || nv / J < o + 2) return 1;
  const int w = nv / J;
  a[0] = 0;
  b[J - 1] = nv;
  for (int j = 0; j + 1 < J; ++j) {
    int c = (j + 1) * w;
    b[j] = c + (o + 1) / 2;
    a[j + 1] = c - o / 2;
  }
  return 0;
}

typedef struct {
  int a, b;      /* node range of the subdomain (inclusive)            */
  int left_if;   /* 1 if the lower end a is an interface (j > 0)       */
  int right_if;  /* 1 if the upper end b is an interface (j < J-1)     */
  int nonovl;    /* 1 if the interfaces have no overlap (shared nodes) */
} sub_t;

/* Solves one subdomain over the whole window for one SWR iteration.
 * lamL: data at the lower interface node a (time levels 1..nt, [nt][nx]),
 * lamR: data at the upper interface node b.  The full node-range solution of
 * every time level 1..nt is written to hist[n-1][node-a][m]. */
static void solve_subdomain(int nx, int nv, int nt, double T, const double *u0,
                            const double *f, const double *s, const sub_t *sd,
                            int tr, double p, double q, const double *lamL,
                            const double *lamR, double *hist) {
  const double hx = 1.0 / nx, hv = 2.0 / nv, dt = T / nt, r = dt / (hv * hv);
  const int a = sd->a, b = sd->b, nn = b - a + 1;
  const int robL = sd->left_if && tr == KFP_O_ROBIN;
  const int robR = sd->right_if && tr == KFP_O_ROBIN;
  const int nonovl = sd->nonovl && tr == KFP_O_ROBIN; /* half-cell interface rows */
  const double hc = 2.0 * dt / hv;                    /* flux weight of a half-cell row */
  /* unknown nodes lo..hi; the others are fixed (zero, or Dirichlet data) */
  const int lo = robL ? a : a + 1;
  const int hi = robR ? b : b - 1;
  const int nu_ = hi - lo + 1;
  const size_t plane = (size_t)nn * nx;
  double *U = (double *)malloc(sizeof(double) * plane);
  double *V = (double *)malloc(sizeof(double) * plane);
  for (int i = a; i <= b; ++i)
    memcpy(U + (size_t)(i - a) * nx, u0 + (size_t)i * nx, sizeof(double) * nx);
  for (int n = 0; n < nt; ++n) {
    const double g = dt * (s ? s[n + 1] : 1.0);
    const double *LL = lamL ? lamL + (size_t)n * nx : NULL; /* level n+1 */
    const double *LR = lamR ? lamR + (size_t)n * nx : NULL;
    for (int i = lo; i <= hi; ++i) {
      double *out = V + (size_t)(i - a) * nx;
      if (!nonovl && ((i == a && robL) || (i == b && robR))) continue; /* Robin rows */
      double v = -1.0 + i * hv;
      transport_row(nx, v * dt / hx, U + (size_t)(i - a) * nx, out);
      for (int m = 0; m < nx; ++m) out[m] += g * f[(size_t)i * nx + m];
    }
#pragma omp parallel
    {
      double *lo_ = (double *)malloc(sizeof(double) * nu_ * 7);
      double *di = lo_ + nu_, *up = di + nu_, *rhs = up + nu_, *cp = rhs + nu_,
             *dp = cp + nu_, *x = dp + nu_;
#pragma omp for schedule(static)
      for (int m = 0; m < nx; ++m) {
        for (int i = lo; i <= hi; ++i) {
          int k = i - lo;
          if (i == a && robL && nonovl) { /* half cell above the shared node */
            lo_[k] = 0.0;
            di[k] = 1.0 + 2.0 * r + hc * q;
            up[k] = -2.0 * r;
            rhs[k] = V[(size_t)(i - a) * nx + m] + hc * LL[m];
          } else if (i == b && robR && nonovl) { /* half cell below the shared node */
            lo_[k] = -2.0 * r;
            di[k] = 1.0 + 2.0 * r + hc * p;
            up[k] = 0.0;
            rhs[k] = V[(size_t)(i - a) * nx + m] + hc * LR[m];
          } else if (i == a && robL) { /* Q_2 u = (q - d/dv) u at alpha */
            lo_[k] = 0.0;
            di[k] = q + 1.0 / hv;
            up[k] = -1.0 / hv;
            rhs[k] = LL[m];
          } else if (i == b && robR) { /* Q_1 u = (p + d/dv) u at beta */
            lo_[k] = -1.0 / hv;
            di[k] = p + 1.0 / hv;
            up[k] = 0.0;
            rhs[k] = LR[m];
          } else {
            lo_[k] = -r;
            di[k] = 1.0 + 2.0 * r;
            up[k] = -r;
            rhs[k] = V[(size_t)(i - a) * nx + m];
            /* a fixed neighbour node moves to the right-hand side */
            if (i - 1 < lo) {
              double fixed = (i - 1 == a && sd->left_if) ? LL[m] : 0.0;
              rhs[k] += r * fixed;
            }
            if (i + 1 > hi) {
              double fixed = (i + 1 == b && sd->right_if) ? LR[m] : 0.0;
              rhs[k] += r * fixed;
            }
          }
        }
        thomas(nu_, lo_, di, up, rhs, x, cp, dp);
        for (int i = lo; i <= hi; ++i) U[(size_t)(i - a) * nx + m] = x[i - lo];
        /* fixed nodes at the new level */
        if (lo > a) U[m] = sd->left_if ? LL[m] : 0.0;
        if (hi < b) U[(size_t)(b - a) * nx + m] = sd->right_if ? LR[m] : 0.0;
      }
      free(lo_);
    }
    memcpy(hist + (size_t)n * plane, U, sizeof(double) * plane);
  }
  free(U);
  free(V);
}

/* ------------------------------------------------------------------ */
/* The paper's own discretisation (Section 6.2, scheme KFP_O_FEM).      */
/* ------------------------------------------------------------------ */
/* Linear finite elements in v on the same nodes: the mass matrix M and the
 * stiffness matrix S of (6.3) have the exact element integrals (the Remark
 * after (6.5): Simpson's rule is exact for them), per element [v_e, v_{e+1}]
 *   M_e = h/6 [[2, 1], [1, 2]],   S_e = 1/h [[1, -1], [-1, 1]].
 * v = -1 and v = +1 carry the homogeneous Neumann condition of (6.1), which
 * is natural: the end nodes are unknowns and their rows hold one element.
 * A time step is the splitting of Section 6.2 in its order:
 *   Step 1  (M/dt + S) W^{n+1} = M/dt G^n,  G^n = U^n + dt s(t_{n+1}) f
 *           (implicit Euler for the v-diffusion, the source taken with it),
 *   Step 2  U^{n+1} = T W^{n+1}, the upwind transport (6.4)/(6.5),
 * both stages over the whole step dt (the half step printed for them would
 * advance the solution by dt/2 per step); U^0 = u0.
 * Every row is multiplied by dt/h, so an element adds
 *   (1/6) [[2, 1], [1, 2]] + r [[1, -1], [-1, 1]],   r = dt/h^2,
 * to the matrix and (1/6) [[2, 1], [1, 2]] G to the right-hand side.
 * Interface conditions act in Step 1.  A Robin condition is natural:
 *   Q_1 u = (p + d/dv) u = lambda_1 at beta (upper end): the boundary term
 *     -u_v(beta) phi_beta = (p u - lambda_1) phi_beta adds dt/h p to the
 *     diagonal and dt/h lambda_1 to the right-hand side;
 *   Q_2 u = (q - d/dv) u = lambda_2 at alpha (lower end): likewise with q.
 * This holds with or without overlap.  A classical (Dirichlet) interface
 * node is a fixed node holding the trace; its element still contributes to
 * the row next to it. */

/* Builds the state U^n of node i (index i - a in the subdomain's history)
 * for column m: u0 at n = 0, else the transport of W^n. */
static double fem_stage_input(int nx, int nv, int nt, double T, const double *u0, int a,
                              int nn, const double *hist, int i, int n, int m) {
  if (n == 0) return u0[(size_t)i * nx + m];
  const double hx = 1.0 / nx, hv = 2.0 / nv, dt = T / nt;
  const double nu = (-1.0 + i * hv) * dt / hx, w = fabs(nu);
  const double *row = hist + ((size_t)(n - 1) * nn + (i - a)) * nx;
  int nb = m;
  if (nu > 0.0) nb = (m - 1 + nx) % nx;
  if (nu < 0.0) nb = (m + 1) % nx;
  return (1.0 - w) * row[m] + w * row[nb];
}

/* One subdomain over the whole window: W^{n+1} of every level of its nodes
 * a..b (fixed nodes included) to hist[n][i-a][m]. */
static void fem_solve_subdomain(int nx, int nv, int nt, double T, const double *u0,
                                const double *f, const double *s, const sub_t *sd, int tr,
                                double p, double q, const double *lamL, const double *lamR,
                                double *hist) {
  const double hx = 1.0 / nx, hv = 2.0 / nv, dt = T / nt, r = dt / (hv * hv), k = dt / hv;
  const int a = sd->a, b = sd->b, nn = b - a + 1;
  const int dirL = sd->left_if && tr == KFP_O_DIRICHLET;
  const int dirR = sd->right_if && tr == KFP_O_DIRICHLET;
  const int robL = sd->left_if && tr == KFP_O_ROBIN;
  const int robR = sd->right_if && tr == KFP_O_ROBIN;
  const int lo = dirL ? a + 1 : a, hi = dirR ? b - 1 : b, nu_ = hi - lo + 1;
  const size_t plane = (size_t)nn * nx;
  double *U = (double *)malloc(sizeof(double) * plane); /* U^n */
  double *G = (double *)malloc(sizeof(double) * plane);
  for (int i = a; i <= b; ++i)
    memcpy(U + (size_t)(i - a) * nx, u0 + (size_t)i * nx, sizeof(double) * nx);
  for (int n = 0; n < nt; ++n) {
    const double gs = dt * (s ? s[n + 1] : 1.0);
    for (int i = a; i <= b; ++i)
      for (int m = 0; m < nx; ++m)
        G[(size_t)(i - a) * nx + m] = U[(size_t)(i - a) * nx + m] + gs * f[(size_t)i * nx + m];
    double *W = hist + (size_t)n * plane;
    const double *LL = lamL ? lamL + (size_t)n * nx : NULL; /* level n+1 */
    const double *LR = lamR ? lamR + (size_t)n * nx : NULL;
#pragma omp parallel
    {
      double *lo_ = (double *)malloc(sizeof(double) * nu_ * 7);
      double *di = lo_ + nu_, *up = di + nu_, *rhs = up + nu_, *cp = rhs + nu_,
             *dp = cp + nu_, *x = dp + nu_;
#pragma omp for schedule(static)
      for (int m = 0; m < nx; ++m) {
        for (int t = 0; t < nu_; ++t) lo_[t] = di[t] = up[t] = rhs[t] = 0.0;
        /* element by element */
        for (int e = a; e < b; ++e) {
          for (int ii = 0; ii < 2; ++ii) {
            const int i = e + ii; /* row */
            if (i < lo || i > hi) continue;
            for (int jj = 0; jj < 2; ++jj) {
              const int jn = e + jj; /* column */
              const double me = (ii == jj ? 2.0 : 1.0) / 6.0;
              const double ke = (ii == jj ? r : -r);
              rhs[i - lo] += me * G[(size_t)(jn - a) * nx + m];
              if (jn >= lo && jn <= hi) {
                if (jn == i) di[i - lo] += me + ke;
                else if (jn < i) lo_[i - lo] += me + ke;
                else up[i - lo] += me + ke;
              } else { /* a fixed (Dirichlet) node: its level n+1 value moves over */
                const double fixed = (jn == a) ? LL[m] : LR[m];
                rhs[i - lo] -= (me + ke) * fixed;
              }
            }
          }
        }
        if (robL) { /* (q - d/dv) u = lambda_2 at alpha */
          di[0] += k * q;
          rhs[0] += k * LL[m];
        }
        if (robR) { /* (p + d/dv) u = lambda_1 at beta */
          di[nu_ - 1] += k * p;
          rhs[nu_ - 1] += k * LR[m];
        }
        thomas(nu_, lo_, di, up, rhs, x, cp, dp);
        for (int i = lo; i <= hi; ++i) W[(size_t)(i - a) * nx + m] = x[i - lo];
        if (dirL) W[m] = LL[m];
        if (dirR) W[(size_t)(b - a) * nx + m] = LR[m];
      }
      free(lo_);
    }
    /* Step 2: U^{n+1} = T W^{n+1}, row by row */
    for (int i = a; i <= b; ++i) {
      const double v = -1.0 + i * hv;
      transport_row(nx, v * dt / hx, W + (size_t)(i - a) * nx, U + (size_t)(i - a) * nx);
    }
  }
  free(U);
  free(G);
}

/* Interface data of the finite-element scheme with overlap.  The derivative
 * in Q is the flux the sender's own elements next to the node carry: the
 * weak form of Step 1 over the element below node i gives u_v(v_i) as
 *   F_lo(i) = h/(6 dt) [(W_{i-1} - G_{i-1}) + 2 (W_i - G_i)] + (W_i - W_{i-1})/h,
 * and over the element above, -u_v(v_i) as
 *   F_up(i) = h/(6 dt) [2 (W_i - G_i) + (W_{i+1} - G_{i+1})] + (W_i - W_{i+1})/h.
 * Q_2 u_j = q W - F_lo at alpha = a_{j+1} (elements of u_j below alpha) and
 * Q_1 u_{j+1} = p W - F_up at beta = b_j (elements of u_{j+1} above beta).
 * The monodomain row of an interior node is F_lo + F_up = 0, so the
 * monodomain solution is a fixed point of the iteration. */
static void fem_emit_trace(int nx, int nv, int nt, double T, const double *u0, const double *f,
                           const double *s, int j, int side, const int *a, const int *b, int o,
                           int tr, double p, double q, const double *Ul, const double *Ur,
                           const double *lam_used, double *lam_out) {
  const size_t P = (size_t)nt * nx;
  const double hv = 2.0 / nv, dt = T / nt, cm = hv / (6.0 * dt);
  const int al = a[j + 1], be = b[j];
  const int nnL = b[j] - a[j] + 1, nnR = b[j + 1] - a[j + 1] + 1;
  for (int n = 0; n < nt; ++n) {
    const double gs = dt * (s ? s[n + 1] : 1.0);
    const double *UL = Ul + (size_t)n * nnL * nx; /* W^{n+1} of u_j */
    const double *UR = Ur + (size_t)n * nnR * nx; /* W^{n+1} of u_{j+1} */
    for (int m = 0; m < nx; ++m) {
      const size_t e = (size_t)n * nx + m;
      if (side == 0) {
        const double w0 = UL[(size_t)(al - a[j]) * nx + m];
        double v = w0;
        if (tr == KFP_O_ROBIN && o == 0) {
          v = (p + q) * w0 - lam_used[(size_t)(2 * j + 1) * P + e];
        } else if (tr == KFP_O_ROBIN) {
          const double w1 = UL[(size_t)(al - 1 - a[j]) * nx + m];
          const double g0 = fem_stage_input(nx, nv, nt, T, u0, a[j], nnL, Ul, al, n, m) +
                            gs * f[(size_t)al * nx + m];
          const double g1 = fem_stage_input(nx, nv, nt, T, u0, a[j], nnL, Ul, al - 1, n, m) +
                            gs * f[(size_t)(al - 1) * nx + m];
          const double flo = cm * ((w1 - g1) + 2.0 * (w0 - g0)) + (w0 - w1) / hv;
          v = q * w0 - flo;
        }
        lam_out[(size_t)(2 * j) * P + e] = v;
      } else {
        const double w0 = UR[(size_t)(be - a[j + 1]) * nx + m];
        double v = w0;
        if (tr == KFP_O_ROBIN && o == 0) {
          v = (p + q) * w0 - lam_used[(size_t)(2 * j) * P + e];
        } else if (tr == KFP_O_ROBIN) {
          const double w1 = UR[(size_t)(be + 1 - a[j + 1]) * nx + m];
          const double g0 = fem_stage_input(nx, nv, nt, T, u0, a[j + 1], nnR, Ur, be, n, m) +
                            gs * f[(size_t)be * nx + m];
          const double g1 = fem_stage_input(nx, nv, nt, T, u0, a[j + 1], nnR, Ur, be + 1, n, m) +
                            gs * f[(size_t)(be + 1) * nx + m];
          const double fup = cm * (2.0 * (w0 - g0) + (w1 - g1)) + (w0 - w1) / hv;
          v = p * w0 - fup;
        }
        lam_out[(size_t)(2 * j + 1) * P + e] = v;
      }
    }
  }
}

/* Owner of node i when the subdomain pieces are glued into one field:
 * the subdomain whose core [c_j, c_{j+1}) holds i, moved one down when i is
 * that subdomain's fixed Dirichlet node. */
static int owner(int i, int nv, int J, const int *a, int tr) {
  int j = i / (nv / J);
  if (j > J - 1) j = J - 1;
  if (j > 0 && i == a[j] && tr == KFP_O_DIRICHLET) j -= 1;
  return j;
}

/* Trace that one side of interface j sends to the other, eqs. (6.9)/(6.11).
 * side 0: plane 2j = Q_2 u_j at alpha = a_{j+1} (the data of subdomain j+1);
 * side 1: plane 2j+1 = Q_1 u_{j+1} at beta = b_j (the data of subdomain j).
 * Ul, Ur: iterates of subdomains j and j+1 over the window; lam_used: the
 * traces the sending subdomain was solved with (read only without overlap,
 * where the derivative comes from the sender's own Robin condition);
 * lam_out: receives the plane. */
static void emit_trace(int nx, int nt, int j, int side, const int *a, const int *b, int o,
                       int tr, double p, double q, double hv, const double *Ul,
                       const double *Ur, const double *lam_used, double *lam_out) {
  const size_t P = (size_t)nt * nx;
  const int al = a[j + 1], be = b[j];
  const int nnL = b[j] - a[j] + 1, nnR = b[j + 1] - a[j + 1] + 1;
  for (int n = 0; n < nt; ++n) {
    const double *UL = Ul + (size_t)n * nnL * nx; /* u_j     */
    const double *UR = Ur + (size_t)n * nnR * nx; /* u_{j+1} */
    for (int m = 0; m < nx; ++m) {
      const size_t e = (size_t)n * nx + m;
      if (side == 0) {
        const double uLa = UL[(size_t)(al - a[j]) * nx + m];
        double v = uLa;
        if (tr == KFP_O_ROBIN && o == 0) {
          v = (p + q) * uLa - lam_used[(size_t)(2 * j + 1) * P + e];
        } else if (tr == KFP_O_ROBIN) {
          const double uLa1 = UL[(size_t)(al + 1 - a[j]) * nx + m];
          v = q * uLa - (uLa1 - uLa) / hv;
        }
        lam_out[(size_t)(2 * j) * P + e] = v;
      } else {
        const double uRb = UR[(size_t)(be - a[j + 1]) * nx + m];
        double v = uRb;
        if (tr == KFP_O_ROBIN && o == 0) {
          v = (p + q) * uRb - lam_used[(size_t)(2 * j) * P + e];
        } else if (tr == KFP_O_ROBIN) {
          const double uRb1 = UR[(size_t)(be - 1 - a[j + 1]) * nx + m];
          v = p * uRb + (uRb - uRb1) / hv;
        }
        lam_out[(size_t)(2 * j + 1) * P + e] = v;
      }
    }
  }
}

/* (6.12): mismatch of the iterates of subdomains j and j+1 on their overlap,
 * over the whole window; *rk: at the two end nodes, *rov: over the closed
 * overlap (a NaN propagates to both). */
static void mismatch(int nx, int nt, int j, const int *a, const int *b, const double *Ul,
                     const double *Ur, double *rk, double *rov) {
  const int al = a[j + 1], be = b[j];
  const int nnL = b[j] - a[j] + 1, nnR = b[j + 1] - a[j + 1] + 1;
  for (int n = 0; n < nt; ++n) {
    const double *UL = Ul + (size_t)n * nnL * nx;
    const double *UR = Ur + (size_t)n * nnR * nx;
    for (int m = 0; m < nx; ++m)
      for (int i = al; i <= be; ++i) {
        double d = fabs(UL[(size_t)(i - a[j]) * nx + m] - UR[(size_t)(i - a[j + 1]) * nx + m]);
        if (!(d <= *rov)) *rov = d;
        if ((i == al || i == be) && !(d <= *rk)) *rk = d;
      }
  }
}

/*
 * oracle_swr_solve_ordered: SWR for J subdomains.
 *   u0, f: [nv+1][nx]; s: [nt+1] or NULL.
 *   tr: 0 Dirichlet (CSWR), 1 Robin: OSWR(p,q) of Section 6.3, the data for
 *     a subdomain's upper interface node is Q_1 u = (p + d/dv) u of its upper
 *     neighbour, the data for its lower node Q_2 u = (q - d/dv) u of its
 *     lower neighbour; q = p is the one-sided OSWR(p).
 *   order: 0 parallel (the Remark after (6.12): every subdomain of iteration
 *     k reads the traces of k-1); 1 multiplicative in red-black order, as
 *     (6.8)-(6.11) are written for two subdomains: iteration k first solves
 *     the even subdomains with the current traces, sends their traces, then
 *     solves the odd ones with those new traces and sends theirs.
 *   lambda_init: [2(J-1)][nt][nx] or NULL (zero).  Plane 2j holds the data
 *     for subdomain j+1 at node a_{j+1} (Q_2 u_j), plane 2j+1 the data for
 *     subdomain j at node b_j (Q_1 u_{j+1}); row n-1 holds time level n.
 *   Stops at the first k >= 1 with r^k < tol, or after max_iter iterations.
 *   Outputs: uT [nv+1][nx]; lambda_out (same shape as lambda_init, or NULL);
 *   iters; res_hist[k-1] = r^k (endpoint form, at the two interface nodes);
 *   ovl_hist[k-1] = the maximum over the whole closed overlap (6.12).
 *   Returns 0 on convergence, 4 when max_iter is reached, 1 on bad input.
 */
int oracle_swr_solve_scheme(int nx, int nv, int nt, double T, const double *u0,
                            const double *f, const double *s, int J, int o, int tr, double p,
                            double q, double tol, int max_iter, const double *lambda_init,
                            int order, int scheme, double *uT, double *lambda_out, int *iters,
                            double *res_hist, double *ovl_hist) {
  if (nx < 1 || nv < 2 || nt < 1 || !(T > 0) || max_iter < 1 || order < 0 || order > 1 ||
      scheme < KFP_O_FD || scheme > KFP_O_FEM)
    return 1;
  int *a = (int *)malloc(sizeof(int) * J), *b = (int *)malloc(sizeof(int) * J);
  if (oracle_partition(nv, J, o, a, b)) {
    free(a);
    free(b);
    return 1;
  }
  if (J > 1 && tr == KFP_O_ROBIN && (!(p > 0) || !(q > 0))) {
    free(a);
    free(b);
    return 1;
  }
  const double hv = 2.0 / nv;
  const size_t P = (size_t)nt * nx; /* one trace plane */
  const int nI = J - 1;
  double *lamOld = (double *)calloc(2 * nI * P + 1, sizeof(double));
  double *lamNew = (double *)calloc(2 * nI * P + 1, sizeof(double));
  if (lambda_init && nI > 0) memcpy(lamOld, lambda_init, sizeof(double) * 2 * nI * P);
  double **hist = (double **)malloc(sizeof(double *) * J);
  sub_t *sd = (sub_t *)malloc(sizeof(sub_t) * J);
  for (int j = 0; j < J; ++j) {
    sd[j].a = a[j];
    sd[j].b = b[j];
    sd[j].left_if = j > 0;
    sd[j].right_if = j < J - 1;
    sd[j].nonovl = o == 0;
    hist[j] = (double *)malloc(sizeof(double) * (size_t)(b[j] - a[j] + 1) * P);
  }
  /* one subdomain solve and one trace, in the chosen discretisation */
#define SOLVE(j, LL, LR)                                                                  \
  do {                                                                                    \
    if (scheme == KFP_O_FEM)                                                              \
      fem_solve_subdomain(nx, nv, nt, T, u0, f, s, &sd[j], tr, p, q, LL, LR, hist[j]);    \
    else                                                                                  \
      solve_subdomain(nx, nv, nt, T, u0, f, s, &sd[j], tr, p, q, LL, LR, hist[j]);        \
  } while (0)
#define EMIT(j, side, used, out)                                                          \
  do {                                                                                    \
    if (scheme == KFP_O_FEM)                                                              \
      fem_emit_trace(nx, nv, nt, T, u0, f, s, j, side, a, b, o, tr, p, q, hist[j],        \
                     hist[(j) + 1], used, out);                                           \
    else                                                                                  \
      emit_trace(nx, nt, j, side, a, b, o, tr, p, q, hv, hist[j], hist[(j) + 1], used,    \
                 out);                                                                    \
  } while (0)
  int k = 0, status = 4;
  for (k = 1; k <= max_iter; ++k) {
    if (order == 0) {
      /* (6.8)/(6.10), parallel form: each subdomain uses traces of k-1 */
      for (int j = 0; j < J; ++j) {
        const double *LL = (j > 0) ? lamOld + (size_t)(2 * (j - 1)) * P : NULL;
        const double *LR = (j < J - 1) ? lamOld + (size_t)(2 * j + 1) * P : NULL;
        SOLVE(j, LL, LR);
      }
      /* (6.9)/(6.11): new interface variables from the neighbours */
      for (int j = 0; j < nI; ++j)
        for (int side = 0; side < 2; ++side) EMIT(j, side, lamOld, lamNew);
      double *t = lamOld;
      lamOld = lamNew;
      lamNew = t;
    } else {
      /* red-black: one set of traces, updated as soon as a colour is solved */
      for (int c = 0; c < 2; ++c) {
        for (int j = c; j < J; j += 2) {
          const double *LL = (j > 0) ? lamOld + (size_t)(2 * (j - 1)) * P : NULL;
          const double *LR = (j < J - 1) ? lamOld + (size_t)(2 * j + 1) * P : NULL;
          SOLVE(j, LL, LR);
        }
        for (int j = 0; j < nI; ++j) {
          if (j % 2 == c) /* subdomain j sends plane 2j */
            EMIT(j, 0, lamOld, lamOld);
          if ((j + 1) % 2 == c) /* subdomain j+1 sends plane 2j+1 */
            EMIT(j, 1, lamOld, lamOld);
        }
      }
    }
    double rk = 0.0, rov = 0.0;
    for (int j = 0; j < nI; ++j) mismatch(nx, nt, j, a, b, hist[j], hist[j + 1], &rk, &rov);
    if (res_hist) res_hist[k - 1] = rk;
    if (ovl_hist) ovl_hist[k - 1] = rov;
    if (rk < tol) {
      status = 0;
      break;
    }
  }
  if (k > max_iter) k = max_iter;
  *iters = k;
#undef SOLVE
#undef EMIT
  /* output: glue the final iterates at t = T (finite elements: glue W^nt,
   * then Step 2 of the last step, row by row) */
  for (int i = 0; i <= nv; ++i) {
    int j = owner(i, nv, J, a, tr);
    const double *src = hist[j] + (size_t)(nt - 1) * (b[j] - a[j] + 1) * nx +
                        (size_t)(i - a[j]) * nx;
    if (scheme == KFP_O_FEM) {
      const double v = -1.0 + i * hv;
      transport_row(nx, v * (T / nt) * nx, src, uT + (size_t)i * nx);
      continue;
    }
    for (int m = 0; m < nx; ++m) uT[(size_t)i * nx + m] = (i == 0 || i == nv) ? 0.0 : src[m];
  }
  if (lambda_out && nI > 0) memcpy(lambda_out, lamOld, sizeof(double) * 2 * nI * P);
  for (int j = 0; j < J; ++j) free(hist[j]);
  free(hist);
  free(sd);
  free(lamOld);
  free(lamNew);
  free(a);
  free(b);
  return status;
}

/* oracle_swr_solve_ordered: oracle_swr_solve_scheme with finite differences. */
int oracle_swr_solve_ordered(int nx, int nv, int nt, double T, const double *u0,
                             const double *f, const double *s, int J, int o, int tr, double p,
                             double q, double tol, int max_iter, const double *lambda_init,
                             int order, double *uT, double *lambda_out, int *iters,
                             double *res_hist, double *ovl_hist) {
  return oracle_swr_solve_scheme(nx, nv, nt, T, u0, f, s, J, o, tr, p, q, tol, max_iter,
                                 lambda_init, order, KFP_O_FD, uT, lambda_out, iters, res_hist,
                                 ovl_hist);
}

/* Monodomain solution of the finite-element scheme (nodes 0..nv, Neumann
 * ends): U^nt = T W^nt. */
int oracle_fem_mono_solve(int nx, int nv, int nt, double T, const double *u0, const double *f,
                          const double *s, double *uT) {
  if (nx < 1 || nv < 2 || nt < 1 || !(T > 0)) return 1;
  sub_t sd = {0, nv, 0, 0, 0};
  const size_t plane = (size_t)(nv + 1) * nx;
  double *hist = (double *)malloc(sizeof(double) * plane * nt);
  fem_solve_subdomain(nx, nv, nt, T, u0, f, s, &sd, KFP_O_DIRICHLET, 0.0, 0.0, NULL, NULL, hist);
  const double hv = 2.0 / nv;
  for (int i = 0; i <= nv; ++i)
    transport_row(nx, (-1.0 + i * hv) * (T / nt) * nx, hist + (size_t)(nt - 1) * plane + (size_t)i * nx,
                  uT + (size_t)i * nx);
  free(hist);
  return 0;
}

/* oracle_swr_solve: the parallel order of oracle_swr_solve_ordered. */
int oracle_swr_solve(int nx, int nv, int nt, double T, const double *u0,
                     const double *f, const double *s, int J, int o, int tr,
                     double p, double q, double tol, int max_iter, const double *lambda_init,
                     double *uT, double *lambda_out, int *iters, double *res_hist,
                     double *ovl_hist) {
  return oracle_swr_solve_ordered(nx, nv, nt, T, u0, f, s, J, o, tr, p, q, tol, max_iter,
                                  lambda_init, 0, uT, lambda_out, iters, res_hist, ovl_hist);
}

/* The "u0-extension" initial guess: lambda^0(n) = Q(u0) at the interface
 * node for every time level n (compatible with u0 at t = 0, Section 2). */
int oracle_u0_guess(int nx, int nv, int nt, const double *u0, int J, int o, int tr,
                    double p, double q, double *lam) {
  int *a = (int *)malloc(sizeof(int) * J), *b = (int *)malloc(sizeof(int) * J);
  if (oracle_partition(nv, J, o, a, b)) {
    free(a);
    free(b);
    return 1;
  }
  const double hv = 2.0 / nv;
  const size_t P = (size_t)nt * nx;
  for (int j = 0; j + 1 < J; ++j) {
    const int al = a[j + 1], be = b[j];
    for (int m = 0; m < nx; ++m) {
      double ua = u0[(size_t)al * nx + m], ua1 = u0[(size_t)(al + 1) * nx + m];
      double ub = u0[(size_t)be * nx + m], ub1 = u0[(size_t)(be - 1) * nx + m];
      double toR = (tr == KFP_O_ROBIN) ? q * ua - (ua1 - ua) / hv : ua;
      double toL = (tr == KFP_O_ROBIN) ? p * ub + (ub - ub1) / hv : ub;
      for (int n = 0; n < nt; ++n) {
        lam[(size_t)(2 * j) * P + (size_t)n * nx + m] = toR;
        lam[(size_t)(2 * j + 1) * P + (size_t)n * nx + m] = toL;
      }
    }
  }
  free(a);
  free(b);
  return 0;
}
