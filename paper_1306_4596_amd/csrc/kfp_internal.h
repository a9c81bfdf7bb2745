// Internal data structures shared by the host runtime and the gfx950 kernels
// of libkfpswr.  Nothing here is part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace kfp {

// How one end of a subdomain's unknown rows meets the outside.
enum EndKind : int {
  END_PHYS = 0,  // v = -1 or v = +1: zero Dirichlet data
  END_DIRI = 1,  // classical interface: the neighbour's trace is a fixed node
  END_ROBIN = 2,  // optimized interface: the end row is a Robin row
  // optimized interface without overlap (the two subdomains share the
  // interface node): the end row is the node's half-cell balance, whose
  // flux through the interface comes from the Robin condition
  END_RFV = 3
};

// One SWR instance, resident in device memory.  All pointers are device
// pointers; lam[0]/lam[1] are the two trace windows (read k-1 / write k).
struct InstDev {
  double *U[2];                 // state ping-pong: rows of all subdomains, [rows][nx]
  const double *u0;             // [nv+1][nx]
  const double *f;              // [nv+1][nx]
  const double *g;              // [nt]: dt * s(t_{n+1})
  double *lam[2];               // [2(J-1)][nt][nx] each
  unsigned long long *res;      // residual of the running iteration (bits of a double >= 0)
  double *V;                    // multi-step path: interface-node values [J-1][6][nt][nx]
  double r;                     // dt / h_v^2
  double p, q;                  // Robin parameters (q = p)
  double hv;                    // h_v
  int nx, nv, nt, tr;
  int active;                   // 0: frozen (converged), skipped by every kernel
  int nonovl;                   // 1: no overlap (END_RFV interface rows)
  int xmode;                    // exchange mode when a launch leaves it to the instance
  int scheme;                   // 0 finite differences; 1 finite elements (FEM_* tables)
  int gconst;                   // 1: g is the same at every level (s constant in time)
};

// Discretisations of the v-diffusion.  SCHEME_FD: finite differences, one
// IMEX step (transport, source, implicit diffusion), zero values at v = +-1.
// SCHEME_FEM: Section 6.2 as printed: linear finite elements with the
// consistent mass matrix, Neumann ends, the diffusion stage before the
// transport.  The march then carries W^n, the diffusion stage's result
// (U^n = T W^n): a step forms G = T W^n + dt s f (G = u0 + dt s f at the
// first step, where nothing has been transported yet) and solves
// (M/dt + S) W^{n+1} = M/dt G; the output is T W^nt.
enum Scheme : int { SCHEME_FD = 0, SCHEME_FEM = 1 };

// One subdomain of one instance.  Rows are local: 0 .. n-1 are the unknown
// rows, row 0 has the smallest v.  Planes index the instance's trace window.
struct SubDev {
  int inst;
  int n;            // unknown rows
  int row_off;      // first row in InstDev::U
  int g_lo;         // global v-node of local row 0
  int tab;          // first RowCoef of this subdomain
  int seg;          // first entry of the segment-start table (P+1 ints)
  int red;          // first RedCoef (P-1 entries)
  int P;            // row segments (one wavefront each)
  int lo_kind, hi_kind;      // EndKind of row 0 / row n-1
  int lam_lo, lam_hi;        // incoming planes for the two ends (-1: none)
  int out_lo_plane, out_lo_row;  // trace Q_1 u at b_{j-1}: plane, local row of b_{j-1}
  int out_hi_plane, out_hi_row;  // trace Q_2 u at a_{j+1}: plane, local row of a_{j+1}
  int res_nb;         // subdomain index of the upper neighbour (-1: no interface above)
  int res_row_a_nb;   // local row of a_{j+1} in the neighbour, -1: fixed node (use plane)
  int res_row_b_self; // local row of b_j here, -1: fixed node (use plane)
  int res_row_b_nb;   // local row of b_j in the neighbour
  int res_plane_a, res_plane_b;  // planes holding the fixed-node values (Dirichlet)
  int pad;            // multi-step layout: leading identity rows of the last segment
  int vsplit;         // first local row with v >= 0 (upwind neighbour at m-1)
  int rinv;           // multi-step layout: first entry of the reduced-system inverse
  int hsides;         // upwind sides of the rows: bit 0 some row has v > 0 (its upwind
                      // neighbour is at m-1), bit 1 some row has v < 0 (at m+1)
};

// Per unknown row: transport weight and the factors of the local (segment)
// Thomas elimination and the two spike vectors of the segment partition.
struct RowCoef {
  double nu;  // signed Courant number v_i dt / h_x
  double fa;  // 1 / pivot
  double fb;  // -sub / pivot (multiplies the previous forward value)
  double bc;  // -c' (multiplies the next backward value)
  double sl;  // spike: response of the segment to its lower separator
  double sr;  // spike: response of the segment to its upper separator
};

// Per padded row of the multi-step layout (every segment exactly SEG rows;
// the last row of a non-final segment is its separator, the last segment
// starts with `pad` identity rows).  The forward elimination is folded into
// the transport: y_k = alpha u_k + beta u_nb + g fs_k + fb y_{k-1}, with
// fs = fa f pre-scaled once per launch; the upwind neighbour u_nb is the
// column at m-1 for v >= 0 and at m+1 for v < 0 (SubDev::vsplit).
// The fields are ordered by the pass that reads them (16-byte pairs): the
// forward elimination (alpha, beta, fb), the spike correction (sl, sr), the
// back substitution (bc); fa and fab are read once per launch.
struct MarchCoef {
  double alpha;  // fa (1 - |nu|)
  double beta;   // fa |nu|
  double fb;     // -sub / pivot
  double fa;     // 1 / pivot (0 on Robin and identity rows: no source there)
  double sl, sr; // spikes (zero on separator and identity rows)
  double bc;     // -c'
  double fab;    // 1 / pivot of an end row that takes boundary data, else 0
};

// The finite-element layout of the same rows (rows scaled by dt/h_v: an
// element adds (1/6)[[2,1],[1,2]] + r[[1,-1],[-1,1]]).  A step first forms G
// in every register (the transport weight |nu| of a row is affine in its
// index and computed in registers), then eliminates with right-hand sides
// wl G_{k-1} + wm G_k + wu G_{k+1}: the mass weights times 1 / pivot
// (unscaled on separator rows).  Rows whose neighbour in G lies outside the
// segment (the first real row below, a separator or the subdomain's last
// row above) have that weight zero here: it is applied from FemSeg or, for a
// separator, in the reduced system.
struct FemCoef {
  double wl, wm, wu;  // mass weights of G_{k-1}, G_k, G_{k+1}, times 1 / pivot
  double fb, bc, sl, sr;  // as in MarchCoef
  double fab;         // 1 / pivot of an end row that takes boundary data, else 0
};

// Per segment of the finite-element layout: the G of the node just below
// the segment's first real row (the separator of the segment below, or the
// fixed node under a classical interface) and just above the subdomain's
// last row (a fixed node above, last segment only).
struct FemSeg {
  double nul, wol;  // signed Courant number of the node below, weight of its G
  double nua, woa;  // the same for the node above
};

// Per separator row of the reduced system.
struct RedCoef {
  double ra;  // sub-diagonal coefficient of the separator row
  double rc;  // super-diagonal coefficient of the separator row
  double g1;  // 1 / pivot of the reduced elimination
  double g2;  // -alpha / pivot
  double h;   // -gamma'
  double rg;  // finite elements: weight of G of the next segment's first row (0 otherwise)
};

// A workgroup's unit of work: subdomain `sub`, x-columns x0 .. x0+63.
struct Item {
  int sub;
  int x0;
};

// One interface of one instance, for the exchange pass of the multi-step path.
struct ExItem {
  int inst;
  int j;      // interface between subdomains j and j+1
  int a, b;   // its nodes a_{j+1} and b_j
};

struct StepTables {
  const InstDev *inst;
  const SubDev *subs;
  const Item *items;
  const RowCoef *rows;
  const RedCoef *reds;
  const int *segs;
  const ExItem *ex;
  const MarchCoef *mrows;
  const FemCoef *frows;  // finite-element layout (instead of mrows)
  const FemSeg *fsegs;   // finite-element layout: per segment, from SubDev::seg
  const double *rinv;  // per multi-step subdomain: (P-1) x (P-1) inverse, row-major
  const int *blk;      // pipelined iterations: time block of each instance this launch
                       // (-1: idle), or nullptr
  int n_items;
  int n_ex;
  int fem;             // the tables are the finite-element layout
};

// Pipelined iterations.  Waveform relaxation is causal in time: iteration k
// at time block b needs only iteration k-1's traces of block b.  Instance
// (slot) i holds iteration k with k mod M = i and marches block
// b = t - d (k-1) at launch t; a one-thread kernel after each launch records
// finished iterations, stops at convergence and schedules the next launch.
struct PipeCtl {
  int t;         // index of the launch scheduled last
  int stop;      // 0 running; k > 0 last iteration (converged or kmax); -1 non-finite r^1
  int done;      // iterations completed
  int kmax;      // iterations allowed
  int M, d, L;   // slots, lag between iterations (launches), launches per window
  int restart_on_nonfinite;
  int last_busy; // last launch index with any slot scheduled
  int rb;        // 1: the units are red-black half-sweeps (iteration k = units 2k-1, 2k)
  double tol;
};

// Slots of the interface-node value planes written by the multi-step kernel:
// the lower subdomain j gives u_j(a_{j+1}), u_j(a_{j+1}+1), u_j(b_j); the
// upper one gives u_{j+1}(a_{j+1}), u_{j+1}(b_j), u_{j+1}(b_j - 1).  With
// finite elements the slots A1_LO / B1_HI hold u_j(a_{j+1}-1) /
// u_{j+1}(b_j+1): the nodes of the element on the sender's side.
enum VSlot : int { V_A_LO = 0, V_A1_LO = 1, V_B_LO = 2, V_A_HI = 3, V_B_HI = 4, V_B1_HI = 5 };

// Kernel launchers (swr_kernels.hip).  Return hipSuccess or the launch error.
// Step launch n: traces and residual of level n (1 <= n <= nt), then the step
// n -> n+1 (n < nt), for every item; par selects the trace window read.
hipError_t launch_step(const StepTables &t, int waves, int seg_max, int n, int par, int grid,
                       hipStream_t s);
bool step_config_supported(int waves, int seg_max);
// Multi-step launch: advances every item by min(S, nt - n0) steps from level
// n0, reading state parity `src` (u0 when n0 == 0) and writing 1 - src; the
// tiles carry a halo of H >= S columns on both sides.
// groups: lane groups per wavefront (each holds its own segment for a tile
// of 64/groups columns); 2 * H * groups < 64
// tiles: 0 the general march kernel (halo on both sides); 1 or 2 the
// finite-difference march kernel with `tiles` x-tiles per wavefront and the
// halo on the upwind sides of each subdomain only (SubDev::hsides; items
// made for it; groups = 1, S <= 16)
hipError_t launch_march(const StepTables &t, int waves, int groups, int seg_max, int tiles,
                        int n0, int S, int H, int src, int par, int grid, hipStream_t s);
bool march_config_supported(int waves, int groups, int seg_max);
bool fd_config_supported(int waves, int seg_max, int tiles);
// Compute units of the current device (256 if it cannot be queried).
int device_cu_count();
// Exchange pass of the multi-step path: traces (6.9)/(6.11) of every level
// and the residual (6.12) from the interface-node value planes.
// S: steps per launch (pipelined tables: the exchange covers the levels of
// each instance's current block only).
// mode: 0 every trace and the residual; 1 / 2 the traces sent by even / odd
// subdomains (2 also the residual)
hipError_t launch_exchange(const StepTables &t, int par, int S, hipStream_t s, int mode = 0);
hipError_t launch_pipe_tick(PipeCtl *c, int *blk, int *iter, unsigned long long *res,
                            double *hist, hipStream_t s);
hipError_t launch_reset_res(const InstDev *inst, int n_inst, hipStream_t s);
// nudt: dt / h_x for the finite-element scheme (the last step's transport
// of every row, v_i = -1 + i hv), 0 for a plain copy.
hipError_t launch_assemble(const double *Ufinal, const int *rowmap, double *uT, int nv, int nx,
                           hipStream_t s, double nudt = 0.0, double hv = 0.0);
hipError_t launch_fill(double *p, size_t n, double v, hipStream_t s);
hipError_t launch_copy(const double *src, double *dst, size_t n, hipStream_t s);
hipError_t launch_count_nonfinite(const double *p, size_t n, unsigned int *count, hipStream_t s);
// ab: device [J-1][2] = (a_{j+1}, b_j) per interface.
hipError_t launch_u0_guess(const double *u0, int nx, int nt, int J, const int *ab, int tr,
                           double p, double q, double hv, double *lam, hipStream_t s);
hipError_t launch_bw_probe(const void *src, void *dst, size_t bytes, hipStream_t s);

}  // namespace kfp
