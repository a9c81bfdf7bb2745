/*
 * kfpswr.h -- C ABI of libkfpswr, a gfx950 (MI355X) library for Schwarz
 * waveform relaxation (SWR) applied to the Kolmogorov equation
 *
 *     u_t + v u_x - u_vv = f   on (0,T) x [0,1)_periodic x [-1,1],
 *
 * (Section 6.1, eq. (6.1)), with u = 0 at v = -1 and v = +1.
 *
 * Discrete problem (Section 6.2, read as one IMEX Euler step per dt):
 *   h_x = 1/nx, x_m = m h_x (m = 0..nx-1); h_v = 2/nv, v_i = -1 + i h_v
 *   (i = 0..nv); dt = T/nt.  One step maps U^n to U^{n+1}:
 *     rhs = (1-|nu_i|) U_{i,m} + |nu_i| U_{i,m-sgn(v_i)} + dt s_{n+1} f_{i,m}
 *           (upwind transport, eqs. (6.4)/(6.5), nu_i = v_i dt/h_x),
 *     -r U_{i-1} + (1+2r) U_i - r U_{i+1} = rhs_i,  r = dt/h_v^2
 *           (implicit diffusion in v, eq. (6.2)).
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer unless marked [host].
 *   - Fields are FP64, row-major [nv+1][nx] (v-node i is the row, x is
 *     contiguous).  Rows 0 and nv of an output are zero.
 *   - Interface traces ("lambda", eq. (6.7)) are FP64 [2(J-1)][nt][nx]:
 *     plane 2j is the data subdomain j+1 receives at its lower node a_{j+1}
 *     (Q_2 u_j, eq. (6.9)); plane 2j+1 is the data subdomain j receives at
 *     its upper node b_j (Q_1 u_{j+1}, eq. (6.11)); row n-1 is time level n.
 *   - Partition (eq. (6.6) generalised to J pieces): core cuts c_j = j nv/J;
 *     a_0 = 0, b_{J-1} = nv; b_j = c_{j+1} + ceil(o/2), a_{j+1} = c_{j+1} -
 *     floor(o/2), so neighbours share o cells.
 *   - Transmission (Section 6.3): KFP_DIRICHLET is Q = I (classical SWR);
 *     KFP_ROBIN is Q_1 = p + d/dv at b_j and Q_2 = p - d/dv at a_{j+1}
 *     (one-sided optimized SWR, q = p, Section 6.4.1); the derivative is a
 *     one-sided first-order difference inside the receiving subdomain.
 *   - Iterations are the parallel (Jacobi) form of the Remark after (6.12):
 *     iteration k reads only the traces of iteration k-1.
 *   - The stopping test is (6.12): the largest |u_j - u_{j+1}| over the
 *     overlap and the whole space-time window, absolute, in FP64.
 *   - stream is a hipStream_t (NULL = the null stream).  The library owns its
 *     workspace (state ping-pong, trace windows, tables); the caller owns all
 *     argument buffers.  Calls on one process are serialised internally.
 *   - Errors: every call returns a kfp_status; on failure kfp_last_error()
 *     describes it.  KFP_EINVAL is returned before any device work.
 */
#ifndef KFPSWR_H
#define KFPSWR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KFP_OK = 0,
  KFP_EINVAL = 1,  /* invalid argument: nothing was written                  */
  KFP_ENOMEM = 2,  /* device or host allocation failed                       */
  KFP_EDEVICE = 3, /* a HIP call failed; message in kfp_last_error()         */
  KFP_ENOCONV = 4  /* max_iter reached: outputs hold the last iterate        */
} kfp_status;

typedef enum { KFP_DIRICHLET = 0, KFP_ROBIN = 1 } kfp_transmission;
/* Discretisation of the v-diffusion (kfp_set_scheme). */
typedef enum { KFP_SCHEME_FD = 0, KFP_SCHEME_FEM = 1 } kfp_scheme;

/* The space-time grid of Section 6.2.  x in [0,1) periodic with nx cells,
 * v in [-1,1] with nv cells (nv+1 nodes), nt steps of dt = T/nt. */
typedef struct {
  int32_t nx, nv, nt;
  double T;
} kfp_grid;

/* Per-solve statistics ([host]). */
typedef struct {
  int32_t iters;        /* SWR iterations performed (k at the stop)          */
  int32_t restarted;    /* 1 if a non-finite initial guess was replaced by 0 */
  double residual;      /* r^k of the last iteration (eq. (6.12))            */
  double seconds;       /* wall time of the call                             */
  double device_seconds;/* device time of the iteration graphs (HIP events)  */
  double step_seconds;  /* the part of it in the time-step kernels (batch:   */
                        /* the whole iteration)                              */
  double step_launches; /* launches of the time-step kernel (0: batch)      */
  double cell_steps;    /* subdomain cell-steps executed (all iterations)    */
  double alg_bytes;     /* algorithmic HBM bytes of those cell-steps         */
  double *res_history;  /* [host] optional, length max_iter: r^1..r^iters   */
} kfp_swr_stats;

/*
 * kfp_mono_solve -- the monodomain discrete solution at t = T (Section 6.2):
 * nt steps of transport + source + implicit diffusion on rows 1..nv-1.
 *   g:   grid (nx >= 2, nv >= 4, nt >= 1, T > 0, dt/h_x <= 1)
 *   u0:  [nv+1][nx] initial data (rows 0 and nv are treated as 0)
 *   f:   [nv+1][nx] source shape; the source at t_n is s[n] * f
 *   s:   [host] nt+1 time factors s(t_n), or NULL for s = 1
 *   uT:  [nv+1][nx] output U^nt
 * Asynchronous on `stream`.
 */
kfp_status kfp_mono_solve(const kfp_grid *g, const double *u0, const double *f,
                          const double *s, double *uT, void *stream);

/*
 * kfp_mono_solve_static -- kfp_mono_solve for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, same kernels and the same result
 * as kfp_mono_solve.  It calls no hipMalloc/hipFree and creates no stream or
 * event: the state ping-pong and the coefficient tables live in a static
 * device workspace of 64 MiB per GPU (held until the process ends), and all
 * work runs on `stream`.
 *   Limit: 2 (nv-1) nx doubles of state plus the tables must fit in 64 MiB
 *   (e.g. nv = 1024 with nx up to about 4000); larger grids return
 *   KFP_EINVAL with nothing written.
 *   The tables are copied in with `stream` synchronised once before the
 *   launches; the march itself is asynchronous on `stream`.
 *   Every call on one GPU shares that GPU's workspace: calls that overlap
 *   in time on one GPU (other streams, other host threads' streams) race.
 */
kfp_status kfp_mono_solve_static(const kfp_grid *g, const double *u0, const double *f,
                                 const double *s, double *uT, void *stream);

/*
 * kfp_swr_solve -- parallel SWR (Section 6.3, eqs. (6.8)-(6.12)) over J
 * subdomains split in v with an overlap of `overlap` cells.
 *   J:           1 <= J, nv % J == 0, nv/J >= overlap + 2
 *   overlap:     >= 1 when J > 1 (classical SWR cannot converge without it,
 *                Section 6.5; the Robin stencil needs one cell)
 *   tr, p:       transmission; Robin needs p > 0 (Section 2)
 *   tol:         > 0, absolute tolerance on r^k
 *   max_iter:    >= 1
 *   lambda_init: [2(J-1)][nt][nx] initial traces lambda^0, or NULL for 0.
 *                A guess holding NaN/Inf is replaced by 0 (stats.restarted).
 *   uT:          [nv+1][nx] output: the glued iterate at t = T (node i comes
 *                from the subdomain whose core [c_j, c_{j+1}) holds it)
 *   lambda_out:  same shape as lambda_init (the last traces), or NULL.
 *                Passing them back as lambda_init resumes the iteration.
 *   stats:       [host] or NULL
 * Returns KFP_OK when r^k < tol, KFP_ENOCONV after max_iter iterations.
 * Synchronises with the device once per iteration (8-byte residual read).
 */
kfp_status kfp_swr_solve(const kfp_grid *g, const double *u0, const double *f,
                         const double *s, int32_t J, int32_t overlap, int32_t tr, double p,
                         double tol, int32_t max_iter, const double *lambda_init, double *uT,
                         double *lambda_out, kfp_swr_stats *stats, void *stream);

/*
 * kfp_swr_solve_pq -- as kfp_swr_solve with the two-sided Robin operators of
 * Section 6.3: Q_1 = p + d/dv (data for a subdomain's upper interface node),
 * Q_2 = q - d/dv (for its lower one), OSWR(p,q) of Section 6.4.2.  Robin
 * needs q > 0 too; kfp_swr_solve is the case q = p.
 */
kfp_status kfp_swr_solve_pq(const kfp_grid *g, const double *u0, const double *f,
                            const double *s, int32_t J, int32_t overlap, int32_t tr, double p,
                            double q, double tol, int32_t max_iter, const double *lambda_init,
                            double *uT, double *lambda_out, kfp_swr_stats *stats,
                            void *stream);

/*
 * kfp_u0_guess -- the compatible initial traces lambda^0(n) = Q(u0) at each
 * interface node, for every time level n (Section 2: initial guesses must
 * agree with u0 at t = 0).  Same argument rules as kfp_swr_solve; writes
 * lambda [2(J-1)][nt][nx].  Asynchronous.
 */
kfp_status kfp_u0_guess(const kfp_grid *g, const double *u0, int32_t J, int32_t overlap,
                        int32_t tr, double p, double *lambda, void *stream);
/* The same with the two-sided operators (q as in kfp_swr_solve_pq). */
kfp_status kfp_u0_guess_pq(const kfp_grid *g, const double *u0, int32_t J, int32_t overlap,
                           int32_t tr, double p, double q, double *lambda, void *stream);

/* One instance of a batch ([host] struct, device pointers inside). */
typedef struct {
  kfp_grid g;
  int32_t J, overlap, tr;
  double p;
  const double *u0, *f;
  const double *s;           /* [host] nt+1 factors or NULL */
  const double *lambda_init; /* or NULL */
  double *uT;
  double *lambda_out;        /* or NULL */
  double q;                  /* second Robin parameter; <= 0 for q = p */
} kfp_instance;

/*
 * kfp_swr_batch -- n independent SWR instances of uneven nx, nv, J (same
 * rules per instance as kfp_swr_solve) advanced together: every time step of
 * every active instance runs in one persistent launch, one iteration is one
 * captured HIP graph, and an instance stops (its buffers freeze) as soon as
 * its own r^k < tol.  stats: [host] array of n, or NULL.
 * Returns KFP_OK if every instance converged, KFP_ENOCONV otherwise.
 */
kfp_status kfp_swr_batch(int32_t n, const kfp_instance *inst, double tol, int32_t max_iter,
                         kfp_swr_stats *stats, void *stream);

/*
 * Launch configuration.  waves = wavefronts per workgroup, each owning one
 * contiguous segment of a subdomain's unknown rows for 64 x-columns (the
 * segments are coupled through a small reduced tridiagonal system);
 * seg_max = largest segment the kernel holds in registers (0: segments of
 * any length staged through memory); steps = time steps per launch: 0 is
 * the general one-step kernel (any segment length, traces of the previous
 * level fused in), >= 1 the register march kernel, which keeps the state on
 * chip for `steps` steps with a halo of max(1, steps) columns on each side
 * of a tile.  kfp_tune times the candidates on the device for one shape
 * and stores the winner in the tuning cache (file named by $KFP_TUNE_CACHE,
 * default ~/.cache/kfpswr_tune.json); solves look the cache up, else use a
 * built-in choice.  kfp_set_config forces a
 * configuration for subsequent calls (waves = 0 returns to automatic
 * choice); KFP_EINVAL if it is not compiled.
 */
kfp_status kfp_tune(const kfp_grid *g, int32_t J, int32_t overlap, int32_t tr, double p,
                    int32_t *waves_out, int32_t *seg_max_out, int32_t *steps_out, void *stream);
kfp_status kfp_set_config(int32_t waves, int32_t seg_max, int32_t steps);

/*
 * kfp_tune_batch -- the launch classes of kfp_swr_batch, tuned.  A batch
 * groups its instances by the height of their tallest subdomain (each
 * height is one launch class with one configuration).  For every height
 * among the n instances, every compiled march configuration that holds it
 * is timed on the instances of that height (`iters` SWR iterations of
 * kfp_swr_batch each, device time); the fastest is stored in the tuning
 * cache under the batch key of that height (and the current
 * discretisation), where later kfp_swr_batch calls look it up.  The
 * instances' outputs are overwritten by the timed runs.  groups_out [host]:
 * the number of heights tuned (may be NULL).  KFP_EINVAL for n < 1, a NULL
 * array, iters < 1 or an invalid instance (as kfp_swr_batch).
 * kfp_get_batch_launch -- the configuration kfp_swr_batch would run this
 * instance's launch class with (tuned, forced or built-in).
 */
kfp_status kfp_tune_batch(int32_t n, const kfp_instance *inst, int32_t iters,
                          int32_t *groups_out, void *stream);
kfp_status kfp_get_batch_launch(const kfp_instance *inst, int32_t *waves_out,
                                int32_t *groups_out, int32_t *seg_max_out, int32_t *steps_out,
                                int32_t *tiles_out);

/*
 * kfp_reload_tune_cache -- forgets the tuning choices held in memory; the
 * next solve re-reads the cache file ($KFP_TUNE_CACHE as it is then).  For a
 * caller that replaces or edits that file while the library is loaded.  A
 * tuned one-step choice (steps = 0) is passed over by red-black solves,
 * which need a march configuration, whenever one holds the shape.
 */
kfp_status kfp_reload_tune_cache(void);

/*
 * kfp_set_launch / kfp_get_launch -- the same with lane groups: a march
 * configuration (steps >= 1) may split each wavefront into `groups` (1, 2
 * or 4) lane groups, each holding its own segment for a tile of 64/groups
 * x-columns, so that a workgroup holds waves * groups segments: subdomains
 * taller than 8 wavefronts of register segments then still march on chip.
 * The halo must leave columns valid: 2 * steps * groups < 64.  The
 * general kernel (steps = 0) takes groups = 1.  kfp_set_config(w, s, k) is
 * kfp_set_launch(w, 1, s, k); kfp_get_config reports waves, seg_max and
 * steps of the configuration kfp_get_launch reports in full (a tuned or
 * built-in choice may use lane groups).  KFP_EINVAL if not compiled.
 */
kfp_status kfp_set_launch(int32_t waves, int32_t groups, int32_t seg_max, int32_t steps);
kfp_status kfp_get_launch(const kfp_grid *g, int32_t J, int32_t overlap, int32_t tr,
                          int32_t *waves_out, int32_t *groups_out, int32_t *seg_max_out,
                          int32_t *steps_out);

/*
 * kfp_set_launch_tiles / kfp_get_launch_tiles -- the same with the march
 * kernel variant: tiles = 0 is the general march kernel above; tiles = 1 or
 * 2 (finite differences, groups = 1, 1 <= steps <= 16) the multi-tile march
 * kernel, whose wavefronts each hold their segment for `tiles` x-tiles of 64
 * columns (shared coefficient reads and barrier, independent elimination
 * chains) and whose tiles carry the halo of `steps` columns only on the
 * upwind sides of each subdomain's rows (one side when all its rows have
 * v >= 0 or all v <= 0).  Same arithmetic and results as the general march
 * kernel.  A forced multi-tile configuration falls back to the general
 * kernel of the same shape for the finite-element scheme or a subdomain
 * taller than waves * seg_max.  KFP_EINVAL if not compiled.
 */
kfp_status kfp_set_launch_tiles(int32_t waves, int32_t groups, int32_t seg_max, int32_t steps,
                                int32_t tiles);
kfp_status kfp_get_launch_tiles(const kfp_grid *g, int32_t J, int32_t overlap, int32_t tr,
                                int32_t *waves_out, int32_t *groups_out, int32_t *seg_max_out,
                                int32_t *steps_out, int32_t *tiles_out);

/*
 * kfp_set_pipeline -- overlap SWR iterations in time.  Iteration k at a
 * time block needs only iteration k-1's traces of that block (the method is
 * causal in time), so iteration k+1 can march d blocks behind iteration k;
 * kfp_swr_solve then keeps `inflight` iterations in flight on its own state
 * and trace window, stops at the first iteration below the tolerance and
 * returns exactly the iterate, traces, count and history of the
 * non-overlapped iteration.  inflight: -1 automatic (when one iteration's
 * launches hold fewer than 512 work items; the default), 0 off, >= 2 forced.
 * Applies to multi-step configurations with J >= 2; KFP_EINVAL otherwise.
 */
kfp_status kfp_set_pipeline(int32_t inflight);

/*
 * kfp_set_ordering -- order of the subdomain solves within one SWR
 * iteration of kfp_swr_solve / kfp_swr_solve_pq (Section 6.3).
 * 0 (default): parallel, the form of the Remark after (6.12): every
 *   subdomain of iteration k reads the traces of iteration k-1.
 * 1: multiplicative in red-black order, the form (6.8)-(6.11) is written in
 *   for two subdomains: the even subdomains march the window with the
 *   current traces and send theirs, then the odd subdomains march with
 *   those new traces and send theirs.  The residual (6.12) is that of the
 *   iterates of the same iteration.  For two subdomains one such iteration
 *   contracts like two parallel ones at the cost of one; the two halves run
 *   one after the other, each with half the work items.  Needs a march
 *   configuration (subdomains of at most 1056 rows; KFP_EINVAL otherwise);
 *   overlapped iterations (kfp_set_pipeline) are not used in this order.
 * Also applies to kfp_swr_batch (each launch class runs its two half-sweeps
 * in turn, the classes side by side) and kfp_swr_solve_windows.
 */
kfp_status kfp_set_ordering(int32_t order);

/*
 * kfp_set_scheme -- discretisation used by every later solve
 * (kfp_mono_solve, kfp_swr_solve / _pq, kfp_swr_batch,
 * kfp_swr_solve_windows; not kfp_u0_guess, whose traces are a guess for
 * either scheme: one-sided differences of the start state).
 * KFP_SCHEME_FD (default): finite differences in v, one IMEX step
 *   (transport, source, implicit diffusion), zero values at v = +-1.
 * KFP_SCHEME_FEM: the discretisation of Section 6.2 as printed: linear
 *   finite elements in v with the consistent mass matrix and the stiffness
 *   matrix of (6.3), homogeneous Neumann conditions at v = +-1 (6.1), and a
 *   time step that first solves the diffusion stage
 *   (M/dt + S) W^{n+1} = M/dt (U^n + dt s(t_{n+1}) f) and then transports
 *   its result, U^{n+1} = T W^{n+1} ((6.4)/(6.5)), each stage over the whole
 *   step dt; U^0 = u0.  Robin transmission is a natural condition (with or
 *   without overlap); a trace sent across an overlap takes the derivative
 *   in Q from the flux of the sender's element next to the interface node;
 *   the iterates, traces and residual (6.12) are those of the diffusion
 *   stage, and uT is U^nt.  Runs on the march kernel only: subdomains of at
 *   most 1056 rows, KFP_EINVAL otherwise (at the solve).
 * Returns KFP_EINVAL for any other value.
 */
kfp_status kfp_set_scheme(int32_t scheme);

/*
 * kfp_swr_solve_windows -- SWR on time windows.  [0, T] is cut into
 * n_windows windows of whole time steps (window w takes the steps
 * floor(w nt / n_windows) .. floor((w+1) nt / n_windows) - 1, all with
 * dt = T / nt), and each window is solved by SWR (as kfp_swr_solve_pq, in
 * the order kfp_set_ordering selects) to the tolerance, starting from the
 * glued iterate at the end of the window before (window 0 from u0) and
 * taking the source levels s[n] of its own steps.  Only one window's trace
 * planes are held, 2(J-1) x (nt / n_windows) x nx per buffer, and
 * waveform relaxation converges in fewer iterations on shorter windows.
 * Converged windows compose to the monodomain solution over [0, T] (the
 * time step is Markov).
 *   guess: initial traces of each window: 0 zero, 1 the extension Q(start
 *     state) of kfp_u0_guess_pq.
 *   window_iters: [host] n_windows, or NULL: the iterations of each window.
 *   stats: iteration counts, cell-steps and times summed over the windows,
 *     residual = the largest final residual of a window; res_history, if
 *     given, has n_windows * max_iter entries: window w's history at
 *     w * max_iter.
 *   Arguments as kfp_swr_solve_pq (u0 and uT may be the same buffer);
 *   1 <= n_windows <= nt, else KFP_EINVAL.  The call allocates two
 *   intermediate fields and (guess = 1) one window of traces, and returns
 *   when the caller's stream has finished with them.  KFP_ENOCONV if a
 *   window did not converge (the remaining windows are still solved).
 */
kfp_status kfp_swr_solve_windows(const kfp_grid *g, const double *u0, const double *f,
                                 const double *s, int32_t J, int32_t overlap, int32_t tr,
                                 double p, double q, double tol, int32_t max_iter,
                                 int32_t n_windows, int32_t guess, double *uT,
                                 int32_t *window_iters, kfp_swr_stats *stats, void *stream);

/*
 * kfp_swr_solve_windows_init -- as kfp_swr_solve_windows, with each window's
 * initial traces taken from lambda_init ([2(J-1)][nt][nx] FP64, device, the
 * traces of the whole [0, T]): window w starts from its own levels of every
 * plane.  Converged windows compose to the monodomain solution, so traces
 * predicted for the whole interval (a learned guess) serve every window.
 * lambda_init NULL with J > 1: KFP_EINVAL.  The call allocates one window
 * of traces besides the two intermediate fields.
 */
kfp_status kfp_swr_solve_windows_init(const kfp_grid *g, const double *u0, const double *f,
                                      const double *s, int32_t J, int32_t overlap, int32_t tr,
                                      double p, double q, double tol, int32_t max_iter,
                                      int32_t n_windows, const double *lambda_init, double *uT,
                                      int32_t *window_iters, kfp_swr_stats *stats,
                                      void *stream);

/*
 * kfp_set_kernel_timing -- with on != 0, overlapped-iteration solves launch
 * their kernels directly (not from a replayed graph) with HIP events around
 * every time-step kernel launch, so that kfp_swr_stats.step_seconds holds
 * those kernels' time alone.  Off by default.
 */
kfp_status kfp_set_kernel_timing(int32_t on);
kfp_status kfp_get_config(const kfp_grid *g, int32_t J, int32_t overlap, int32_t tr,
                          int32_t *waves_out, int32_t *seg_max_out, int32_t *steps_out);

/* Unknown rows summed over the subdomains (the cell-steps of one SWR
 * iteration are nx * nt * rows).  [host] out. */
kfp_status kfp_subdomain_rows(const kfp_grid *g, int32_t J, int32_t overlap, int32_t tr,
                              int64_t *rows_out);

/*
 * kfp_bw_probe -- streaming copy of `bytes` bytes (multiple of 16) from src
 * to dst, used to measure the attainable HBM bandwidth.  Asynchronous.
 */
kfp_status kfp_bw_probe(const void *src, void *dst, int64_t bytes, void *stream);

/*
 * kfp_tile_probe -- V = U + F/2 over [rows][nx] FP64 arrays (row-major, row
 * stride nx; device pointers; V must not overlap U or F), read and written in
 * the tile shape of the register march at one time step per launch: a
 * workgroup of `waves` wavefronts per 64-column x tile, `rows_per_wave` rows
 * per wavefront, one column per lane.  Used to measure the streaming ceiling
 * of that access shape.  Supported (waves, rows_per_wave): (8, 17), (8, 9),
 * (4, 1); others, null pointers, rows < 0, nx < 1 or more than 65535 row
 * blocks give KFP_EINVAL before any device work.  Asynchronous on `stream`.
 */
kfp_status kfp_tile_probe(const double *U, const double *F, double *V, int64_t rows, int32_t nx,
                          int32_t waves, int32_t rows_per_wave, void *stream);

/* ======================================================================
 * Learned initial interface traces.
 *
 * A multilayer perceptron maps the 64 coefficients of the seeded fields
 * (u0, f) to the converged interface traces of one problem shape
 * (standardised per output).  Its prediction is passed to kfp_swr_solve as
 * lambda_init.  The SWR iteration still runs to the same tolerance, so it is
 * both the fallback and the measure of the network's error.
 *
 * Network: depth hidden layers Linear(hidden) -> GELU (erf form), then
 * Linear(out).  Weights W[out][in] with FP32 master copies and BF16 copies
 * used by the products (BF16 operands, FP32 accumulation); biases FP32.
 * Loss: mean squared error over the batch and the outputs.  Optimizer:
 * Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 * All X, Y, T buffers are device FP32, row-major [B][width].
 * ==================================================================== */
typedef struct kfp_mlp kfp_mlp;

/* in, hidden, out: positive multiples of 8; depth 0..16.  Weights drawn
 * N(0, 1/in) from a counter-based generator seeded by `seed`; biases 0.
 * The handle is owned by the caller (kfp_mlp_destroy). */
kfp_status kfp_mlp_create(int32_t in, int32_t hidden, int32_t depth, int64_t out, uint64_t seed,
                          kfp_mlp **mlp);
/* As kfp_mlp_create, with flags: KFP_MLP_SKIP makes the output layer read
 * the last hidden activations followed by the network input (a GELU trunk
 * plus a linear map of the input; its W is [out][hidden + in]).  Ignored
 * for depth 0.  Other bits: KFP_EINVAL. */
#define KFP_MLP_SKIP 1
kfp_status kfp_mlp_create_ex(int32_t in, int32_t hidden, int32_t depth, int64_t out,
                             int32_t flags, uint64_t seed, kfp_mlp **mlp);
void kfp_mlp_destroy(kfp_mlp *mlp);
/* Y[B][out] = net(X[B][in]).  Asynchronous. */
kfp_status kfp_mlp_forward(kfp_mlp *mlp, int32_t B, const float *X, float *Y, void *stream);
/* Gradients of the loss at (X, T) into the handle's gradient buffers
 * (allocated by the first call); loss: [host] or NULL (synchronises when
 * given).  B: multiple of 8. */
kfp_status kfp_mlp_backward(kfp_mlp *mlp, int32_t B, const float *X, const float *T,
                            double *loss, void *stream);
/* One Adam step with the stored gradients (learning rate lr); KFP_EINVAL
 * before the first kfp_mlp_backward. */
kfp_status kfp_mlp_adam(kfp_mlp *mlp, float lr, void *stream);
/* One training step: the same products and update arithmetic as
 * kfp_mlp_backward followed by kfp_mlp_adam (the same weights, bit for bit),
 * with the loss gradient formed in the output layer's epilogue and each
 * layer's Adam step applied in its weight-gradient product, so neither the
 * output nor the weight gradient is stored (the gradient buffers keep what
 * the last kfp_mlp_backward wrote). */
kfp_status kfp_mlp_train_step(kfp_mlp *mlp, int32_t B, const float *X, const float *T, float lr,
                              double *loss, void *stream);
/* Layers are 0..depth; [host] outputs. */
kfp_status kfp_mlp_layer_shape(const kfp_mlp *mlp, int32_t layer, int32_t *in, int64_t *out);
/* Copy a parameter to (set = 0) or from (set = 1) a device FP32 buffer:
 * which 0 = W [out][in], 1 = b [out], 2 = dW (read only; KFP_EINVAL before the
 * first kfp_mlp_backward), 3 = db (read only). */
kfp_status kfp_mlp_param(kfp_mlp *mlp, int32_t layer, int32_t which, int32_t set, float *buf,
                         void *stream);
/* Checkpoint: FP32 masters, Adam moments and step count. */
kfp_status kfp_mlp_save(const kfp_mlp *mlp, const char *path);
kfp_status kfp_mlp_load(const char *path, kfp_mlp **mlp);

/* Data helpers for building training sets from solver output.  All device
 * pointers, asynchronous.  kfp_cast_f64_f32: dst = (float)(src - base), base
 * NULL for none (a network can learn the correction to a cheaper guess);
 * kfp_column_stats: per-column mean and standard deviation (at least floor_)
 * of X[rows][cols]; kfp_standardize: X = (X - mean) / std in place;
 * kfp_destandardize: lam = base + mean + std * Y in FP64, base [rows][cols]
 * FP64 or NULL. */
kfp_status kfp_cast_f64_f32(const double *src, const double *base, float *dst, int64_t n,
                            void *stream);
/* y += alpha * x and y *= a (element-wise), n FP32 values: the residual
 * targets and composed scales of a network fitted in stages. */
kfp_status kfp_axpy_f32(const float *x, float *y, float alpha, int64_t n, void *stream);
kfp_status kfp_mul_f32(const float *a, float *y, int64_t n, void *stream);
kfp_status kfp_column_stats(const float *X, int32_t rows, int64_t cols, float floor_,
                            float *mean, float *stdv, void *stream);
kfp_status kfp_standardize(float *X, int32_t rows, int64_t cols, const float *mean,
                           const float *stdv, void *stream);
kfp_status kfp_destandardize(const float *Y, int32_t rows, int64_t cols, const float *mean,
                             const float *stdv, const double *base, double *lam, void *stream);

/* Traces as x-Fourier coefficients.  Every operator of the discretisation is
 * circulant in the periodic x direction (upwind transport (6.4)/(6.5) and a
 * v-solve that is the same for every column), so fields made of the
 * discrete modes cos/sin(2 pi m x_i), x_i = i/nx, give traces made of
 * exactly those modes at every level.  Device pointers, asynchronous;
 * modes: [host] nmodes (1..8) frequencies, each 1 <= m < nx/2.
 * kfp_trace_modes: for each row r of lam[rows][nx] (FP64),
 *   coef[r][2k]   = (2/nx) sum_i lam[r][i] cos(2 pi m_k i/nx),
 *   coef[r][2k+1] = (2/nx) sum_i lam[r][i] sin(2 pi m_k i/nx).
 * kfp_trace_synth: the inverse on another grid: lam[p][n][i] (FP64,
 *   [planes][nt][nx]) = sum_k a_k cos(2 pi m_k i/nx) + b_k sin(2 pi m_k i/nx),
 *   with (a_k, b_k) of level n (time (n+1)/nt of the window) interpolated
 *   linearly between the levels of coef[planes][ntc][2 nmodes] (level kc at
 *   time (kc+1)/ntc), held at the first and last level outside them.
 * Used to carry traces predicted on a coarse grid to a fine one. */
kfp_status kfp_trace_modes(const double *lam, int64_t rows, int32_t nx, int32_t nmodes,
                           const int32_t *modes, double *coef, void *stream);
kfp_status kfp_trace_synth(const double *coef, int32_t planes, int32_t ntc, int32_t nmodes,
                           const int32_t *modes, int32_t nt, int32_t nx, double *lam,
                           void *stream);

/* Frees all cached workspace (plans, graphs, trace windows). */
void kfp_release_workspace(void);

/* Message of the last failing call on this thread ("" if none). */
const char *kfp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KFPSWR_H */
