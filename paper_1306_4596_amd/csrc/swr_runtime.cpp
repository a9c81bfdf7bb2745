// Host runtime of libkfpswr: argument validation, the planner (partition,
// elimination tables, workspace), the SWR iteration driver with HIP-graph
// captured iterations, the batch scheduler and the launch-configuration
// tuner.  Exposes the C ABI declared in include/kfpswr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "../../include/kfpswr.h"
#include "../../include/kfpswr_debug.h"
#include "kfp_internal.h"
#include "probe_internal.h"

namespace kfp {

// ------------------------------------------------------------------ errors --
thread_local std::string g_err;  // shared with the network runtime

static kfp_status fail(kfp_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? KFP_ENOMEM : KFP_EDEVICE, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                      \
  } while (0)

static std::recursive_mutex g_mu;

// ---------------------------------------------------------------- geometry --
struct SubGeo {
  int a, b;    // node range [a_j, b_j]
  int lo, hi;  // unknown nodes
  int n;
  int lo_kind, hi_kind;
};

struct Geo {
  int nx, nv, nt, J, o, tr;
  int scheme = SCHEME_FD;
  double T;
  std::vector<SubGeo> sub;
  std::vector<int> row_off;
  std::vector<int> rowmap;  // [nv+1]: absolute row in U of the node's owner, -1 = zero
  int rows = 0;
  int n_max = 0;
};

static kfp_status validate_grid(const kfp_grid *g) {
  if (!g) return fail(KFP_EINVAL, "grid is NULL");
  if (g->nx < 2) return fail(KFP_EINVAL, "nx must be >= 2 (got %d)", g->nx);
  if (g->nv < 4) return fail(KFP_EINVAL, "nv must be >= 4 (got %d)", g->nv);
  if (g->nt < 1) return fail(KFP_EINVAL, "nt must be >= 1 (got %d)", g->nt);
  if (!(g->T > 0.0) || !std::isfinite(g->T)) return fail(KFP_EINVAL, "T must be > 0");
  const double hx = 1.0 / g->nx, dt = g->T / g->nt;
  // the largest |v| on a transported row is 1 - h_v; the bound is taken over
  // every node (|v| <= 1), i.e. dt <= h_x, so the upwind weights stay convex
  if (dt / hx > 1.0 + 1e-12)
    return fail(KFP_EINVAL, "CFL violated: dt/h_x = %g > 1", dt / hx);
  return KFP_OK;
}

// scheme: SCHEME_FEM makes v = -1 and v = +1 unknown rows (Neumann ends).
static kfp_status make_geo(const kfp_grid *g, int J, int o, int tr, double p, Geo &geo,
                           int scheme) {
  kfp_status st = validate_grid(g);
  if (st) return st;
  if (J < 1) return fail(KFP_EINVAL, "J must be >= 1 (got %d)", J);
  if (tr != KFP_DIRICHLET && tr != KFP_ROBIN) return fail(KFP_EINVAL, "unknown transmission %d", tr);
  if (g->nv % J) return fail(KFP_EINVAL, "nv %% J != 0 (nv=%d, J=%d)", g->nv, J);
  if (o < 0) return fail(KFP_EINVAL, "overlap must be >= 0");
  if (J > 1) {
    if (o < 1 && tr == KFP_DIRICHLET)
      return fail(KFP_EINVAL, "overlap must be >= 1 for classical SWR with J > 1 (it does not "
                              "converge without overlap)");
    if (g->nv / J < o + 2) return fail(KFP_EINVAL, "nv/J must be >= overlap + 2");
    if (tr == KFP_ROBIN && !(p > 0.0 && std::isfinite(p)))
      return fail(KFP_EINVAL, "Robin parameter p must be > 0 (got %g)", p);
    // The mismatch (6.12) is reduced at the two end nodes of each overlap.
    // That equals the maximum over the whole overlap by the discrete maximum
    // principle, which the finite-element step satisfies only while its
    // element matrix is an M-matrix (off-diagonal 1/6 - r <= 0).
    const double hv = 2.0 / g->nv, r = (g->T / g->nt) / (hv * hv);
    if (scheme == SCHEME_FEM && r < 1.0 / 6.0)
      return fail(KFP_EINVAL,
                  "the finite-element scheme needs r = dt/h_v^2 >= 1/6 with J > 1 (got r = %g): "
                  "below it the end-node mismatch can understate (6.12)", r);
  }
  geo.nx = g->nx;
  geo.nv = g->nv;
  geo.nt = g->nt;
  geo.T = g->T;
  geo.J = J;
  geo.o = o;
  geo.tr = tr;
  geo.scheme = scheme;
  const int w = g->nv / J;
  std::vector<int> a(J), b(J);
  a[0] = 0;
  b[J - 1] = g->nv;
  for (int j = 0; j + 1 < J; ++j) {
    const int c = (j + 1) * w;
    b[j] = c + (o + 1) / 2;
    a[j + 1] = c - o / 2;
  }
  geo.sub.resize(J);
  geo.row_off.resize(J);
  geo.rows = 0;
  geo.n_max = 0;
  for (int j = 0; j < J; ++j) {
    SubGeo &s = geo.sub[j];
    s.a = a[j];
    s.b = b[j];
    // optimized interfaces: Robin rows, or with no overlap the shared node's
    // half-cell rows; both are unknown rows of the subdomain
    const int ifk = tr == KFP_ROBIN ? (o == 0 ? END_RFV : END_ROBIN) : END_DIRI;
    s.lo_kind = j == 0 ? END_PHYS : ifk;
    s.hi_kind = j == J - 1 ? END_PHYS : ifk;
    const bool fem = scheme == SCHEME_FEM;
    s.lo = s.lo_kind == END_ROBIN || s.lo_kind == END_RFV || (fem && s.lo_kind == END_PHYS)
               ? s.a : s.a + 1;
    s.hi = s.hi_kind == END_ROBIN || s.hi_kind == END_RFV || (fem && s.hi_kind == END_PHYS)
               ? s.b : s.b - 1;
    s.n = s.hi - s.lo + 1;
    geo.row_off[j] = geo.rows;
    geo.rows += s.n;
    geo.n_max = std::max(geo.n_max, s.n);
  }
  geo.rowmap.assign(g->nv + 1, -1);
  const int i_end = scheme == SCHEME_FEM ? g->nv : g->nv - 1;
  for (int i = scheme == SCHEME_FEM ? 0 : 1; i <= i_end; ++i) {
    int j = std::min(J - 1, i / w);
    if (j > 0 && i == geo.sub[j].a && tr == KFP_DIRICHLET) j -= 1;
    const SubGeo &s = geo.sub[j];
    geo.rowmap[i] = geo.row_off[j] + (i - s.lo);
  }
  return KFP_OK;
}

// Upwind sides of subdomain j's rows (SubDev::hsides): bit 0 a row with
// v > 0, bit 1 a row with v < 0 (v_i = -1 + i h_v as in the tables).
static int sub_hsides(const Geo &g, int j) {
  const SubGeo &s = g.sub[j];
  const double hv = 2.0 / g.nv;
  return (-1.0 + (s.lo + s.n - 1) * hv > 0.0 ? 1 : 0) | (-1.0 + s.lo * hv < 0.0 ? 2 : 0);
}

// ---------------------------------------------------------- launch config --
// steps == 0: the general one-step kernel (any segment length, traces fused
// one level behind); steps >= 1: the register march kernel, `steps` time
// steps per launch with a halo of max(1, steps) columns per side.
struct Config {
  int waves = 0;
  int seg = 0;
  int steps = 0;
  int groups = 1;  // march kernel: lane groups per wavefront (segments of 64/groups columns)
  int tiles = 0;   // 1, 2: the finite-difference march kernel, x-tiles per wavefront
};

static bool config_supported(const Config &c) {
  if (c.tiles != 0)
    return c.tiles > 0 && c.groups == 1 && c.steps >= 1 && c.steps <= 16 &&
           fd_config_supported(c.waves, c.seg, c.tiles);
  if (c.steps == 0) return c.groups == 1 && step_config_supported(c.waves, c.seg);
  return c.steps >= 1 && c.steps <= 24 && 2 * c.steps * c.groups < 64 &&
         march_config_supported(c.waves, c.groups, c.seg);
}

static int halo_of(const Config &c) { return c.steps > 1 ? c.steps : 1; }

static const int kWaves[] = {1, 2, 4, 8, 16};
static const int kSegs[] = {8, 16, 24, 32, 48, 64};

// Does a multi-step configuration hold every subdomain (P = ceil(n/SEG) <=
// segments per workgroup, waves * groups)?
static bool march_fits(int n_max, int waves, int seg, int groups = 1) {
  return seg >= 2 && (n_max + seg - 1) / seg <= waves * groups;
}

// Smallest compiled multi-step segment length for `waves` wavefronts of
// `groups` lane groups, 0 if none.
static int march_seg_for(int n_max, int waves, int groups = 1) {
  for (int sm = 2; sm <= 64; ++sm)
    if (march_fits(n_max, waves, sm, groups) && march_config_supported(waves, groups, sm))
      return sm;
  return 0;
}

static int segs_for(int n, int waves) {
  const int P = std::max(1, std::min(waves, n / 2));
  return (n + P - 1) / P;
}

// Smallest compiled seg_max holding every subdomain with `waves` segments;
// 0 selects the global-staged variant.
static int seg_for(int n_max, int waves) {
  const int need = segs_for(n_max, waves);
  for (int s : kSegs)
    if (s >= need && step_config_supported(waves, s)) return s;
  return 0;
}

static Config default_config(int n_max) {
  Config c;
  for (int w : kWaves) {
    if (segs_for(n_max, w) <= 24 || w == 16) {
      c.waves = w;
      break;
    }
  }
  c.seg = seg_for(n_max, c.waves);
  return c;
}

// Default multi-step configuration: the fewest wavefronts (at most 8, where
// the registers hold a segment without spilling) whose register segment
// holds the subdomain, and 16 steps per launch (a 32-column tile) unless the
// 48-column tiles of 8 steps already give every compute unit two
// workgroups: then the smaller halo wins.  `items8`: work items of the whole
// launch set at 8 steps per launch (0: unknown).
static Config default_march(int n_max, long items8 = 0) {
  for (int w : kWaves) {
    if (w > 8) break;
    const int sm = march_seg_for(n_max, w);
    if (sm && (sm <= 24 || w == 8)) return Config{w, sm, items8 >= 2L * 256 ? 8 : 16};
  }
  // taller subdomains: eight wavefronts of two (then four) lane groups; the
  // steps per launch are the measured best trade between the halo share of
  // the narrower tile and the launches per window (6 of 32 columns, 4 of 16)
  for (int g : {2, 4}) {
    const int sm = march_seg_for(n_max, 8, g);
    if (sm) return Config{8, sm, g == 2 ? 6 : 4, g};
  }
  return Config{};
}

// Built-in choice of the multi-tile finite-difference march: the smallest
// compiled segment that holds the subdomain on 8 wavefronts (4 for
// subdomains of at most 48 rows); one tile per wavefront at 12 steps per
// launch when a launch holds two or more work items per compute unit (the
// 128-register build: two workgroups per compute unit), 15 steps when it
// holds eight or more (fewer launches for a slightly wider halo: at 4096 x
// 4096, J = 32, 161.0 ms per iteration against 165.9 at 12 steps, 162.7 at
// 14 and 164.7 at 16, interleaved repeats), otherwise two tiles at 16 steps
// (half the work items, each with twice the columns per lane).
// items1: work items of a launch with one tile at 12 steps (0: unknown, many).
static Config default_fd(int n_max, long items1) {
  const int waves = n_max <= 48 ? 4 : 8;
  for (int sm = 2; sm <= 33; ++sm) {
    if (!march_fits(n_max, waves, sm)) continue;
    const bool t1 = fd_config_supported(waves, sm, 1), t2 = fd_config_supported(waves, sm, 2);
    if (!t1 && !t2) continue;
    const bool many = items1 == 0 || items1 >= 2L * device_cu_count();
    if (t1 && (!t2 || (many && waves == 8 && (sm == 12 || sm == 17)))) {
      const bool very_many = items1 >= 8L * device_cu_count();
      return Config{waves, sm, very_many && waves == 8 && sm == 17 ? 15 : 12, 1, 1};
    }
    return Config{waves, sm, 16, 1, 2};
  }
  return Config{};
}

// 1 when the source factor g_n = dt s(t_{n+1}) is the same at every level.
static int g_is_const(const std::vector<double> &gv) {
  for (double x : gv)
    if (x != gv[0]) return 0;
  return 1;
}

static Config g_forced;  // waves == 0: automatic
static int g_pipe = -1;  // pipelined iterations: -1 automatic, 0 off, F >= 2 in flight
// Automatic overlap below this many work items per launch (half the compute
// units: one 8-wave workgroup per CU runs at a time), aiming at this many
// items per overlapped launch (several rounds, so the last round's tail is
// a small share).
static const long kPipeItems = 128;
static const long kPipeTarget = 1024;
static bool g_ktime = false;  // time every step-kernel launch with HIP events
// order of the subdomain solves within an iteration: 0 parallel (Jacobi),
// 1 multiplicative red-black (even subdomains, then odd ones with the traces
// the even ones just sent)
static int g_order = 0;
// discretisation of every solve (SCHEME_FD or SCHEME_FEM), set by kfp_set_scheme
static int g_scheme = SCHEME_FD;

// The output's last transport stage (finite elements): dt / h_x, else 0.
static double out_nudt(const Geo &g) {
  return g.scheme == SCHEME_FEM ? (g.T / g.nt) * g.nx : 0.0;
}

// The finite-element scheme runs on the march kernel only.
static kfp_status fem_needs_march(const Geo &g, const Config &c) {
  if (g.scheme == SCHEME_FEM && c.steps == 0)
    return fail(KFP_EINVAL,
                "the finite-element scheme needs a march configuration (subdomains of at most "
                "1056 rows; tallest here %d)", g.n_max);
  return KFP_OK;
}

// Tuning cache: a flat JSON object {"key": [waves, seg, steps, groups], ...}
// (groups may be absent: 1).
static std::string tune_path() {
  const char *e = getenv("KFP_TUNE_CACHE");
  if (e && *e) return e;
  const char *h = getenv("HOME");
  return std::string(h ? h : ".") + "/.cache/kfpswr_tune.json";
}

static std::map<std::string, Config> load_tune() {
  std::map<std::string, Config> out;
  FILE *fp = fopen(tune_path().c_str(), "r");
  if (!fp) return out;
  std::string s;
  char buf[4096];
  size_t k;
  while ((k = fread(buf, 1, sizeof buf, fp)) > 0) s.append(buf, k);
  fclose(fp);
  size_t pos = 0;
  while ((pos = s.find('"', pos)) != std::string::npos) {
    size_t e = s.find('"', pos + 1);
    if (e == std::string::npos) break;
    std::string key = s.substr(pos + 1, e - pos - 1);
    Config c;
    const int got = sscanf(s.c_str() + e + 1, " : [ %d , %d , %d , %d , %d ]", &c.waves,
                           &c.seg, &c.steps, &c.groups, &c.tiles);
    if (got == 3) c.groups = 1;
    if (got <= 4) c.tiles = 0;
    if (got >= 3 && config_supported(c)) out[key] = c;
    pos = e + 1;
  }
  return out;
}

// Creates every missing folder of `dir` (no child process: the caller's
// process holds a GPU context).
static void make_dirs(const std::string &dir) {
  for (size_t i = 1; i <= dir.size(); ++i)
    if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
}

static void save_tune(const std::map<std::string, Config> &m) {
  const std::string path = tune_path();
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0) make_dirs(path.substr(0, slash));
  std::string tmp = path + ".tmp";
  FILE *fp = fopen(tmp.c_str(), "w");
  if (!fp) return;
  fprintf(fp, "{\n");
  size_t i = 0;
  for (auto &kv : m)
    fprintf(fp, "  \"%s\": [%d, %d, %d, %d, %d]%s\n", kv.first.c_str(), kv.second.waves,
            kv.second.seg, kv.second.steps, kv.second.groups, kv.second.tiles,
            ++i < m.size() ? "," : "");
  fprintf(fp, "}\n");
  fclose(fp);
  rename(tmp.c_str(), path.c_str());
}

static std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::string a = prop.gcnArchName;
  size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

static std::string tune_key(const Geo &g) {
  char buf[160];
  snprintf(buf, sizeof buf, "%s/nx%d/nmax%d/J%d/tr%d%s", arch_name().c_str(), g.nx, g.n_max, g.J,
           g.tr, g.scheme == SCHEME_FEM ? "/fem" : "");
  return buf;
}

static std::map<std::string, Config> *g_tune = nullptr;

static long count_items(const Geo &g, const Config &c, int colour = -1);

// order: the solve order the configuration will run in (1: red-black, which
// needs a march configuration; a tuned one-step choice is then passed over).
static Config choose_config(const Geo &g, int order = 0) {
  if (g_forced.waves > 0) {
    Config c = g_forced;
    // the multi-tile kernel is finite differences with one segment per
    // wavefront: otherwise the general march kernel of the same shape
    if (c.tiles > 0 && (g.scheme == SCHEME_FEM || !march_fits(g.n_max, c.waves, c.seg))) c.tiles = 0;
    if (c.steps >= 1 && !march_fits(g.n_max, c.waves, c.seg, c.groups)) {
      const int sm = march_seg_for(g.n_max, c.waves, c.groups);
      if (sm) {
        c.seg = sm;  // widen to the next compiled segment length
      } else {
        c.steps = 0;  // no register segment holds it: the general step kernel
        c.groups = 1;
        c.seg = seg_for(g.n_max, c.waves);
      }
    }
    if (c.steps == 0 && c.seg > 0 && segs_for(g.n_max, c.waves) > c.seg)
      c.seg = seg_for(g.n_max, c.waves);
    return c;
  }
  if (!g_tune) g_tune = new std::map<std::string, Config>(load_tune());
  auto it = g_tune->find(tune_key(g));
  if (it != g_tune->end()) {
    const Config &c = it->second;
    const bool usable = c.tiles > 0 ? g.scheme != SCHEME_FEM && march_fits(g.n_max, c.waves, c.seg)
                        : c.steps >= 1 ? march_fits(g.n_max, c.waves, c.seg, c.groups)
                                     : (c.seg == 0 || segs_for(g.n_max, c.waves) <= c.seg) &&
                                           !(order == 1 && march_seg_for(g.n_max, 8, 4));
    if (usable) return c;
  }
  if (g.scheme == SCHEME_FD && g.J > 0 && g.nx > 0) {
    Config probe = default_fd(g.n_max, 0);
    if (probe.waves) {
      probe.tiles = 1;
      probe.steps = 12;
      const long items1 = fd_config_supported(probe.waves, probe.seg, 1)
                              ? count_items(g, probe, order == 1 ? 0 : -1)
                              : 0;
      const Config c = default_fd(g.n_max, items1 > 0 ? items1 : 1);
      if (c.waves) return c;
    }
  }
  if (g.J > 0 && g.nx > 0) {
    // overlapped iterations (see pipe_params) supply work items to spare:
    // then the smaller halo of 8 steps per launch
    const long items8 = (long)g.J * ((g.nx + 47) / 48);
    const bool piped = g_pipe != 0 && g.J > 1 && (g_pipe > 0 || items8 < kPipeItems);
    const Config c = default_march(g.n_max, piped ? (1L << 20) : items8);
    if (c.waves) return c;
  }
  return default_config(g.n_max);
}

// ------------------------------------------------------------------ tables --
struct HostTables {
  bool fem = false;  // the march tables are the finite-element layout
  std::vector<SubDev> subs;
  std::vector<RowCoef> rows;
  std::vector<MarchCoef> mrows;
  std::vector<FemCoef> frows;
  std::vector<FemSeg> fsegs;
  std::vector<double> rinv;
  std::vector<RedCoef> reds;
  std::vector<int> segs;
  std::vector<Item> items;
  std::vector<ExItem> ex;
};

// Row coefficients of subdomain s (local rows 0..n-1):  lo x_{k-1} + di x_k + up x_{k+1}.
static void row_matrix(const SubGeo &s, double r, double p, double q, double hv,
                       std::vector<double> &lo, std::vector<double> &di, std::vector<double> &up) {
  lo.assign(s.n, -r);
  di.assign(s.n, 1.0 + 2.0 * r);
  up.assign(s.n, -r);
  if (s.lo_kind == END_ROBIN) {  // (q - d/dv) u = lambda at the lower interface node
    lo[0] = 0.0;
    di[0] = q + 1.0 / hv;
    up[0] = -1.0 / hv;
  }
  if (s.hi_kind == END_ROBIN) {  // (p + d/dv) u = lambda at the upper interface node
    lo[s.n - 1] = -1.0 / hv;
    di[s.n - 1] = p + 1.0 / hv;
    up[s.n - 1] = 0.0;
  }
  // no overlap: the shared interface node balances its half cell, the flux
  // through the interface being lambda - q u (lower end) or lambda - p u
  // (upper end); times 2 dt / h_v:
  //   (1 + 2r + 2 dt q / h_v) u_0 - 2r u_1 = T u + dt s f + 2 dt/h_v lambda
  const double fv = 2.0 * r * hv;  // 2 dt / h_v
  if (s.lo_kind == END_RFV) {
    lo[0] = 0.0;
    di[0] = 1.0 + 2.0 * r + fv * q;
    up[0] = -2.0 * r;
  }
  if (s.hi_kind == END_RFV) {
    lo[s.n - 1] = -2.0 * r;
    di[s.n - 1] = 1.0 + 2.0 * r + fv * p;
    up[s.n - 1] = 0.0;
  }
}

// The finite-element rows of subdomain s (Section 6.2: linear elements,
// rows times dt / h_v), assembled element by element: each element
// [v_e, v_{e+1}] inside [a, b] adds (1/6)[[2,1],[1,2]] + r[[1,-1],[-1,1]] to
// the matrix and (1/6)[[2,1],[1,2]] to the mass weights ml, mm, mu of the
// right-hand side M/dt G.  A Robin condition is natural at its end node, with
// or without overlap: dt/h_v p (upper end) or dt/h_v q (lower end) on the
// diagonal.  A fixed (classical) node's coupling moves to the right-hand side
// with the trace (weight r - 1/6 of the row next to it) and its G enters
// through the mass weight of that row.
static void fem_row_matrix(const SubGeo &s, double r, double p, double q, double hv,
                           std::vector<double> &lo, std::vector<double> &di,
                           std::vector<double> &up, std::vector<double> &ml,
                           std::vector<double> &mm, std::vector<double> &mu) {
  lo.assign(s.n, 0.0);
  di.assign(s.n, 0.0);
  up.assign(s.n, 0.0);
  ml.assign(s.n, 0.0);
  mm.assign(s.n, 0.0);
  mu.assign(s.n, 0.0);
  for (int k = 0; k < s.n; ++k) {
    const int i = s.lo + k;  // node
    if (i > s.a) {           // the element below the node
      lo[k] += 1.0 / 6.0 - r;
      di[k] += 1.0 / 3.0 + r;
      ml[k] += 1.0 / 6.0;
      mm[k] += 1.0 / 3.0;
    }
    if (i < s.b) {  // the element above
      up[k] += 1.0 / 6.0 - r;
      di[k] += 1.0 / 3.0 + r;
      mu[k] += 1.0 / 6.0;
      mm[k] += 1.0 / 3.0;
    }
  }
  const double kr = r * hv;  // dt / h_v
  if (s.lo_kind == END_ROBIN || s.lo_kind == END_RFV) di[0] += kr * q;
  if (s.hi_kind == END_ROBIN || s.hi_kind == END_RFV) di[s.n - 1] += kr * p;
}

// The matrix of either scheme.
static void any_row_matrix(const SubGeo &s, int scheme, double r, double p, double q, double hv,
                           std::vector<double> &lo, std::vector<double> &di,
                           std::vector<double> &up) {
  if (scheme == SCHEME_FEM) {
    std::vector<double> ml, mm, mu;
    fem_row_matrix(s, r, p, q, hv, lo, di, up, ml, mm, mu);
  } else {
    row_matrix(s, r, p, q, hv, lo, di, up);
  }
}

// Appends the tables of one subdomain (partitioned into P segments).
static void add_subdomain(const Geo &g, int j, double p, double q, int waves, int inst, int sub_base,
                          HostTables &t) {
  const SubGeo &s = g.sub[j];
  const double hx = 1.0 / g.nx, hv = 2.0 / g.nv, dt = g.T / g.nt, r = dt / (hv * hv);
  const int n = s.n;
  const int P = std::max(1, std::min(waves, n / 2));
  std::vector<double> lo, di, up;
  row_matrix(s, r, p, q, hv, lo, di, up);

  SubDev d{};
  d.inst = inst;
  d.n = n;
  d.row_off = g.row_off[j];
  d.g_lo = s.lo;
  d.tab = (int)t.rows.size();
  d.seg = (int)t.segs.size();
  d.red = (int)t.reds.size();
  d.P = P;
  d.lo_kind = s.lo_kind;
  d.hi_kind = s.hi_kind;
  {
    // v_i = -1 + i h_v >= 0 from the first node at or above v = 0
    const double hv = 2.0 / g.nv;
    int i = 0;
    while (i <= g.nv && -1.0 + i * hv < 0.0) ++i;
    d.vsplit = i - s.lo;
    d.hsides = sub_hsides(g, j);
  }
  d.lam_lo = j > 0 ? 2 * (j - 1) : -1;
  d.lam_hi = j < g.J - 1 ? 2 * j + 1 : -1;
  d.out_hi_plane = j < g.J - 1 ? 2 * j : -1;
  d.out_hi_row = j < g.J - 1 ? g.sub[j + 1].a - s.lo : -1;
  d.out_lo_plane = j > 0 ? 2 * (j - 1) + 1 : -1;
  d.out_lo_row = j > 0 ? g.sub[j - 1].b - s.lo : -1;
  if (j < g.J - 1) {
    const SubGeo &nb = g.sub[j + 1];
    d.res_nb = sub_base + j + 1;
    d.res_row_a_nb = nb.lo_kind == END_ROBIN || nb.lo_kind == END_RFV ? nb.a - nb.lo : -1;
    d.res_row_b_self = s.hi_kind == END_ROBIN || s.hi_kind == END_RFV ? s.b - s.lo : -1;
    d.res_row_b_nb = s.b - nb.lo;
    d.res_plane_a = 2 * j;
    d.res_plane_b = 2 * j + 1;
  } else {
    d.res_nb = -1;
    d.res_row_a_nb = d.res_row_b_self = d.res_row_b_nb = -1;
    d.res_plane_a = d.res_plane_b = -1;
  }
  t.subs.push_back(d);

  // segments: P nearly equal pieces; every piece but the last ends with a
  // separator row
  std::vector<int> start(P + 1);
  start[0] = 0;
  for (int k = 0; k < P; ++k) start[k + 1] = start[k] + n / P + (k < n % P ? 1 : 0);
  for (int k = 0; k <= P; ++k) t.segs.push_back(start[k]);

  std::vector<RowCoef> rc(n);
  for (int k = 0; k < n; ++k) {
    const double v = -1.0 + (s.lo + k) * hv;
    rc[k].nu = v * dt / hx;
  }
  // local Thomas factors and spikes per block
  std::vector<std::vector<double>> gL(P), gR(P);
  for (int sgi = 0; sgi < P; ++sgi) {
    const int r0 = start[sgi];
    const int r1 = (sgi < P - 1) ? start[sgi + 1] - 2 : n - 1;  // last block row
    const int nb = r1 - r0 + 1;
    std::vector<double> cp(nb), piv(nb);
    for (int k = 0; k < nb; ++k) {
      const int i = r0 + k;
      piv[k] = (k == 0) ? di[i] : di[i] - lo[i] * cp[k - 1];
      cp[k] = (k < nb - 1) ? up[i] / piv[k] : 0.0;
      rc[i].fa = 1.0 / piv[k];
      rc[i].fb = (k == 0) ? 0.0 : -lo[i] / piv[k];
      rc[i].bc = (k < nb - 1) ? -cp[k] : 0.0;
    }
    auto solve = [&](std::vector<double> rhs) {
      std::vector<double> y(nb), x(nb);
      for (int k = 0; k < nb; ++k) {
        const int i = r0 + k;
        y[k] = (k == 0 ? rhs[k] : rhs[k] - lo[i] * y[k - 1]) / piv[k];
      }
      for (int k = nb - 1; k >= 0; --k) x[k] = (k == nb - 1) ? y[k] : y[k] - cp[k] * x[k + 1];
      return x;
    };
    std::vector<double> e(nb, 0.0);
    gL[sgi].assign(nb, 0.0);
    gR[sgi].assign(nb, 0.0);
    if (sgi > 0) {
      e.assign(nb, 0.0);
      e[0] = lo[r0];
      gL[sgi] = solve(e);
    }
    if (sgi < P - 1) {
      e.assign(nb, 0.0);
      e[nb - 1] = up[r1];
      gR[sgi] = solve(e);
    }
    for (int k = 0; k < nb; ++k) {
      rc[r0 + k].sl = gL[sgi][k];
      rc[r0 + k].sr = gR[sgi][k];
    }
    if (sgi < P - 1) {  // separator row: not part of the block elimination
      RowCoef &c = rc[r1 + 1];
      c.fa = c.fb = c.bc = c.sl = c.sr = 0.0;
    }
  }
  for (int k = 0; k < n; ++k) t.rows.push_back(rc[k]);

  // reduced tridiagonal system over the P-1 separators
  if (P > 1) {
    const int m = P - 1;
    std::vector<double> al(m), be(m), ga(m);
    for (int sgi = 0; sgi < m; ++sgi) {
      const int rho = start[sgi + 1] - 1;
      const double a_r = lo[rho], c_r = up[rho];
      const double gLs_end = gL[sgi].back(), gRs_end = gR[sgi].back();
      const double gL1_first = gL[sgi + 1].front(), gR1_first = gR[sgi + 1].front();
      al[sgi] = -a_r * gLs_end;
      be[sgi] = di[rho] - a_r * gRs_end - c_r * gL1_first;
      ga[sgi] = -c_r * gR1_first;
      RedCoef c{};
      c.ra = a_r;
      c.rc = c_r;
      t.reds.push_back(c);
    }
    double cprev = 0.0;
    for (int sgi = 0; sgi < m; ++sgi) {
      const double piv = (sgi == 0) ? be[0] : be[sgi] - al[sgi] * cprev;
      const double cpk = (sgi < m - 1) ? ga[sgi] / piv : 0.0;
      RedCoef &c = t.reds[d.red + sgi];
      c.g1 = 1.0 / piv;
      c.g2 = (sgi == 0) ? 0.0 : -al[sgi] / piv;
      c.h = -cpk;
      cprev = cpk;
    }
  }
}

// Thomas factors of the block [r0, r1] of a tridiagonal matrix and the two
// spikes (responses to the couplings lo[r0] below and up[r1] above).
struct BlockFactors {
  std::vector<double> piv, cp, gL, gR;
};

static BlockFactors factor_block(const std::vector<double> &lo, const std::vector<double> &di,
                                 const std::vector<double> &up, int r0, int r1, bool below,
                                 bool above) {
  BlockFactors b;
  const int nb = r1 - r0 + 1;
  b.piv.resize(nb);
  b.cp.resize(nb);
  for (int k = 0; k < nb; ++k) {
    const int i = r0 + k;
    b.piv[k] = (k == 0) ? di[i] : di[i] - lo[i] * b.cp[k - 1];
    b.cp[k] = (k < nb - 1) ? up[i] / b.piv[k] : 0.0;
  }
  auto solve = [&](std::vector<double> rhs) {
    std::vector<double> y(nb), x(nb);
    for (int k = 0; k < nb; ++k) y[k] = (k == 0 ? rhs[k] : rhs[k] - lo[r0 + k] * y[k - 1]) / b.piv[k];
    for (int k = nb - 1; k >= 0; --k) x[k] = (k == nb - 1) ? y[k] : y[k] - b.cp[k] * x[k + 1];
    return x;
  };
  b.gL.assign(nb, 0.0);
  b.gR.assign(nb, 0.0);
  if (below) {
    std::vector<double> e(nb, 0.0);
    e[0] = lo[r0];
    b.gL = solve(e);
  }
  if (above) {
    std::vector<double> e(nb, 0.0);
    e[nb - 1] = up[r1];
    b.gR = solve(e);
  }
  return b;
}

// Subdomain descriptor fields shared by both layouts.
static SubDev sub_descriptor(const Geo &g, int j, int inst, int sub_base) {
  const SubGeo &s = g.sub[j];
  SubDev d{};
  d.inst = inst;
  d.n = s.n;
  d.row_off = g.row_off[j];
  d.g_lo = s.lo;
  d.lo_kind = s.lo_kind;
  d.hi_kind = s.hi_kind;
  {
    // v_i = -1 + i h_v >= 0 from the first node at or above v = 0
    const double hv = 2.0 / g.nv;
    int i = 0;
    while (i <= g.nv && -1.0 + i * hv < 0.0) ++i;
    d.vsplit = i - s.lo;
    d.hsides = sub_hsides(g, j);
  }
  d.lam_lo = j > 0 ? 2 * (j - 1) : -1;
  d.lam_hi = j < g.J - 1 ? 2 * j + 1 : -1;
  d.out_hi_plane = j < g.J - 1 ? 2 * j : -1;
  d.out_hi_row = j < g.J - 1 ? g.sub[j + 1].a - s.lo : -1;
  d.out_lo_plane = j > 0 ? 2 * (j - 1) + 1 : -1;
  d.out_lo_row = j > 0 ? g.sub[j - 1].b - s.lo : -1;
  if (j < g.J - 1) {
    const SubGeo &nb = g.sub[j + 1];
    d.res_nb = sub_base + j + 1;
    d.res_row_a_nb = nb.lo_kind == END_ROBIN || nb.lo_kind == END_RFV ? nb.a - nb.lo : -1;
    d.res_row_b_self = s.hi_kind == END_ROBIN || s.hi_kind == END_RFV ? s.b - s.lo : -1;
    d.res_row_b_nb = s.b - nb.lo;
    d.res_plane_a = 2 * j;
    d.res_plane_b = 2 * j + 1;
  } else {
    d.res_nb = -1;
    d.res_row_a_nb = d.res_row_b_self = d.res_row_b_nb = -1;
    d.res_plane_a = d.res_plane_b = -1;
  }
  return d;
}

// Tables of one subdomain in the multi-step layout: P = ceil(n / SEG)
// segments of exactly SEG rows; a non-final segment ends with its separator;
// the final one starts with pad = P SEG - n identity rows.
// Inverse of the m x m tridiagonal matrix with sub-diagonal al[1..m-1],
// diagonal be and super-diagonal ga[0..m-2] (row-major into inv), column by
// column with the Thomas factorisation (the reduced matrix of a diagonally
// dominant system is diagonally dominant: no pivoting needed).
static void tridiag_inverse(const std::vector<double> &al, const std::vector<double> &be,
                            const std::vector<double> &ga, std::vector<double> &inv) {
  const int m = (int)be.size();
  inv.assign((size_t)m * m, 0.0);
  std::vector<double> cp(m), piv(m), z(m);
  for (int i = 0; i < m; ++i) {
    piv[i] = (i == 0) ? be[0] : be[i] - al[i] * cp[i - 1];
    cp[i] = (i < m - 1) ? ga[i] / piv[i] : 0.0;
  }
  for (int col = 0; col < m; ++col) {
    for (int i = 0; i < m; ++i) {
      const double rhs = (i == col) ? 1.0 : 0.0;
      z[i] = (i == 0) ? rhs / piv[0] : (rhs - al[i] * z[i - 1]) / piv[i];
    }
    for (int i = m - 1; i >= 0; --i) {
      const double x = (i == m - 1) ? z[i] : z[i] - cp[i] * inv[(size_t)(i + 1) * m + col];
      inv[(size_t)i * m + col] = x;
    }
  }
}

static void add_subdomain_march(const Geo &g, int j, double p, double q, int seg, int inst,
                                int sub_base,
                                HostTables &t) {
  const SubGeo &s = g.sub[j];
  const double hx = 1.0 / g.nx, hv = 2.0 / g.nv, dt = g.T / g.nt, r = dt / (hv * hv);
  const int n = s.n;
  const int P = (n + seg - 1) / seg;
  const int pad = P * seg - n;
  const bool fem = g.scheme == SCHEME_FEM;
  std::vector<double> lo, di, up, ml, mm, mu;
  if (fem)
    fem_row_matrix(s, r, p, q, hv, lo, di, up, ml, mm, mu);
  else
    row_matrix(s, r, p, q, hv, lo, di, up);
  t.fem = fem;
  SubDev d = sub_descriptor(g, j, inst, sub_base);
  d.tab = fem ? (int)t.frows.size() : (int)t.mrows.size();
  d.seg = fem ? (int)t.fsegs.size() : -1;
  d.red = (int)t.reds.size();
  d.rinv = (int)t.rinv.size();
  d.P = P;
  d.pad = pad;
  t.subs.push_back(d);
  std::vector<MarchCoef> mc((size_t)P * seg);
  for (auto &c : mc) c = MarchCoef{0, 0, 0, 0, 0, 0, 0, 0};
  // block w covers real rows [b0, b1]; separators at w*seg + seg - 1
  std::vector<BlockFactors> bf(P);
  std::vector<int> b0(P), b1(P);
  for (int w = 0; w < P; ++w) {
    b0[w] = w * seg;
    b1[w] = (w < P - 1) ? w * seg + seg - 2 : n - 1;
    bf[w] = factor_block(lo, di, up, b0[w], b1[w], w > 0, w < P - 1);
  }
  auto is_robin = [&](int i) {
    return (i == 0 && s.lo_kind == END_ROBIN) || (i == n - 1 && s.hi_kind == END_ROBIN);
  };
  auto takes_data = [&](int i) {
    return (i == 0 && s.lo_kind != END_PHYS) || (i == n - 1 && s.hi_kind != END_PHYS);
  };
  for (int w = 0; w < P; ++w) {
    const int k0 = (w == P - 1) ? pad : 0;
    // padding rows: no transport, no source, multiplier 1 (they pass the
    // elimination's starting value, the low boundary data, to row k0); the
    // back substitution copies row k0's value down into them (bc = 1: their
    // forward values are zero in a last segment that is not the first), so
    // that register 0 of every segment holds its first real row
    for (int k = 0; k < k0; ++k) mc[(size_t)w * seg + k].fb = mc[(size_t)w * seg + k].bc = 1.0;
    for (int k = k0; k < seg; ++k) {
      const int i = w * seg + k - k0;  // local row
      MarchCoef &c = mc[(size_t)w * seg + k];
      const double nu = (-1.0 + (s.lo + i) * hv) * dt / hx;
      const double wgt = std::fabs(nu);
      if (w < P - 1 && k == seg - 1) {  // separator: identity in the local solve
        c.alpha = 1.0 - wgt;
        c.beta = wgt;
        c.fa = 1.0;
        c.fb = c.bc = c.sl = c.sr = 0.0;
        c.fab = takes_data(i) ? 1.0 : 0.0;
        continue;
      }
      const int kb = i - b0[w];
      const double fa = 1.0 / bf[w].piv[kb];
      const bool rob = is_robin(i);
      c.alpha = rob ? 0.0 : fa * (1.0 - wgt);
      c.beta = rob ? 0.0 : fa * wgt;
      c.fa = rob ? 0.0 : fa;
      // the first row of a segment adds the incoming value once (it is the
      // low boundary data in the segment holding row 0, zero elsewhere)
      c.fb = (kb == 0) ? 1.0 : -lo[i] * fa;
      c.bc = (i < b1[w]) ? -bf[w].cp[kb] : 0.0;
      c.sl = bf[w].gL[kb];
      c.sr = bf[w].gR[kb];
      c.fab = takes_data(i) ? fa : 0.0;
    }
  }
  if (fem) {
    // the same partition in the finite-element layout
    auto nu_of = [&](int i) { return (-1.0 + (s.lo + i) * hv) * dt / hx; };
    for (int w = 0; w < P; ++w) {
      const int k0 = (w == P - 1) ? pad : 0;
      FemSeg sg{0.0, 0.0, 0.0, 0.0};
      for (int k = 0; k < seg; ++k) {
        FemCoef c{0, 0, 0, 0, 0, 0, 0, 0};
        if (k < k0) {  // padding: passes the starting value on
          c.fb = 1.0;
          t.frows.push_back(c);
          continue;
        }
        const int i = w * seg + k - k0;
        if (w < P - 1 && k == seg - 1) {  // separator: its unscaled right-hand side
          c.wl = ml[i];
          c.wm = mm[i];
          c.wu = 0.0;  // G of the next segment's first row: in the reduced system
          c.fab = takes_data(i) ? 1.0 : 0.0;
          t.frows.push_back(c);
          continue;
        }
        const int kb = i - b0[w];
        const double fa = 1.0 / bf[w].piv[kb];
        c.wl = k == k0 ? 0.0 : fa * ml[i];
        c.wm = fa * mm[i];
        c.wu = k == seg - 1 ? 0.0 : fa * mu[i];
        c.fb = (kb == 0) ? 1.0 : -lo[i] * fa;
        c.bc = (i < b1[w]) ? -bf[w].cp[kb] : 0.0;
        c.sl = bf[w].gL[kb];
        c.sr = bf[w].gR[kb];
        c.fab = takes_data(i) ? fa : 0.0;
        if (k == k0) {  // the node below the first real row
          sg.nul = nu_of(i - 1);
          sg.wol = fa * ml[i];
        }
        if (i == n - 1) {  // the node above the subdomain's last row
          sg.nua = nu_of(i + 1);
          sg.woa = fa * mu[i];
        }
        t.frows.push_back(c);
      }
      t.fsegs.push_back(sg);
    }
  } else {
    for (auto &c : mc) t.mrows.push_back(c);
  }
  if (P > 1) {
    const int m = P - 1;
    std::vector<double> al(m), be(m), ga(m);
    for (int sgi = 0; sgi < m; ++sgi) {
      const int rho = sgi * seg + seg - 1;
      const double a_r = lo[rho], c_r = up[rho];
      al[sgi] = -a_r * bf[sgi].gL.back();
      be[sgi] = di[rho] - a_r * bf[sgi].gR.back() - c_r * bf[sgi + 1].gL.front();
      ga[sgi] = -c_r * bf[sgi + 1].gR.front();
      RedCoef c{};
      c.ra = a_r;
      c.rc = c_r;
      c.rg = fem ? mu[rho] : 0.0;
      t.reds.push_back(c);
    }
    double cprev = 0.0;
    for (int sgi = 0; sgi < m; ++sgi) {
      const double piv = (sgi == 0) ? be[0] : be[sgi] - al[sgi] * cprev;
      const double cpk = (sgi < m - 1) ? ga[sgi] / piv : 0.0;
      RedCoef &c = t.reds[d.red + sgi];
      c.g1 = 1.0 / piv;
      c.g2 = (sgi == 0) ? 0.0 : -al[sgi] / piv;
      c.h = -cpk;
      cprev = cpk;
    }
    // the multi-step kernel applies the explicit inverse of the reduced
    // system (at most 31 x 31): every separator value is then an independent
    // dot product instead of a link in a serial chain
    std::vector<double> inv;
    tridiag_inverse(al, be, ga, inv);
    t.rinv.insert(t.rinv.end(), inv.begin(), inv.end());
  }
}

static void add_instance(const Geo &g, double p, double q, int waves, int inst, HostTables &t) {
  const int sub_base = (int)t.subs.size();
  for (int j = 0; j < g.J; ++j) add_subdomain(g, j, p, q, waves, inst, sub_base, t);
}

static void add_instance_cfg(const Geo &g, double p, double q, int waves, int seg, int steps,
                             int inst,
                             HostTables &t) {
  if (steps == 0) {
    add_instance(g, p, q, waves, inst, t);
    return;
  }
  const int sub_base = (int)t.subs.size();
  for (int j = 0; j < g.J; ++j) add_subdomain_march(g, j, p, q, seg, inst, sub_base, t);
}



// Output tile width of a configuration: 64 lanes (64/groups for the lane
// groups of the multi-step kernel), minus its halo on both sides.
static int tile_width(const Config &c) {
  return c.steps >= 1 ? 64 / c.groups - 2 * halo_of(c) : 64;
}

// x-columns one work item of subdomain j covers: the finite-difference
// kernel's tiles have the halo on the upwind sides only, `tiles` per item.
static int item_width(const Geo &g, int j, const Config &c) {
  if (c.tiles < 1) return tile_width(c);
  const int hs = sub_hsides(g, j), H = halo_of(c);
  return c.tiles * (64 - ((hs & 1) ? H : 0) - ((hs & 2) ? H : 0));
}

static void make_items(const Geo &g, int sub_base, const Config &c, std::vector<Item> &items) {
  // subdomain-fastest order: consecutive workgroups (and so the XCDs they are
  // dealt to round-robin) take different subdomains of the same x-range
  std::vector<int> width(g.J), tiles(g.J);
  int tmax = 0;
  for (int j = 0; j < g.J; ++j) {
    width[j] = item_width(g, j, c);
    tiles[j] = (g.nx + width[j] - 1) / width[j];
    tmax = std::max(tmax, tiles[j]);
  }
  for (int x = 0; x < tmax; ++x)
    for (int j = 0; j < g.J; ++j)
      if (x < tiles[j]) items.push_back(Item{sub_base + j, x * width[j]});
}

// Work items of one instance (colour 0 / 1: those of the even / odd
// subdomains only).
static long count_items(const Geo &g, const Config &c, int colour) {
  long n = 0;
  for (int j = 0; j < g.J; ++j)
    if (colour < 0 || (j & 1) == colour) n += (g.nx + item_width(g, j, c) - 1) / item_width(g, j, c);
  return n;
}

static void make_ex(const Geo &g, int inst, std::vector<ExItem> &ex) {
  for (int j = 0; j + 1 < g.J; ++j) ex.push_back(ExItem{inst, j, g.sub[j + 1].a, g.sub[j].b});
}

// ------------------------------------------------------------------ device --
template <class T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  hipError_t alloc(size_t count) {
    if (count <= n && p) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    hipError_t e = hipMalloc((void **)&p, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) n = count;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

// Device tables of one launch set (single instance or batch).
struct DevTables {
  DevBuf<InstDev> inst;
  DevBuf<SubDev> subs;
  DevBuf<Item> items;
  DevBuf<RowCoef> rows;
  DevBuf<RedCoef> reds;
  DevBuf<int> segs;
  DevBuf<ExItem> ex;
  DevBuf<MarchCoef> mrows;
  DevBuf<FemCoef> frows;
  DevBuf<FemSeg> fsegs;
  DevBuf<double> rinv;
  bool fem = false;
  StepTables view() const {
    StepTables t;
    t.inst = inst.p;
    t.subs = subs.p;
    t.items = items.p;
    t.rows = rows.p;
    t.reds = reds.p;
    t.segs = segs.p;
    t.ex = ex.p;
    t.mrows = mrows.p;
    t.frows = frows.p;
    t.fsegs = fsegs.p;
    t.rinv = rinv.p;
    t.blk = nullptr;
    t.n_items = (int)items.n;
    t.n_ex = (int)ex.n;
    t.fem = fem ? 1 : 0;
    return t;
  }
  hipError_t upload(const HostTables &h, const std::vector<InstDev> &in, hipStream_t s) {
    hipError_t e;
    if ((e = inst.alloc(in.size())) != hipSuccess) return e;
    if ((e = subs.alloc(h.subs.size())) != hipSuccess) return e;
    if ((e = items.alloc(h.items.size())) != hipSuccess) return e;
    if ((e = rows.alloc(h.rows.size())) != hipSuccess) return e;
    if ((e = reds.alloc(std::max<size_t>(h.reds.size(), 1))) != hipSuccess) return e;
    if ((e = segs.alloc(h.segs.size())) != hipSuccess) return e;
    if ((e = ex.alloc(std::max<size_t>(h.ex.size(), 1))) != hipSuccess) return e;
    if ((e = mrows.alloc(std::max<size_t>(h.mrows.size(), 1))) != hipSuccess) return e;
    if ((e = frows.alloc(std::max<size_t>(h.frows.size(), 1))) != hipSuccess) return e;
    if ((e = fsegs.alloc(std::max<size_t>(h.fsegs.size(), 1))) != hipSuccess) return e;
    fem = h.fem;
    if ((e = rinv.alloc(std::max<size_t>(h.rinv.size(), 1))) != hipSuccess) return e;
    items.n = h.items.size();
    ex.n = h.ex.size();
    auto cp = [&](void *d, const void *src, size_t bytes) {
      return bytes ? hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    if ((e = cp(inst.p, in.data(), in.size() * sizeof(InstDev))) != hipSuccess) return e;
    if ((e = cp(subs.p, h.subs.data(), h.subs.size() * sizeof(SubDev))) != hipSuccess) return e;
    if ((e = cp(items.p, h.items.data(), h.items.size() * sizeof(Item))) != hipSuccess) return e;
    if ((e = cp(rows.p, h.rows.data(), h.rows.size() * sizeof(RowCoef))) != hipSuccess) return e;
    if ((e = cp(reds.p, h.reds.data(), h.reds.size() * sizeof(RedCoef))) != hipSuccess) return e;
    if ((e = cp(segs.p, h.segs.data(), h.segs.size() * sizeof(int))) != hipSuccess) return e;
    if ((e = cp(ex.p, h.ex.data(), h.ex.size() * sizeof(ExItem))) != hipSuccess) return e;
    if ((e = cp(mrows.p, h.mrows.data(), h.mrows.size() * sizeof(MarchCoef))) != hipSuccess)
      return e;
    if ((e = cp(frows.p, h.frows.data(), h.frows.size() * sizeof(FemCoef))) != hipSuccess)
      return e;
    if ((e = cp(fsegs.p, h.fsegs.data(), h.fsegs.size() * sizeof(FemSeg))) != hipSuccess)
      return e;
    if ((e = cp(rinv.p, h.rinv.data(), h.rinv.size() * sizeof(double))) != hipSuccess) return e;
    return hipStreamSynchronize(s);  // host vectors may go out of scope
  }
  void release() {
    inst.release();
    subs.release();
    items.release();
    rows.release();
    reds.release();
    segs.release();
    ex.release();
    rinv.release();
    mrows.release();
    frows.release();
    fsegs.release();
  }
};

static bool use_graphs() {
  const char *e = getenv("KFP_NO_GRAPH");
  return !(e && *e && *e != '0');
}

// A cached single-instance workspace.  The graphs capture kernel launches
// whose arguments point at device tables only, so later calls with other
// data pointers, p, T or s refresh the tables and reuse the graphs.
struct Plan {
  Geo geo;
  Config cfg;
  DevTables dt;
  DevBuf<double> U0, U1, lam0, lam1, g, V;
  DevBuf<int> rowmap, ab;
  DevBuf<unsigned long long> res;
  DevBuf<unsigned int> cnt;
  unsigned long long *h_res = nullptr;  // pinned
  hipStream_t cs = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev0 = nullptr, ev1 = nullptr, evm = nullptr;
  // per parity: the time steps of an iteration, then its exchange (if any)
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipGraphExec_t gexch[2] = {nullptr, nullptr};
  bool captured = false;
  // red-black order: the work items of even subdomains come first; the odd
  // half-sweep runs on a second stream one time block behind the even one
  int order = 0, n_red = 0;
  hipStream_t cs2 = nullptr, cs3 = nullptr;  // odd half-sweep; per-block exchange
  hipEvent_t ev_fork = nullptr, ev_blk = nullptr, ev_join = nullptr, ev_mar = nullptr,
             ev_join3 = nullptr;
  DevBuf<int> blkseq;  // 0, 1, ..., L-1: the time block of each launch
  // [2][nv+1]: rowmap restricted to nodes owned by even / odd subdomains
  // (-2 elsewhere), for the output of pipelined red-black iterations
  DevBuf<int> rowmap_rb;
  // pipelined iterations (M > 0): M slot instances with their own state and
  // trace window; slot i writes window i and reads window i-1 (mod M)
  int M = 0, d = 0, L = 0, G = 0;
  DevBuf<double> slotU, W, hist;
  DevBuf<unsigned long long> pres;
  DevBuf<int> blk, iter;
  DevBuf<PipeCtl> ctl;
  PipeCtl *h_ctl = nullptr;  // pinned
  hipGraphExec_t gpipe = nullptr;
  const double *gpipe_hist = nullptr;  // history buffer the chunk graph was captured with
  std::vector<hipEvent_t> tev;  // around each march launch of the chunk graph
  ~Plan() {
    if (gpipe) (void)hipGraphExecDestroy(gpipe);
    for (auto e : tev)
      if (e) (void)hipEventDestroy(e);
    slotU.release();
    W.release();
    hist.release();
    pres.release();
    blk.release();
    iter.release();
    ctl.release();
    if (h_ctl) (void)hipHostFree(h_ctl);
    blkseq.release();
    rowmap_rb.release();
    if (cs2) (void)hipStreamDestroy(cs2);
    if (cs3) (void)hipStreamDestroy(cs3);
    for (hipEvent_t e : {ev_fork, ev_blk, ev_join, ev_mar, ev_join3})
      if (e) (void)hipEventDestroy(e);
    for (auto &ge : gexch)
      if (ge) (void)hipGraphExecDestroy(ge);
    for (auto &ge : gexec)
      if (ge) (void)hipGraphExecDestroy(ge);
    dt.release();
    U0.release();
    U1.release();
    lam0.release();
    lam1.release();
    g.release();
    V.release();
    rowmap.release();
    ab.release();
    res.release();
    cnt.release();
    if (h_res) (void)hipHostFree(h_res);
    if (cs) (void)hipStreamDestroy(cs);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (evm) (void)hipEventDestroy(evm);
  }
};

static std::map<std::string, std::unique_ptr<Plan>> g_plans;
static std::vector<std::string> g_plan_lru;
static const size_t kMaxPlans = 3;

struct PipeParams {
  int M = 0, d = 0;
};

// Pipelined iterations when one iteration's launches leave the GPU short of
// work: F iterations in flight (d = L / F launches apart) so that a launch
// holds about kPipeTarget work items; M = ceil(L/d) + 1 slots, each with a
// state and a trace window, within a memory budget.
// Red-black order (order 1): the units in flight are half-sweeps, each with
// the work items of one colour; they overlap below half the target, and the
// slot count is even, so that every slot serves one colour.
static PipeParams pipe_params(const Geo &g, const Config &c, int order = 0) {
  PipeParams pp;
  if (g_pipe == 0 || c.steps < 1 || g.J < 2) return pp;
  const int L = (g.nt + c.steps - 1) / c.steps;
  const long items = order == 1 ? count_items(g, c, 0) : count_items(g, c);
  if (g_pipe < 0 && items >= (order == 1 ? kPipeTarget / 2 : kPipeItems)) return pp;
  long F = g_pipe > 0 ? g_pipe : (kPipeTarget + items - 1) / items;
  F = std::min<long>(F, L);
  if (F < 2) return pp;
  int d = std::max(1, (int)(L / F));
  // trace window and state per slot (and, finite elements in the parallel
  // order, the interface-node value planes: see get_plan)
  const double v_planes = order == 0 && g.scheme == SCHEME_FEM ? 6.0 * (g.J - 1) * g.nt * g.nx : 0.0;
  const double per_slot =
      8.0 * ((double)2 * (g.J - 1) * g.nt * g.nx + 2.0 * g.rows * g.nx + v_planes);
  const double budget = 24e9;
  for (;;) {
    int M = (L + d - 1) / d + 1;
    if (order == 1) M += M & 1;
    if (M * per_slot <= budget || d >= L) {
      if (M >= 3) {
        pp.M = M;
        pp.d = d;
      }
      return pp;
    }
    d *= 2;
  }
}

static std::string plan_key(const Geo &g, const Config &c, int M, int order) {
  char buf[200];
  snprintf(buf, sizeof buf, "%d/%d/%d/%d/%d/%d/w%d/g%d/s%d/k%d/M%d/o%d/e%d", g.nx, g.nv, g.nt,
           g.J, g.o, g.tr, c.waves, c.groups, c.seg, c.steps, M, order, g.scheme);
  return buf;
}

static kfp_status get_plan(const Geo &geo, const Config &cfg, Plan **out,
                           PipeParams pp = PipeParams(), int order = 0) {
  const std::string key = plan_key(geo, cfg, pp.M, order);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    g_plan_lru.erase(std::find(g_plan_lru.begin(), g_plan_lru.end(), key));
    g_plan_lru.push_back(key);
    // the key leaves out T (buffers and partition do not depend on it); the
    // coefficient tables built from the plan's geometry must see this call's
    it->second->geo = geo;
    *out = it->second.get();
    return KFP_OK;
  }
  while (g_plans.size() >= kMaxPlans) {
    g_plans.erase(g_plan_lru.front());
    g_plan_lru.erase(g_plan_lru.begin());
  }
  std::unique_ptr<Plan> pl(new Plan());
  pl->geo = geo;
  pl->cfg = cfg;
  pl->order = order;
  if (order == 1) {
    const int L = (geo.nt + cfg.steps - 1) / cfg.steps;  // launches per window
    std::vector<int> seq(L);
    for (int l = 0; l < L; ++l) seq[l] = l;
    HIP_TRY(pl->blkseq.alloc(L));
    HIP_TRY(hipMemcpy(pl->blkseq.p, seq.data(), sizeof(int) * L, hipMemcpyHostToDevice));
    std::vector<int> rm(2 * (size_t)(geo.nv + 1), -2);
    for (int i = 0; i <= geo.nv; ++i) {
      const int r = geo.rowmap[i];
      if (r < 0) {
        rm[i] = rm[geo.nv + 1 + i] = r;
        continue;
      }
      int j = 0;
      while (j + 1 < geo.J && r >= geo.row_off[j + 1]) ++j;
      rm[(j & 1) * (geo.nv + 1) + i] = r;
    }
    HIP_TRY(pl->rowmap_rb.alloc(rm.size()));
    HIP_TRY(hipMemcpy(pl->rowmap_rb.p, rm.data(), sizeof(int) * rm.size(),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipStreamCreateWithFlags(&pl->cs2, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&pl->cs3, hipStreamNonBlocking));
    for (hipEvent_t *e : {&pl->ev_fork, &pl->ev_blk, &pl->ev_join, &pl->ev_mar, &pl->ev_join3})
      HIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
  }
  const size_t state = (size_t)geo.rows * geo.nx;
  const size_t win = (size_t)2 * (geo.J - 1) * geo.nt * geo.nx;
  HIP_TRY(pl->U0.alloc(state));
  HIP_TRY(pl->U1.alloc(state));
  HIP_TRY(pl->lam0.alloc(std::max<size_t>(win, 1)));
  HIP_TRY(pl->lam1.alloc(std::max<size_t>(win, 1)));
  HIP_TRY(pl->g.alloc(geo.nt));
  // interface-node value planes.  Overlapped iterations in the parallel
  // order with finite elements keep one set per slot: the exchange of a block
  // reads the level before it, which the next iteration, one launch behind,
  // rewrites in the same launch.  (Red-black half-sweeps share one set: the
  // two colours write different entries, the closing residual reads both,
  // and a colour's next half-sweep runs two units behind.)
  const bool v_per_slot = pp.M > 0 && order == 0 && geo.scheme == SCHEME_FEM;
  if (cfg.steps >= 1 && geo.J > 1)
    HIP_TRY(pl->V.alloc((size_t)6 * (geo.J - 1) * geo.nt * geo.nx * (v_per_slot ? pp.M : 1)));
  HIP_TRY(pl->rowmap.alloc(geo.nv + 1));
  HIP_TRY(pl->ab.alloc(std::max(2 * (geo.J - 1), 1)));
  HIP_TRY(pl->res.alloc(1));
  HIP_TRY(pl->cnt.alloc(1));
  HIP_TRY(hipHostMalloc((void **)&pl->h_res, sizeof(unsigned long long)));
  HIP_TRY(hipStreamCreateWithFlags(&pl->cs, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&pl->ev_in, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&pl->ev_out, hipEventDisableTiming));
  HIP_TRY(hipEventCreate(&pl->ev0));
  HIP_TRY(hipEventCreate(&pl->ev1));
  HIP_TRY(hipEventCreate(&pl->evm));
  HIP_TRY(hipMemcpy(pl->rowmap.p, geo.rowmap.data(), sizeof(int) * (geo.nv + 1),
                    hipMemcpyHostToDevice));
  std::vector<int> ab;
  for (int j = 0; j + 1 < geo.J; ++j) {
    ab.push_back(geo.sub[j + 1].a);
    ab.push_back(geo.sub[j].b);
  }
  if (!ab.empty())
    HIP_TRY(hipMemcpy(pl->ab.p, ab.data(), sizeof(int) * ab.size(), hipMemcpyHostToDevice));
  if (pp.M > 0) {
    pl->M = pp.M;
    pl->d = pp.d;
    pl->L = (geo.nt + cfg.steps - 1) / cfg.steps;
    pl->G = std::min(16, pl->L);
    HIP_TRY(pl->slotU.alloc((size_t)pp.M * 2 * state));
    HIP_TRY(pl->W.alloc((size_t)pp.M * win));
    HIP_TRY(pl->pres.alloc(pp.M));
    HIP_TRY(pl->blk.alloc(pp.M));
    HIP_TRY(pl->iter.alloc(pp.M));
    HIP_TRY(pl->ctl.alloc(1));
    HIP_TRY(hipHostMalloc((void **)&pl->h_ctl, sizeof(PipeCtl)));
    pl->tev.assign(2 * pl->G, nullptr);
    for (auto &e : pl->tev) HIP_TRY(hipEventCreate(&e));
  }
  *out = pl.get();
  g_plans[key] = std::move(pl);
  g_plan_lru.push_back(key);
  return KFP_OK;
}

// Uploads the per-call tables (data pointers, p, T, s) of a single instance.
static kfp_status load_instance(Plan &pl, const double *u0, const double *f, const double *s,
                                double p, double q) {
  const Geo &geo = pl.geo;
  HostTables h;
  const int n_inst = pl.M > 0 ? pl.M : 1;
  for (int i = 0; i < n_inst; ++i) {
    const int sub_base = (int)h.subs.size();
    add_instance_cfg(geo, p, q, pl.cfg.waves, pl.cfg.seg, pl.cfg.steps, i, h);
    if (pl.M > 0 && pl.order == 1) {
      // red-black half-sweep slots: odd slots march the even subdomains,
      // even slots the odd ones
      std::vector<Item> all;
      make_items(geo, sub_base, pl.cfg, all);
      const int colour = (i & 1) ? 0 : 1;
      for (const Item &it : all)
        if (((it.sub - sub_base) & 1) == colour) h.items.push_back(it);
    } else {
      make_items(geo, sub_base, pl.cfg, h.items);
    }
    make_ex(geo, i, h.ex);
  }
  pl.n_red = 0;
  if (pl.order == 1 && pl.M == 0) {  // even subdomains first (single instance: sub = j)
    std::stable_partition(h.items.begin(), h.items.end(),
                          [](const Item &it) { return (it.sub & 1) == 0; });
    for (const Item &it : h.items) pl.n_red += (it.sub & 1) == 0;
  }
  InstDev in{};
  in.U[0] = pl.U0.p;
  in.U[1] = pl.U1.p;
  in.u0 = u0;
  in.f = f;
  in.g = pl.g.p;
  in.lam[0] = pl.lam0.p;
  in.lam[1] = pl.order == 1 ? pl.lam0.p : pl.lam1.p;  // red-black: one window, in place
  in.res = pl.res.p;
  in.V = pl.V.p;
  const double hv = 2.0 / geo.nv, dt = geo.T / geo.nt;
  in.r = dt / (hv * hv);
  in.p = p;
  in.q = q;
  in.hv = hv;
  in.nx = geo.nx;
  in.nv = geo.nv;
  in.nt = geo.nt;
  in.tr = geo.tr;
  in.nonovl = geo.J > 1 && geo.o == 0 && geo.tr == KFP_ROBIN;
  in.scheme = geo.scheme;
  in.active = 1;
  std::vector<double> gv(geo.nt);
  for (int n = 0; n < geo.nt; ++n) gv[n] = dt * (s ? s[n + 1] : 1.0);
  in.gconst = g_is_const(gv);
  HIP_TRY(hipMemcpyAsync(pl.g.p, gv.data(), sizeof(double) * geo.nt, hipMemcpyHostToDevice, pl.cs));
  std::vector<InstDev> ins(n_inst, in);
  if (pl.M > 0) {
    const size_t state = (size_t)geo.rows * geo.nx;
    const size_t win = (size_t)2 * (geo.J - 1) * geo.nt * geo.nx;
    for (int i = 0; i < pl.M; ++i) {
      ins[i].U[0] = pl.slotU.p + (size_t)i * 2 * state;
      ins[i].U[1] = ins[i].U[0] + state;
      ins[i].lam[0] = pl.W.p + (size_t)((i + pl.M - 1) % pl.M) * win;  // read: iteration k-1
      ins[i].lam[1] = pl.W.p + (size_t)i * win;                        // written: iteration k
      ins[i].res = pl.pres.p + i;
      if (geo.scheme == SCHEME_FEM && pl.order == 0 && pl.V.p)
        ins[i].V = pl.V.p + (size_t)i * 6 * (geo.J - 1) * geo.nt * geo.nx;
      if (pl.order == 1) ins[i].xmode = (i & 1) ? 1 : 2;  // the traces its colour sends
    }
  }
  HIP_TRY(pl.dt.upload(h, ins, pl.cs));
  return KFP_OK;
}

// Number of state ping-pong flips of one window: the parity of U holding the
// final state is launches & 1.
static int march_launches(int nt, const Config &cfg) {
  return cfg.steps >= 1 ? (nt + cfg.steps - 1) / cfg.steps : nt;
}

// One iteration's launches: part 1 = the time steps (with the residual
// reset), part 2 = the exchange of the multi-step path, 0 = both.
static kfp_status launch_iteration_direct(const StepTables &t, int n_inst, const InstDev *inst,
                                          const Config &cfg, int nt, int par, int grid,
                                          hipStream_t s, int part = 0) {
  if (part != 2) {
    HIP_TRY(launch_reset_res(inst, n_inst, s));
    if (cfg.steps == 0) {
      for (int n = 0; n <= nt; ++n) HIP_TRY(launch_step(t, cfg.waves, cfg.seg, n, par, grid, s));
    } else {
      const int L = march_launches(nt, cfg);
      for (int l = 0; l < L; ++l)
        HIP_TRY(launch_march(t, cfg.waves, cfg.groups, cfg.seg, cfg.tiles, l * cfg.steps, cfg.steps, halo_of(cfg),
                             l & 1, par, grid, s));
    }
  }
  if (part != 1 && cfg.steps != 0) HIP_TRY(launch_exchange(t, par, cfg.steps, s));
  return KFP_OK;
}

// One iteration in red-black order: the even subdomains march the window and
// send their traces, the odd ones march with those traces and send theirs,
// which also reduces the residual.  The method is causal in time, so the odd
// subdomains march time block l as soon as the even ones have finished it
// and sent its traces: the even half-sweep runs back to back on the solve's
// stream, the traces of each block are sent on a third stream, and the odd
// half-sweep follows on a second one, so the two halves share the device.
// part 1: everything before the last exchange, 2: the last exchange, 0: both.
static kfp_status launch_iteration_rb(const Plan &pl, hipStream_t s, int part = 0) {
  const Config &cfg = pl.cfg;
  const StepTables t = pl.dt.view();
  StepTables tc[2] = {t, t};
  tc[0].n_items = pl.n_red;
  tc[1].items = t.items + pl.n_red;
  tc[1].n_items = t.n_items - pl.n_red;
  if (part != 2) {
    HIP_TRY(launch_reset_res(pl.dt.inst.p, 1, s));
    const int L = march_launches(pl.geo.nt, cfg);
    HIP_TRY(hipEventRecord(pl.ev_fork, s));
    HIP_TRY(hipStreamWaitEvent(pl.cs2, pl.ev_fork, 0));
    HIP_TRY(hipStreamWaitEvent(pl.cs3, pl.ev_fork, 0));
    for (int l = 0; l < L; ++l) {
      // even subdomains, block l: reads only the traces of the previous
      // iteration and writes only even rows and value planes of block l
      if (tc[0].n_items > 0)
        HIP_TRY(launch_march(tc[0], cfg.waves, cfg.groups, cfg.seg, cfg.tiles, l * cfg.steps, cfg.steps,
                             halo_of(cfg), l & 1, 0, tc[0].n_items, s));
      HIP_TRY(hipEventRecord(pl.ev_mar, s));
      HIP_TRY(hipStreamWaitEvent(pl.cs3, pl.ev_mar, 0));
      StepTables tx = t;  // the traces of block l only
      tx.blk = pl.blkseq.p + l;
      HIP_TRY(launch_exchange(tx, 0, cfg.steps, pl.cs3, 1));
      HIP_TRY(hipEventRecord(pl.ev_blk, pl.cs3));
      HIP_TRY(hipStreamWaitEvent(pl.cs2, pl.ev_blk, 0));
      if (tc[1].n_items > 0)
        HIP_TRY(launch_march(tc[1], cfg.waves, cfg.groups, cfg.seg, cfg.tiles, l * cfg.steps, cfg.steps,
                             halo_of(cfg), l & 1, 0, tc[1].n_items, pl.cs2));
    }
    HIP_TRY(hipEventRecord(pl.ev_join, pl.cs2));
    HIP_TRY(hipStreamWaitEvent(s, pl.ev_join, 0));
    HIP_TRY(hipEventRecord(pl.ev_join3, pl.cs3));
    HIP_TRY(hipStreamWaitEvent(s, pl.ev_join3, 0));
  }
  if (part != 1) HIP_TRY(launch_exchange(t, 0, cfg.steps, s, 2));
  return KFP_OK;
}

static kfp_status capture_graphs(Plan &pl) {
  if (pl.captured) return KFP_OK;
  if (pl.order == 1) {  // one pair of graphs: the window does not alternate
    for (int part = 1; part <= 2; ++part) {
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(pl.cs, hipStreamCaptureModeThreadLocal));
      kfp_status st = launch_iteration_rb(pl, pl.cs, part);
      hipError_t e = hipStreamEndCapture(pl.cs, &graph);
      if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
      }
      HIP_TRY(e);
      e = hipGraphInstantiate(part == 1 ? &pl.gexec[0] : &pl.gexch[0], graph, nullptr, nullptr,
                              0);
      (void)hipGraphDestroy(graph);
      HIP_TRY(e);
    }
    pl.captured = true;
    return KFP_OK;
  }
  const StepTables t = pl.dt.view();
  const int parts = pl.cfg.steps != 0 ? 2 : 1;
  for (int par = 0; par < 2; ++par)
    for (int part = 1; part <= parts; ++part) {
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(pl.cs, hipStreamCaptureModeThreadLocal));
      kfp_status st = launch_iteration_direct(t, 1, pl.dt.inst.p, pl.cfg, pl.geo.nt, par,
                                              t.n_items, pl.cs, part);
      hipError_t e = hipStreamEndCapture(pl.cs, &graph);
      if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
      }
      HIP_TRY(e);
      e = hipGraphInstantiate(part == 1 ? &pl.gexec[par] : &pl.gexch[par], graph, nullptr,
                              nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIP_TRY(e);
    }
  pl.captured = true;
  return KFP_OK;
}

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static double bits_to_double(unsigned long long b) {
  double d;
  memcpy(&d, &b, sizeof d);
  return d;
}

static kfp_status sync_in(hipStream_t user, Plan &pl) {
  HIP_TRY(hipEventRecord(pl.ev_in, user));
  HIP_TRY(hipStreamWaitEvent(pl.cs, pl.ev_in, 0));
  return KFP_OK;
}

static kfp_status sync_out(hipStream_t user, Plan &pl) {
  HIP_TRY(hipEventRecord(pl.ev_out, pl.cs));
  HIP_TRY(hipStreamWaitEvent(user, pl.ev_out, 0));
  return KFP_OK;
}

// ------------------------------------------------------- pipelined solve --
// One chunk: G launches, each the march of every slot's current block, the
// exchange of those blocks, and the scheduler.  Captured once as a graph and
// replayed until the scheduler stops; with kernel timing on, launched
// directly with HIP events around each march launch instead.
static kfp_status launch_pipe_chunk(Plan &pl, bool timed) {
  StepTables t = pl.dt.view();
  t.blk = pl.blk.p;
  const Config &c = pl.cfg;
  for (int l = 0; l < pl.G; ++l) {
    if (timed) HIP_TRY(hipEventRecord(pl.tev[2 * l], pl.cs));
    HIP_TRY(launch_march(t, c.waves, c.groups, c.seg, c.tiles, 0, c.steps, halo_of(c), 0, 0, t.n_items, pl.cs));
    if (timed) HIP_TRY(hipEventRecord(pl.tev[2 * l + 1], pl.cs));
    HIP_TRY(launch_exchange(t, 0, c.steps, pl.cs));
    HIP_TRY(launch_pipe_tick(pl.ctl.p, pl.blk.p, pl.iter.p, pl.pres.p, pl.hist.p, pl.cs));
  }
  return KFP_OK;
}

static kfp_status capture_pipe_graph(Plan &pl) {
  if (pl.gpipe) return KFP_OK;
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(pl.cs, hipStreamCaptureModeThreadLocal));
  kfp_status st = launch_pipe_chunk(pl, false);
  hipError_t e = hipStreamEndCapture(pl.cs, &graph);
  if (st) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  HIP_TRY(e);
  e = hipGraphInstantiate(&pl.gpipe, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIP_TRY(e);
  return KFP_OK;
}

static kfp_status pipe_solve(Plan &pl, const Geo &geo, const Config &cfg, double tol,
                             int max_iter, bool had_guess, int restarted, double *uT,
                             double *lambda_out, kfp_swr_stats *stats, hipStream_t user,
                             double t_start) {
  const size_t win = (size_t)2 * (geo.J - 1) * geo.nt * geo.nx;
  const size_t state = (size_t)geo.rows * geo.nx;
  HIP_TRY(pl.hist.alloc(max_iter));
  if (pl.gpipe && pl.gpipe_hist != pl.hist.p) {
    // the chunk graph holds the history pointer: capture again after a resize
    (void)hipGraphExecDestroy(pl.gpipe);
    pl.gpipe = nullptr;
  }
  const bool timed = g_ktime || !use_graphs();
  if (!timed) {
    kfp_status st = capture_pipe_graph(pl);
    if (st) return st;
    pl.gpipe_hist = pl.hist.p;
  }
  const long units = pl.order == 1 ? 2L * max_iter : (long)max_iter;
  const long max_launches = (long)pl.L + (long)pl.d * (units - 1) + pl.G;
  double dev_ms = 0.0, step_ms = 0.0;
  long launches = 0;
  for (;;) {
    PipeCtl c{};
    c.t = -1;
    c.kmax = max_iter;
    c.M = pl.M;
    c.d = pl.d;
    c.L = pl.L;
    c.restart_on_nonfinite = (had_guess && !restarted) ? 1 : 0;
    c.last_busy = -1;
    c.rb = pl.order == 1 ? 1 : 0;
    c.tol = tol;
    HIP_TRY(hipMemcpyAsync(pl.ctl.p, &c, sizeof c, hipMemcpyHostToDevice, pl.cs));
    HIP_TRY(hipMemsetAsync(pl.blk.p, 0xff, sizeof(int) * pl.M, pl.cs));  // all idle
    HIP_TRY(launch_pipe_tick(pl.ctl.p, pl.blk.p, pl.iter.p, pl.pres.p, pl.hist.p, pl.cs));
    long chunks = 0;
    for (;;) {
      HIP_TRY(hipEventRecord(pl.ev0, pl.cs));
      if (timed) {
        kfp_status st = launch_pipe_chunk(pl, true);
        if (st) return st;
      } else {
        HIP_TRY(hipGraphLaunch(pl.gpipe, pl.cs));
      }
      HIP_TRY(hipEventRecord(pl.ev1, pl.cs));
      HIP_TRY(hipMemcpyAsync(pl.h_ctl, pl.ctl.p, sizeof(PipeCtl), hipMemcpyDeviceToHost, pl.cs));
      HIP_TRY(hipStreamSynchronize(pl.cs));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, pl.ev0, pl.ev1));
      dev_ms += ms;
      // march launches that had work (the chunk's tail after the stop idles)
      for (int l = 0; l < pl.G; ++l) {
        if (chunks * pl.G + l > pl.h_ctl->last_busy) break;
        if (timed) {
          float m = 0.f;
          HIP_TRY(hipEventElapsedTime(&m, pl.tev[2 * l], pl.tev[2 * l + 1]));
          step_ms += m;
        }
        ++launches;
      }
      ++chunks;
      if (pl.h_ctl->stop != 0 || pl.h_ctl->done >= max_iter) break;
      if (chunks * pl.G > max_launches)
        return fail(KFP_EDEVICE, "pipelined iterations did not finish (%d done)",
                    pl.h_ctl->done);
    }
    if (pl.h_ctl->stop == -1) {
      // a finite-looking guess that still produced a non-finite mismatch:
      // restart once from zero traces
      HIP_TRY(launch_fill(pl.W.p, win, 0.0, pl.cs));
      restarted = 1;
      continue;
    }
    break;
  }
  const int k = pl.h_ctl->stop > 0 ? pl.h_ctl->stop : pl.h_ctl->done;
  std::vector<double> hist(k);
  HIP_TRY(hipMemcpyAsync(hist.data(), pl.hist.p, sizeof(double) * k, hipMemcpyDeviceToHost,
                         pl.cs));
  HIP_TRY(hipStreamSynchronize(pl.cs));
  const double r = hist[k - 1];
  const size_t fin = (pl.L & 1) ? state : 0;  // ping-pong half holding level nt
  if (pl.order == 1) {
    // iteration k: the even subdomains' state and traces from the slot of
    // half-sweep 2k-1, the odd ones' from the slot of half-sweep 2k
    const int sr = (2 * k - 1) % pl.M, sb = (2 * k) % pl.M;
    HIP_TRY(launch_assemble(pl.slotU.p + (size_t)sr * 2 * state + fin, pl.rowmap_rb.p, uT,
                            geo.nv, geo.nx, pl.cs, out_nudt(geo), 2.0 / geo.nv));
    HIP_TRY(launch_assemble(pl.slotU.p + (size_t)sb * 2 * state + fin,
                            pl.rowmap_rb.p + (geo.nv + 1), uT, geo.nv, geo.nx, pl.cs,
                            out_nudt(geo), 2.0 / geo.nv));
    if (lambda_out && win) {
      const size_t plane = (size_t)geo.nt * geo.nx;
      for (int pidx = 0; pidx < 2 * (geo.J - 1); ++pidx) {
        const int j = pidx / 2, sender = (pidx & 1) ? j + 1 : j;
        const int slot = (sender & 1) ? sb : sr;
        HIP_TRY(launch_copy(pl.W.p + (size_t)slot * win + pidx * plane,
                            lambda_out + pidx * plane, plane, pl.cs));
      }
    }
  } else {
    const int slot = k % pl.M;
    HIP_TRY(launch_assemble(pl.slotU.p + (size_t)slot * 2 * state + fin, pl.rowmap.p, uT,
                            geo.nv, geo.nx, pl.cs, out_nudt(geo), 2.0 / geo.nv));
    if (lambda_out && win)
      HIP_TRY(launch_copy(pl.W.p + (size_t)slot * win, lambda_out, win, pl.cs));
  }
  kfp_status st2 = sync_out(user, pl);
  if (st2) return st2;
  HIP_TRY(hipStreamSynchronize(pl.cs));
  const bool converged = r < tol;
  if (stats) {
    stats->iters = k;
    stats->restarted = restarted;
    stats->residual = r;
    stats->device_seconds = dev_ms * 1e-3;
    stats->step_seconds = (timed ? step_ms : dev_ms) * 1e-3;
    stats->step_launches = (double)launches;
    stats->cell_steps = (double)k * geo.nt * geo.nx * geo.rows;
    stats->alg_bytes = 24.0 * stats->cell_steps;
    stats->seconds = now_s() - t_start;
    if (stats->res_history)
      for (int i = 0; i < k; ++i) stats->res_history[i] = hist[i];
  }
  (void)cfg;
  if (!converged) return fail(KFP_ENOCONV, "no convergence after %d iterations (r = %g)", k, r);
  return KFP_OK;
}

// ------------------------------------------------------------------ solves --
static kfp_status swr_solve_impl(const kfp_grid *g, const double *u0, const double *f,
                                 const double *s, int J, int o, int tr, double p, double q,
                                 double tol,
                                 int max_iter, const double *lambda_init, double *uT,
                                 double *lambda_out, kfp_swr_stats *stats, hipStream_t user) {
  const double t_start = now_s();
  Geo geo;
  kfp_status st = make_geo(g, J, o, tr, p, geo, g_scheme);
  if (st) return st;
  if (!u0 || !f || !uT) return fail(KFP_EINVAL, "u0, f and uT must be non-NULL");
  if (!(tol > 0.0)) return fail(KFP_EINVAL, "tol must be > 0");
  if (max_iter < 1) return fail(KFP_EINVAL, "max_iter must be >= 1");
  if (s)
    for (int n = 0; n <= g->nt; ++n)
      if (!std::isfinite(s[n])) return fail(KFP_EINVAL, "s[%d] is not finite", n);
  const int order = J > 1 ? g_order : 0;
  const Config cfg = choose_config(geo, order);
  if ((st = fem_needs_march(geo, cfg))) return st;
  if (order == 1 && cfg.steps == 0)
    return fail(KFP_EINVAL,
                "red-black order needs a march configuration (subdomains of at most 1056 rows; "
                "tallest here %d)", geo.n_max);
  const PipeParams pp = pipe_params(geo, cfg, order);
  Plan *pl = nullptr;
  if ((st = get_plan(geo, cfg, &pl, pp, order))) return st;
  if ((st = sync_in(user, *pl))) return st;
  if ((st = load_instance(*pl, u0, f, s, p, q))) return st;
  const size_t win = (size_t)2 * (J - 1) * geo.nt * geo.nx;
  int restarted = 0;
  // lambda^0 goes to window 0 (pipelined: read by the slot of iteration 1)
  double *lam_first = pl->M > 0 ? pl->W.p : pl->lam0.p;
  if (win) {
    if (lambda_init) {
      HIP_TRY(launch_copy(lambda_init, lam_first, win, pl->cs));
      HIP_TRY(hipMemsetAsync(pl->cnt.p, 0, sizeof(unsigned int), pl->cs));
      HIP_TRY(launch_count_nonfinite(lam_first, win, pl->cnt.p, pl->cs));
      unsigned int bad = 0;
      HIP_TRY(hipMemcpyAsync(&bad, pl->cnt.p, sizeof bad, hipMemcpyDeviceToHost, pl->cs));
      HIP_TRY(hipStreamSynchronize(pl->cs));
      if (bad) {
        HIP_TRY(launch_fill(lam_first, win, 0.0, pl->cs));
        restarted = 1;
      }
    } else {
      HIP_TRY(launch_fill(lam_first, win, 0.0, pl->cs));
    }
  }
  if (pl->M > 0)
    return pipe_solve(*pl, geo, cfg, tol, max_iter, lambda_init != nullptr, restarted, uT,
                      lambda_out, stats, user, t_start);
  const bool graphs = use_graphs();
  if (graphs && (st = capture_graphs(*pl))) return st;
  const StepTables t = pl->dt.view();
  double dev_ms = 0.0, step_ms = 0.0, r = INFINITY;
  int k = 0;
  for (k = 1; k <= max_iter; ++k) {
    // red-black: one window updated in place, so no parity
    const int par = order == 1 ? 0 : (k - 1) & 1;
    HIP_TRY(hipEventRecord(pl->ev0, pl->cs));
    if (graphs) {
      HIP_TRY(hipGraphLaunch(pl->gexec[par], pl->cs));
    } else if ((st = order == 1 ? launch_iteration_rb(*pl, pl->cs, 1)
                                : launch_iteration_direct(t, 1, pl->dt.inst.p, cfg, geo.nt, par,
                                                          t.n_items, pl->cs, 1))) {
      return st;
    }
    HIP_TRY(hipEventRecord(pl->evm, pl->cs));
    if (cfg.steps != 0) {
      if (graphs) {
        HIP_TRY(hipGraphLaunch(pl->gexch[par], pl->cs));
      } else if ((st = order == 1 ? launch_iteration_rb(*pl, pl->cs, 2)
                                  : launch_iteration_direct(t, 1, pl->dt.inst.p, cfg, geo.nt,
                                                            par, t.n_items, pl->cs, 2))) {
        return st;
      }
    }
    HIP_TRY(hipEventRecord(pl->ev1, pl->cs));
    HIP_TRY(hipMemcpyAsync(pl->h_res, pl->res.p, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           pl->cs));
    HIP_TRY(hipStreamSynchronize(pl->cs));
    float ms = 0.f, ms_step = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, pl->ev0, pl->ev1));
    HIP_TRY(hipEventElapsedTime(&ms_step, pl->ev0, pl->evm));
    dev_ms += ms;
    step_ms += ms_step;
    r = bits_to_double(*pl->h_res);
    if (J == 1) r = 0.0;
    if (stats && stats->res_history) stats->res_history[k - 1] = r;
    if (!std::isfinite(r) && k == 1 && lambda_init && !restarted) {
      // a finite-looking guess that still produced a non-finite mismatch:
      // restart once from zero traces
      HIP_TRY(launch_fill(pl->lam0.p, win, 0.0, pl->cs));
      restarted = 1;
      k = 0;
      continue;
    }
    if (r < tol) break;
  }
  const bool converged = k <= max_iter;
  if (!converged) k = max_iter;
  double *Ufin = (march_launches(geo.nt, cfg) & 1) ? pl->U1.p : pl->U0.p;
  HIP_TRY(launch_assemble(Ufin, pl->rowmap.p, uT, geo.nv, geo.nx, pl->cs, out_nudt(geo),
                          2.0 / geo.nv));
  if (lambda_out && win)
    HIP_TRY(launch_copy((order == 0 && (k & 1)) ? pl->lam1.p : pl->lam0.p, lambda_out, win,
                        pl->cs));
  if ((st = sync_out(user, *pl))) return st;
  HIP_TRY(hipStreamSynchronize(pl->cs));
  if (stats) {
    stats->iters = k;
    stats->restarted = restarted;
    stats->residual = r;
    stats->device_seconds = dev_ms * 1e-3;
    stats->step_seconds = step_ms * 1e-3;
    stats->step_launches = (double)k * march_launches(geo.nt, cfg);
    stats->cell_steps = (double)k * geo.nt * geo.nx * geo.rows;
    stats->alg_bytes = 24.0 * stats->cell_steps;
    stats->seconds = now_s() - t_start;
  }
  if (!converged) return fail(KFP_ENOCONV, "no convergence after %d iterations (r = %g)", k, r);
  return KFP_OK;
}

static kfp_status mono_solve_impl(const kfp_grid *g, const double *u0, const double *f,
                                  const double *s, double *uT, hipStream_t user) {
  Geo geo;
  kfp_status st = make_geo(g, 1, 0, KFP_DIRICHLET, 0.0, geo, g_scheme);
  if (st) return st;
  if (!u0 || !f || !uT) return fail(KFP_EINVAL, "u0, f and uT must be non-NULL");
  if (s)
    for (int n = 0; n <= g->nt; ++n)
      if (!std::isfinite(s[n])) return fail(KFP_EINVAL, "s[%d] is not finite", n);
  const Config cfg = choose_config(geo);
  if ((st = fem_needs_march(geo, cfg))) return st;
  Plan *pl = nullptr;
  if ((st = get_plan(geo, cfg, &pl))) return st;
  if ((st = sync_in(user, *pl))) return st;
  if ((st = load_instance(*pl, u0, f, s, 0.0, 0.0))) return st;
  const StepTables t = pl->dt.view();
  if (cfg.steps == 0) {
    for (int n = 0; n < geo.nt; ++n)
      HIP_TRY(launch_step(t, cfg.waves, cfg.seg, n, 0, t.n_items, pl->cs));
  } else {
    const int L = march_launches(geo.nt, cfg);
    for (int l = 0; l < L; ++l)
      HIP_TRY(launch_march(t, cfg.waves, cfg.groups, cfg.seg, cfg.tiles, l * cfg.steps, cfg.steps, halo_of(cfg), l & 1,
                           0, t.n_items, pl->cs));
  }
  double *Ufin = (march_launches(geo.nt, cfg) & 1) ? pl->U1.p : pl->U0.p;
  HIP_TRY(launch_assemble(Ufin, pl->rowmap.p, uT, geo.nv, geo.nx, pl->cs, out_nudt(geo),
                          2.0 / geo.nv));
  return sync_out(user, *pl);
}

// ------------------------------------------------------- static workspace --
// Workspace of kfp_mono_solve_static, for callers that cannot allocate: a
// file-scope device array (each GPU the library runs on holds its own copy
// until the process ends).  In host code the array's name is only a
// stand-in: the device address of the current GPU's copy is looked up once
// per device with hipGetSymbolAddress and only that address is handed to
// kernels and copies.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
static std::map<int, unsigned char *> g_scratch_ptr;  // device -> address of its copy

static kfp_status static_scratch(unsigned char **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(KFP_EDEVICE, "no device address for the static workspace");
    it = g_scratch_ptr.emplace(dev, static_cast<unsigned char *>(p)).first;
  }
  *out = it->second;
  return KFP_OK;
}

// The monodomain march of mono_solve_impl with every buffer carved out of the
// static workspace, launched on the caller's stream: no device allocation,
// no stream or event of its own.  The tables are copied in and the stream is
// synchronised once before the launches (the host tables are temporaries).
static kfp_status mono_solve_static_impl(const kfp_grid *g, const double *u0, const double *f,
                                         const double *s, double *uT, hipStream_t stream) {
  Geo geo;
  kfp_status st = make_geo(g, 1, 0, KFP_DIRICHLET, 0.0, geo, g_scheme);
  if (st) return st;
  if (!u0 || !f || !uT) return fail(KFP_EINVAL, "u0, f and uT must be non-NULL");
  if (s)
    for (int n = 0; n <= g->nt; ++n)
      if (!std::isfinite(s[n])) return fail(KFP_EINVAL, "s[%d] is not finite", n);
  const Config cfg = choose_config(geo);
  if ((st = fem_needs_march(geo, cfg))) return st;
  HostTables h;
  add_instance_cfg(geo, 0.0, 0.0, cfg.waves, cfg.seg, cfg.steps, 0, h);
  make_items(geo, 0, cfg, h.items);
  // the layout of the workspace: 256-byte aligned parts
  size_t used = 0;
  auto take = [&](size_t bytes) {
    const size_t at = used;
    used += (std::max<size_t>(bytes, 8) + 255) & ~(size_t)255;
    return at;
  };
  const size_t state = (size_t)geo.rows * geo.nx;
  const size_t o_u0 = take(state * 8), o_u1 = take(state * 8), o_g = take((size_t)geo.nt * 8);
  const size_t o_lam = take(8), o_res = take(8), o_rowmap = take((size_t)(geo.nv + 1) * 4);
  const size_t o_inst = take(sizeof(InstDev)), o_subs = take(h.subs.size() * sizeof(SubDev));
  const size_t o_items = take(h.items.size() * sizeof(Item));
  const size_t o_rows = take(h.rows.size() * sizeof(RowCoef));
  const size_t o_reds = take(h.reds.size() * sizeof(RedCoef));
  const size_t o_segs = take(h.segs.size() * sizeof(int));
  const size_t o_mrows = take(h.mrows.size() * sizeof(MarchCoef));
  const size_t o_frows = take(h.frows.size() * sizeof(FemCoef));
  const size_t o_fsegs = take(h.fsegs.size() * sizeof(FemSeg));
  const size_t o_rinv = take(h.rinv.size() * sizeof(double));
  if (used > kStaticScratchBytes)
    return fail(KFP_EINVAL,
                "kfp_mono_solve_static: this grid needs %zu bytes of workspace; the static "
                "workspace holds %zu (state of (nv-1) x nx doubles twice, plus tables)",
                used, kStaticScratchBytes);
  unsigned char *base = nullptr;
  if ((st = static_scratch(&base))) return st;
  auto at = [&](size_t o) { return (void *)(base + o); };
  InstDev in{};
  in.U[0] = (double *)at(o_u0);
  in.U[1] = (double *)at(o_u1);
  in.u0 = u0;
  in.f = f;
  in.g = (const double *)at(o_g);
  in.lam[0] = in.lam[1] = (double *)at(o_lam);
  in.res = (unsigned long long *)at(o_res);
  in.V = nullptr;
  const double hv = 2.0 / geo.nv, dt = geo.T / geo.nt;
  in.r = dt / (hv * hv);
  in.hv = hv;
  in.nx = geo.nx;
  in.nv = geo.nv;
  in.nt = geo.nt;
  in.tr = geo.tr;
  in.scheme = geo.scheme;
  in.active = 1;
  std::vector<double> gv(geo.nt);
  for (int n = 0; n < geo.nt; ++n) gv[n] = dt * (s ? s[n + 1] : 1.0);
  in.gconst = g_is_const(gv);
  auto cp = [&](size_t o, const void *src, size_t bytes) {
    return bytes ? hipMemcpyAsync(at(o), src, bytes, hipMemcpyHostToDevice, stream) : hipSuccess;
  };
  HIP_TRY(cp(o_g, gv.data(), gv.size() * 8));
  HIP_TRY(cp(o_rowmap, geo.rowmap.data(), (size_t)(geo.nv + 1) * 4));
  HIP_TRY(cp(o_inst, &in, sizeof in));
  HIP_TRY(cp(o_subs, h.subs.data(), h.subs.size() * sizeof(SubDev)));
  HIP_TRY(cp(o_items, h.items.data(), h.items.size() * sizeof(Item)));
  HIP_TRY(cp(o_rows, h.rows.data(), h.rows.size() * sizeof(RowCoef)));
  HIP_TRY(cp(o_reds, h.reds.data(), h.reds.size() * sizeof(RedCoef)));
  HIP_TRY(cp(o_segs, h.segs.data(), h.segs.size() * sizeof(int)));
  HIP_TRY(cp(o_mrows, h.mrows.data(), h.mrows.size() * sizeof(MarchCoef)));
  HIP_TRY(cp(o_frows, h.frows.data(), h.frows.size() * sizeof(FemCoef)));
  HIP_TRY(cp(o_fsegs, h.fsegs.data(), h.fsegs.size() * sizeof(FemSeg)));
  HIP_TRY(cp(o_rinv, h.rinv.data(), h.rinv.size() * sizeof(double)));
  HIP_TRY(hipStreamSynchronize(stream));  // the host tables go out of scope
  StepTables t{};
  t.inst = (const InstDev *)at(o_inst);
  t.subs = (const SubDev *)at(o_subs);
  t.items = (const Item *)at(o_items);
  t.rows = (const RowCoef *)at(o_rows);
  t.reds = (const RedCoef *)at(o_reds);
  t.segs = (const int *)at(o_segs);
  t.ex = nullptr;
  t.mrows = (const MarchCoef *)at(o_mrows);
  t.frows = (const FemCoef *)at(o_frows);
  t.fsegs = (const FemSeg *)at(o_fsegs);
  t.rinv = (const double *)at(o_rinv);
  t.blk = nullptr;
  t.n_items = (int)h.items.size();
  t.n_ex = 0;
  t.fem = h.fem ? 1 : 0;
  if (cfg.steps == 0) {
    for (int n = 0; n < geo.nt; ++n)
      HIP_TRY(launch_step(t, cfg.waves, cfg.seg, n, 0, t.n_items, stream));
  } else {
    const int L = march_launches(geo.nt, cfg);
    for (int l = 0; l < L; ++l)
      HIP_TRY(launch_march(t, cfg.waves, cfg.groups, cfg.seg, cfg.tiles, l * cfg.steps, cfg.steps,
                           halo_of(cfg), l & 1, 0, t.n_items, stream));
  }
  const double *Ufin = (march_launches(geo.nt, cfg) & 1) ? in.U[1] : in.U[0];
  HIP_TRY(launch_assemble(Ufin, (const int *)at(o_rowmap), uT, geo.nv, geo.nx, stream,
                          out_nudt(geo), 2.0 / geo.nv));
  return KFP_OK;
}

// ------------------------------------------------------------------- batch --
struct BatchInst {
  Geo geo;
  double p, q;
  double *U0 = nullptr, *U1 = nullptr, *lam0 = nullptr, *lam1 = nullptr, *g = nullptr,
         *V = nullptr;
  int *rowmap = nullptr;
  size_t win = 0;
  int cls = 0;  // launch class
};

// Instances whose tallest subdomain needs the same launch configuration
// share tables and launches; every class advances in the same iteration.
struct BatchClass {
  Config cfg;
  std::vector<int> members;
  HostTables h;
  DevTables dt;
  int grid = 1;
  int nt_max = 0;
  int n_red = 0;  // red-black order: the work items of even subdomains come first
};

static std::string batch_key(int n_max) {
  char key[96];
  snprintf(key, sizeof key, "%s/batch/nmax%d%s", arch_name().c_str(), n_max,
           g_scheme == SCHEME_FEM ? "/fem" : "");
  return key;
}

// A configuration the tuner is trying for the batch instances of one
// height (kfp_tune_batch), ahead of the cache and the built-in choice.
static std::map<int, Config> g_batch_try;

// Can a batch class of subdomains of at most n_max rows run configuration c
// in the current discretisation?
static bool batch_usable(const Config &c, int n_max) {
  if (!config_supported(c) || c.steps < 1) return false;
  if (c.tiles > 0) return g_scheme == SCHEME_FD && march_fits(n_max, c.waves, c.seg);
  return march_fits(n_max, c.waves, c.seg, c.groups);
}

static Config batch_config(int n_max) {
  if (g_forced.waves > 0) {
    Geo probe;
    probe.nx = 0;
    probe.n_max = n_max;
    probe.J = 0;
    probe.tr = -1;
    probe.scheme = g_scheme;
    return choose_config(probe);
  }
  auto tr = g_batch_try.find(n_max);
  if (tr != g_batch_try.end()) return tr->second;
  if (!g_tune) g_tune = new std::map<std::string, Config>(load_tune());
  auto it = g_tune->find(batch_key(n_max));
  if (it != g_tune->end() && batch_usable(it->second, n_max)) return it->second;
  // a batch has many work items: the multi-tile kernel with one tile for
  // finite differences, the general march kernel's 8-step layout otherwise
  if (g_scheme == SCHEME_FD) {
    const Config c = default_fd(n_max, 0);
    if (c.waves) return c;
  }
  const Config c = default_march(n_max, 1L << 20);
  return c.waves ? c : default_config(n_max);
}

static kfp_status swr_batch_impl(int n_inst, const kfp_instance *in, double tol, int max_iter,
                                 kfp_swr_stats *stats, hipStream_t user) {
  const double t_start = now_s();
  const int order = g_order;
  if (n_inst < 1 || !in) return fail(KFP_EINVAL, "batch needs n >= 1 instances");
  if (!(tol > 0.0)) return fail(KFP_EINVAL, "tol must be > 0");
  if (max_iter < 1) return fail(KFP_EINVAL, "max_iter must be >= 1");
  std::vector<BatchInst> bi(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    kfp_status st = make_geo(&in[i].g, in[i].J, in[i].overlap, in[i].tr, in[i].p, bi[i].geo, g_scheme);
    if (st) return fail(st, "instance %d: %s", i, g_err.c_str());
    if (!in[i].u0 || !in[i].f || !in[i].uT)
      return fail(KFP_EINVAL, "instance %d: u0, f and uT must be non-NULL", i);
    if (in[i].s)
      for (int n = 0; n <= in[i].g.nt; ++n)
        if (!std::isfinite(in[i].s[n])) return fail(KFP_EINVAL, "instance %d: s not finite", i);
    bi[i].p = in[i].p;
    bi[i].q = in[i].q > 0.0 ? in[i].q : in[i].p;  // q <= 0: one-sided
  }
  // launch classes
  std::vector<BatchClass> cls;
  for (int i = 0; i < n_inst; ++i) {
    const Config c = batch_config(bi[i].geo.n_max);
    int k = 0;
    for (; k < (int)cls.size(); ++k)
      if (cls[k].cfg.waves == c.waves && cls[k].cfg.seg == c.seg && cls[k].cfg.steps == c.steps &&
          cls[k].cfg.groups == c.groups && cls[k].cfg.tiles == c.tiles)
        break;
    if (k == (int)cls.size()) {
      cls.emplace_back();
      cls.back().cfg = c;
    }
    cls[k].members.push_back(i);
    cls[k].nt_max = std::max(cls[k].nt_max, bi[i].geo.nt);
    bi[i].cls = k;
  }
  for (int i = 0; i < n_inst; ++i) {
    kfp_status st = fem_needs_march(bi[i].geo, cls[bi[i].cls].cfg);
    if (st) return fail(st, "instance %d: %s", i, g_err.c_str());
  }
  if (order == 1)
    for (const auto &c : cls)
      if (c.cfg.steps == 0)
        return fail(KFP_EINVAL, "red-black order needs a march configuration for every "
                                "instance (subdomains of at most 1056 rows)");

  hipStream_t cs;
  HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  struct Guard {
    std::vector<void *> ptrs;
    hipStream_t s;
    std::vector<hipGraphExec_t> ge;
    std::vector<BatchClass> *cls;
    ~Guard() {
      for (auto g : ge)
        if (g) (void)hipGraphExecDestroy(g);
      for (auto &c : *cls) c.dt.release();
      for (void *p : ptrs) (void)hipFree(p);
      (void)hipStreamDestroy(s);
    }
  } guard{{}, cs, {nullptr, nullptr}, &cls};
  auto dalloc = [&](size_t bytes, void **p) -> hipError_t {
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 8));
    if (e == hipSuccess) guard.ptrs.push_back(*p);
    return e;
  };
  hipEvent_t ev;
  HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(ev, user));
  HIP_TRY(hipStreamWaitEvent(cs, ev, 0));
  HIP_TRY(hipEventDestroy(ev));

  std::vector<InstDev> idev(n_inst);
  unsigned long long *res = nullptr;
  InstDev *d_inst = nullptr;
  HIP_TRY(dalloc(sizeof(unsigned long long) * n_inst, (void **)&res));
  HIP_TRY(dalloc(sizeof(InstDev) * n_inst, (void **)&d_inst));
  for (int i = 0; i < n_inst; ++i) {
    BatchInst &b = bi[i];
    const Geo &geo = b.geo;
    const Config &cfg = cls[b.cls].cfg;
    const size_t state = (size_t)geo.rows * geo.nx;
    b.win = (size_t)2 * (geo.J - 1) * geo.nt * geo.nx;
    HIP_TRY(dalloc(state * 8, (void **)&b.U0));
    HIP_TRY(dalloc(state * 8, (void **)&b.U1));
    HIP_TRY(dalloc(b.win * 8, (void **)&b.lam0));
    HIP_TRY(dalloc(b.win * 8, (void **)&b.lam1));
    HIP_TRY(dalloc(geo.nt * 8, (void **)&b.g));
    HIP_TRY(dalloc((geo.nv + 1) * sizeof(int), (void **)&b.rowmap));
    if (cfg.steps >= 1 && geo.J > 1)
      HIP_TRY(dalloc((size_t)6 * (geo.J - 1) * geo.nt * geo.nx * 8, (void **)&b.V));
    HIP_TRY(hipMemcpyAsync(b.rowmap, geo.rowmap.data(), (geo.nv + 1) * sizeof(int),
                           hipMemcpyHostToDevice, cs));
    std::vector<double> gv(geo.nt);
    const double hv = 2.0 / geo.nv, dt = geo.T / geo.nt;
    for (int n = 0; n < geo.nt; ++n) gv[n] = dt * (in[i].s ? in[i].s[n + 1] : 1.0);
    HIP_TRY(hipMemcpyAsync(b.g, gv.data(), sizeof(double) * geo.nt, hipMemcpyHostToDevice, cs));
    HIP_TRY(hipStreamSynchronize(cs));
    InstDev &d = idev[i];
    d.U[0] = b.U0;
    d.U[1] = b.U1;
    d.u0 = in[i].u0;
    d.f = in[i].f;
    d.g = b.g;
    d.lam[0] = b.lam0;
    d.lam[1] = order == 1 ? b.lam0 : b.lam1;  // red-black: one window, in place
    d.res = res + i;
    d.V = b.V;
    d.r = dt / (hv * hv);
    d.p = b.p;
    d.q = b.q;
    d.hv = hv;
    d.nx = geo.nx;
    d.nv = geo.nv;
    d.nt = geo.nt;
    d.tr = geo.tr;
    d.nonovl = geo.J > 1 && geo.o == 0 && geo.tr == KFP_ROBIN;
    d.scheme = geo.scheme;
    d.gconst = g_is_const(gv);
    d.active = 1;
    if (b.win) {
      if (in[i].lambda_init) {
        HIP_TRY(launch_copy(in[i].lambda_init, b.lam0, b.win, cs));
      } else {
        HIP_TRY(launch_fill(b.lam0, b.win, 0.0, cs));
      }
    }
  }
  HIP_TRY(hipMemcpyAsync(d_inst, idev.data(), sizeof(InstDev) * n_inst, hipMemcpyHostToDevice, cs));
  int dev_id = 0, cus = 256;
  if (hipGetDevice(&dev_id) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev_id) == hipSuccess) cus = prop.multiProcessorCount;
  }
  // per class: tables, items sorted largest first (LPT) for the persistent
  // grid (red-black: the even subdomains' items first, each colour LPT)
  for (auto &c : cls) {
    std::vector<std::pair<long, Item>> weighted;
    for (int i : c.members) {
      const Geo &geo = bi[i].geo;
      const int sub_base = (int)c.h.subs.size();
      add_instance_cfg(geo, bi[i].p, bi[i].q, c.cfg.waves, c.cfg.seg, c.cfg.steps, i, c.h);
      make_ex(geo, i, c.h.ex);
      std::vector<Item> it;
      make_items(geo, sub_base, c.cfg, it);
      for (const Item &x : it) {
        const long odd = order == 1 ? ((x.sub - sub_base) & 1) : 0;
        weighted.push_back({(long)c.h.subs[x.sub].n * geo.nt - (odd << 40), x});
      }
    }
    std::stable_sort(weighted.begin(), weighted.end(),
                     [](const std::pair<long, Item> &x, const std::pair<long, Item> &y) {
                       return x.first > y.first;
                     });
    for (auto &w : weighted) {
      c.h.items.push_back(w.second);
      if (w.first >= 0) ++c.n_red;
    }
    HIP_TRY(c.dt.upload(c.h, {}, cs));
    c.grid = std::max(1, std::min<int>((int)c.h.items.size(),
                                       cus * std::max(1, 32 / c.cfg.waves)));
  }
  auto view = [&](BatchClass &c) {
    StepTables t = c.dt.view();
    t.inst = d_inst;
    return t;
  };

  // non-finite guesses fall back to zero
  std::vector<int> restarted(n_inst, 0);
  {
    unsigned int *cnt = nullptr;
    HIP_TRY(dalloc(sizeof(unsigned int) * n_inst, (void **)&cnt));
    HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(unsigned int) * n_inst, cs));
    for (int i = 0; i < n_inst; ++i)
      if (in[i].lambda_init && bi[i].win) HIP_TRY(launch_count_nonfinite(bi[i].lam0, bi[i].win, cnt + i, cs));
    std::vector<unsigned int> hc(n_inst);
    HIP_TRY(hipMemcpyAsync(hc.data(), cnt, sizeof(unsigned int) * n_inst, hipMemcpyDeviceToHost, cs));
    HIP_TRY(hipStreamSynchronize(cs));
    for (int i = 0; i < n_inst; ++i)
      if (hc[i]) {
        HIP_TRY(launch_fill(bi[i].lam0, bi[i].win, 0.0, cs));
        restarted[i] = 1;
      }
  }

  // launch classes run side by side: one stream each, forked from and joined
  // back into the batch stream (inside the captured graph: parallel branches)
  struct Streams {
    std::vector<hipStream_t> s;
    std::vector<hipEvent_t> e;
    ~Streams() {
      for (auto x : s)
        if (x) (void)hipStreamDestroy(x);
      for (auto x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } side;
  side.s.assign(cls.size(), nullptr);
  side.e.assign(cls.size() + 1, nullptr);
  for (auto &x : side.s) HIP_TRY(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
  for (auto &x : side.e) HIP_TRY(hipEventCreateWithFlags(&x, hipEventDisableTiming));
  auto iteration = [&](int par) -> kfp_status {
    HIP_TRY(launch_reset_res(d_inst, n_inst, cs));
    HIP_TRY(hipEventRecord(side.e[cls.size()], cs));
    for (size_t ci = 0; ci < cls.size(); ++ci) {
      BatchClass &c = cls[ci];
      hipStream_t s = side.s[ci];
      HIP_TRY(hipStreamWaitEvent(s, side.e[cls.size()], 0));
      const StepTables t = view(c);
      if (order == 1) {
        // red-black: the even subdomains march the window and send their
        // traces, then the odd ones march with them and send theirs
        StepTables tc[2] = {t, t};
        tc[0].n_items = c.n_red;
        tc[1].items = t.items + c.n_red;
        tc[1].n_items = t.n_items - c.n_red;
        const int L = march_launches(c.nt_max, c.cfg);
        for (int h = 0; h < 2; ++h) {
          const int grid = std::min(c.grid, tc[h].n_items);
          if (grid > 0)
            for (int l = 0; l < L; ++l)
              HIP_TRY(launch_march(tc[h], c.cfg.waves, c.cfg.groups, c.cfg.seg, c.cfg.tiles, l * c.cfg.steps,
                                   c.cfg.steps, halo_of(c.cfg), l & 1, 0, grid, s));
          HIP_TRY(launch_exchange(t, 0, c.cfg.steps, s, h + 1));
        }
      } else if (c.cfg.steps == 0) {
        for (int n = 0; n <= c.nt_max; ++n)
          HIP_TRY(launch_step(t, c.cfg.waves, c.cfg.seg, n, par, c.grid, s));
      } else {
        const int L = march_launches(c.nt_max, c.cfg);
        for (int l = 0; l < L; ++l)
          HIP_TRY(launch_march(t, c.cfg.waves, c.cfg.groups, c.cfg.seg, c.cfg.tiles, l * c.cfg.steps, c.cfg.steps,
                               halo_of(c.cfg), l & 1, par, c.grid, s));
        HIP_TRY(launch_exchange(t, par, c.cfg.steps, s));
      }
      HIP_TRY(hipEventRecord(side.e[ci], s));
      HIP_TRY(hipStreamWaitEvent(cs, side.e[ci], 0));
    }
    return KFP_OK;
  };

  const bool graphs = use_graphs();
  if (graphs) {
    for (int par = 0; par < 2; ++par) {
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      kfp_status st = iteration(par);
      hipError_t e = hipStreamEndCapture(cs, &graph);
      if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
      }
      HIP_TRY(e);
      e = hipGraphInstantiate(&guard.ge[par], graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIP_TRY(e);
    }
  }
  unsigned long long *h_res = nullptr;
  HIP_TRY(hipHostMalloc((void **)&h_res, sizeof(unsigned long long) * n_inst));
  struct HGuard {
    void *p;
    ~HGuard() { (void)hipHostFree(p); }
  } hg{h_res};
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  struct EGuard {
    hipEvent_t a, b;
    ~EGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } eg{e0, e1};
  std::vector<int> iters(n_inst, 0), done(n_inst, 0);
  std::vector<double> resid(n_inst, INFINITY);
  double dev_ms = 0.0;
  int active = n_inst;
  for (int k = 1; k <= max_iter && active > 0; ++k) {
    const int par = order == 1 ? 0 : (k - 1) & 1;
    HIP_TRY(hipEventRecord(e0, cs));
    if (graphs) {
      HIP_TRY(hipGraphLaunch(guard.ge[par], cs));
    } else {
      kfp_status st = iteration(par);
      if (st) return st;
    }
    HIP_TRY(hipEventRecord(e1, cs));
    HIP_TRY(hipMemcpyAsync(h_res, res, sizeof(unsigned long long) * n_inst, hipMemcpyDeviceToHost, cs));
    HIP_TRY(hipStreamSynchronize(cs));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    dev_ms += ms;
    bool changed = false;
    for (int i = 0; i < n_inst; ++i) {
      if (done[i]) continue;
      iters[i] = k;
      const Geo &geo = bi[i].geo;
      double r = geo.J == 1 ? 0.0 : bits_to_double(h_res[i]);
      resid[i] = r;
      if (stats && stats[i].res_history) stats[i].res_history[k - 1] = r;
      if (r < tol) {
        done[i] = 1;
        --active;
        idev[i].active = 0;
        changed = true;
      }
    }
    if (changed) {
      HIP_TRY(hipMemcpyAsync(d_inst, idev.data(), sizeof(InstDev) * n_inst, hipMemcpyHostToDevice,
                             cs));
      HIP_TRY(hipStreamSynchronize(cs));
    }
  }
  for (int i = 0; i < n_inst; ++i) {
    const BatchInst &b = bi[i];
    const Geo &geo = b.geo;
    double *Ufin = (march_launches(geo.nt, cls[b.cls].cfg) & 1) ? b.U1 : b.U0;
    HIP_TRY(launch_assemble(Ufin, b.rowmap, in[i].uT, geo.nv, geo.nx, cs, out_nudt(geo),
                            2.0 / geo.nv));
    if (in[i].lambda_out && b.win)
      HIP_TRY(launch_copy((order == 0 && (iters[i] & 1)) ? b.lam1 : b.lam0, in[i].lambda_out,
                          b.win, cs));
  }
  HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(ev, cs));
  HIP_TRY(hipStreamWaitEvent(user, ev, 0));
  HIP_TRY(hipStreamSynchronize(cs));
  HIP_TRY(hipEventDestroy(ev));
  const double secs = now_s() - t_start;
  if (stats) {
    for (int i = 0; i < n_inst; ++i) {
      const Geo &geo = bi[i].geo;
      stats[i].iters = iters[i];
      stats[i].restarted = restarted[i];
      stats[i].residual = resid[i];
      stats[i].seconds = secs;
      stats[i].device_seconds = dev_ms * 1e-3;
      stats[i].step_seconds = dev_ms * 1e-3;  // batch iterations are not split
      stats[i].step_launches = 0;
      stats[i].cell_steps = (double)iters[i] * geo.nt * geo.nx * geo.rows;
      stats[i].alg_bytes = 24.0 * stats[i].cell_steps;
    }
  }
  if (active > 0) return fail(KFP_ENOCONV, "%d of %d instances did not converge", active, n_inst);
  return KFP_OK;
}

// -------------------------------------------------------------------- tune --
static kfp_status tune_impl(const kfp_grid *g, int J, int o, int tr, double p, int *w_out,
                            int *s_out, int *k_out, hipStream_t user) {
  Geo geo;
  kfp_status st = make_geo(g, J, o, tr, p, geo, g_scheme);
  if (st) return st;
  const size_t nfield = (size_t)(g->nv + 1) * g->nx;
  double *u0 = nullptr, *f = nullptr;
  HIP_TRY(hipMalloc((void **)&u0, nfield * 8));
  struct F {
    double **a, **b;
    ~F() {
      if (*a) (void)hipFree(*a);
      if (*b) (void)hipFree(*b);
    }
  } fr{&u0, &f};
  HIP_TRY(hipMalloc((void **)&f, nfield * 8));
  HIP_TRY(launch_fill(u0, nfield, 0.5, nullptr));
  HIP_TRY(launch_fill(f, nfield, 0.25, nullptr));
  HIP_TRY(hipDeviceSynchronize());
  const Config saved = g_forced;
  Config best;
  double best_ms = INFINITY;
  const int steps = std::min(g->nt, 96);
  std::vector<Config> cands;
  for (int w : kWaves) {
    const int s0 = seg_for(geo.n_max, w);
    if (s0 > 0) cands.push_back(Config{w, s0, 0});
    cands.push_back(Config{w, 0, 0});
    const int sm = march_seg_for(geo.n_max, w);
    if (sm)
      for (int k : {1, 4, 8, 12, 16}) cands.push_back(Config{w, sm, k});
  }
  for (int g : {2, 4}) {
    const int sm = march_seg_for(geo.n_max, 8, g);
    if (sm)
      for (int k : {2, 3, 4, 6, 8}) cands.push_back(Config{8, sm, k, g});
  }
  // the multi-tile finite-difference kernel (one segment per wavefront)
  if (geo.scheme == SCHEME_FD)
    for (int w : {4, 8})
      for (int tl : {1, 2})
        for (int sm = 2; sm <= 33; ++sm)
          if (march_fits(geo.n_max, w, sm) && fd_config_supported(w, sm, tl)) {
            for (int k : {4, 8, 12, 15, 16}) cands.push_back(Config{w, sm, k, 1, tl});
            break;
          }
  {
    for (const Config &c : cands) {
      const int w = c.waves, sm = c.seg;
      if (!config_supported(c)) continue;
      if (geo.scheme == SCHEME_FEM && c.steps == 0) continue;  // march kernel only
      Plan *pl = nullptr;
      if ((st = get_plan(geo, c, &pl))) return st;
      if ((st = load_instance(*pl, u0, f, nullptr, tr == KFP_ROBIN ? p : 1.0,
                              tr == KFP_ROBIN ? p : 1.0)))
        return st;
      if (geo.J > 1) HIP_TRY(launch_fill(pl->lam0.p, (size_t)2 * (geo.J - 1) * geo.nt * geo.nx, 0.0, pl->cs));
      const StepTables t = pl->dt.view();
      auto run = [&](int nsteps) -> kfp_status {
        if (c.steps == 0) {
          for (int n = 0; n < nsteps; ++n) HIP_TRY(launch_step(t, w, sm, n, 0, t.n_items, pl->cs));
        } else {
          for (int n = 0; n < nsteps; n += c.steps)
            HIP_TRY(launch_march(t, w, c.groups, sm, c.tiles, n, c.steps, halo_of(c), (n / c.steps) & 1,
                                 0, t.n_items, pl->cs));
        }
        return KFP_OK;
      };
      if ((st = run(std::min(steps, 16)))) return st;
      HIP_TRY(hipEventRecord(pl->ev0, pl->cs));
      if ((st = run(steps))) return st;
      HIP_TRY(hipEventRecord(pl->ev1, pl->cs));
      HIP_TRY(hipStreamSynchronize(pl->cs));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, pl->ev0, pl->ev1));
      if (c.steps >= 1 && geo.J > 1) {
        // the exchange pass runs once per window: charge its share
        float ex_ms = 0.f;
        HIP_TRY(hipEventRecord(pl->ev0, pl->cs));
        HIP_TRY(launch_exchange(t, 0, c.steps, pl->cs));
        HIP_TRY(hipEventRecord(pl->ev1, pl->cs));
        HIP_TRY(hipStreamSynchronize(pl->cs));
        HIP_TRY(hipEventElapsedTime(&ex_ms, pl->ev0, pl->ev1));
        ms += ex_ms * (float)steps / (float)geo.nt;
      }
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
  }
  g_forced = saved;
  if (best.waves == 0) return fem_needs_march(geo, Config{});
  if (!g_tune) g_tune = new std::map<std::string, Config>(load_tune());
  (*g_tune)[tune_key(geo)] = best;
  save_tune(*g_tune);
  if (w_out) *w_out = best.waves;
  if (s_out) *s_out = best.seg;
  if (k_out) *k_out = best.steps;
  (void)user;
  return KFP_OK;
}

// Batch tuning: the instances are grouped by the height of their tallest
// subdomain (the key of a batch launch class); for each height every
// compiled march configuration that holds it is timed on the group's
// instances (`iters` SWR iterations of kfp_swr_batch, device time) and the
// fastest is stored under the batch key of that height.
static kfp_status tune_batch_impl(int n, const kfp_instance *in, int iters, int *groups_out,
                                  hipStream_t user) {
  if (n < 1 || !in) return fail(KFP_EINVAL, "batch tuning needs n >= 1 instances");
  if (iters < 1) return fail(KFP_EINVAL, "iters must be >= 1");
  std::map<int, std::vector<int>> by_h;
  for (int i = 0; i < n; ++i) {
    Geo geo;
    kfp_status st = make_geo(&in[i].g, in[i].J, in[i].overlap, in[i].tr, in[i].p, geo, g_scheme);
    if (st) return fail(st, "instance %d: %s", i, g_err.c_str());
    by_h[geo.n_max].push_back(i);
  }
  const Config saved = g_forced;
  g_forced = Config{};
  g_batch_try.clear();
  struct Restore {
    Config c;
    ~Restore() {
      g_forced = c;
      g_batch_try.clear();
    }
  } restore{saved};
  if (!g_tune) g_tune = new std::map<std::string, Config>(load_tune());
  std::vector<kfp_swr_stats> stats(n);
  for (auto &hv : by_h) {
    const int n_max = hv.first;
    std::vector<kfp_instance> sub;
    for (int i : hv.second) sub.push_back(in[i]);
    std::vector<Config> cands;
    if (g_scheme == SCHEME_FD)
      for (int w : {4, 8})
        for (int tl : {1, 2})
          for (int sm = 2; sm <= 33; ++sm)
            if (march_fits(n_max, w, sm) && fd_config_supported(w, sm, tl)) {
              for (int k : {8, 12, 15, 16}) cands.push_back(Config{w, sm, k, 1, tl});
              break;
            }
    for (int w : kWaves) {
      const int sm = march_seg_for(n_max, w);
      if (sm)
        for (int k : {8, 16}) cands.push_back(Config{w, sm, k});
    }
    for (int g : {2, 4}) {
      const int sm = march_seg_for(n_max, 8, g);
      if (sm)
        for (int k : {4, 6}) cands.push_back(Config{8, sm, k, g});
    }
    Config best;
    double best_s = INFINITY;
    for (const Config &c : cands) {
      if (!batch_usable(c, n_max)) continue;
      g_batch_try[n_max] = c;
      for (auto &x : stats) x = kfp_swr_stats{};
      kfp_status st = swr_batch_impl((int)sub.size(), sub.data(), 1e-300, iters, stats.data(), user);
      if (st != KFP_OK && st != KFP_ENOCONV) return st;
      g_err.clear();
      if (stats[0].device_seconds < best_s) {
        best_s = stats[0].device_seconds;
        best = c;
      }
    }
    g_batch_try.erase(n_max);
    if (best.waves) (*g_tune)[batch_key(n_max)] = best;
  }
  save_tune(*g_tune);
  if (groups_out) *groups_out = (int)by_h.size();
  return KFP_OK;
}

}  // namespace kfp

// ====================================================================== ABI ==
using namespace kfp;

extern "C" {

kfp_status kfp_mono_solve(const kfp_grid *g, const double *u0, const double *f, const double *s,
                          double *uT, void *stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  return mono_solve_impl(g, u0, f, s, uT, (hipStream_t)stream);
}

kfp_status kfp_mono_solve_static(const kfp_grid *g, const double *u0, const double *f,
                                 const double *s, double *uT, void *stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  return mono_solve_static_impl(g, u0, f, s, uT, (hipStream_t)stream);
}

kfp_status kfp_swr_solve(const kfp_grid *g, const double *u0, const double *f, const double *s,
                         int32_t J, int32_t overlap, int32_t tr, double p, double tol,
                         int32_t max_iter, const double *lambda_init, double *uT,
                         double *lambda_out, kfp_swr_stats *stats, void *stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  return swr_solve_impl(g, u0, f, s, J, overlap, tr, p, p, tol, max_iter, lambda_init, uT,
                        lambda_out, stats, (hipStream_t)stream);
}

kfp_status kfp_swr_solve_pq(const kfp_grid *g, const double *u0, const double *f,
                            const double *s, int32_t J, int32_t overlap, int32_t tr, double p,
                            double q, double tol, int32_t max_iter, const double *lambda_init,
                            double *uT, double *lambda_out, kfp_swr_stats *stats,
                            void *stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  if (tr == KFP_ROBIN && !(q > 0.0 && std::isfinite(q)))
    return fail(KFP_EINVAL, "Robin transmission needs q > 0 (got %g)", q);
  return swr_solve_impl(g, u0, f, s, J, overlap, tr, p, q, tol, max_iter, lambda_init, uT,
                        lambda_out, stats, (hipStream_t)stream);
}

static kfp_status u0_guess_impl(const kfp_grid *g, const double *u0, int32_t J, int32_t overlap,
                                int32_t tr, double p, double q, double *lambda, void *stream);

// Time windows: [0, T] cut into W windows of whole steps (window w takes the
// steps floor(w nt / W) .. floor((w+1) nt / W) - 1, the same dt); each is
// solved by SWR to the tolerance from the glued iterate at the end of the
// window before (window 0 from u0), with the source levels of its steps, so
// only one window's traces are held.  guess: initial traces of each window
// 0 zero, 1 the extension Q(start state) of kfp_u0_guess.
// lam_full: initial traces of the whole [0, T] ([2(J-1)][nt][nx]); window w
// starts from its levels (guess is then ignored).
static kfp_status swr_windows_impl(const kfp_grid *g, const double *u0, const double *f,
                                   const double *s, int J, int o, int tr, double p, double q,
                                   double tol, int max_iter, int W, int guess, double *uT,
                                   int32_t *window_iters, kfp_swr_stats *stats,
                                   hipStream_t user, const double *lam_full = nullptr) {
  const double t_start = now_s();
  Geo geo;
  kfp_status st = make_geo(g, J, o, tr, p, geo, g_scheme);
  if (st) return st;
  if (W < 1 || W > g->nt) return fail(KFP_EINVAL, "n_windows must be in 1..nt (got %d)", W);
  if (guess != 0 && guess != 1) return fail(KFP_EINVAL, "guess must be 0 or 1");
  if (!u0 || !f || !uT) return fail(KFP_EINVAL, "u0, f and uT must be non-NULL");
  if (!(tol > 0.0)) return fail(KFP_EINVAL, "tol must be > 0");
  if (max_iter < 1) return fail(KFP_EINVAL, "max_iter must be >= 1");
  const double dt = g->T / g->nt;
  const size_t field = (size_t)(g->nv + 1) * g->nx;
  const int ntw_max = (g->nt + W - 1) / W;
  struct Bufs {
    double *tmp = nullptr, *lam = nullptr;
    int *ab = nullptr;
    ~Bufs() {
      if (tmp) (void)hipFree(tmp);
      if (lam) (void)hipFree(lam);
      if (ab) (void)hipFree(ab);
    }
  } b;
  if (W > 1) HIP_TRY(hipMalloc((void **)&b.tmp, 2 * field * sizeof(double)));
  const bool use_full = lam_full != nullptr && J > 1;
  const bool use_guess = guess == 1 && J > 1 && !use_full;
  if (use_full)
    HIP_TRY(hipMalloc((void **)&b.lam, (size_t)2 * (J - 1) * ntw_max * g->nx * sizeof(double)));
  if (use_guess) {
    HIP_TRY(hipMalloc((void **)&b.lam, (size_t)2 * (J - 1) * ntw_max * g->nx * sizeof(double)));
    std::vector<int> ab;
    for (int j = 0; j + 1 < J; ++j) {
      ab.push_back(geo.sub[j + 1].a);
      ab.push_back(geo.sub[j].b);
    }
    HIP_TRY(hipMalloc((void **)&b.ab, ab.size() * sizeof(int)));
    HIP_TRY(hipMemcpy(b.ab, ab.data(), ab.size() * sizeof(int), hipMemcpyHostToDevice));
  }
  kfp_swr_stats agg{};
  kfp_status worst = KFP_OK;
  const double *start = u0;
  for (int w = 0; w < W; ++w) {
    const int n0 = (int)((long)w * g->nt / W);
    const int n1 = (int)((long)(w + 1) * g->nt / W);
    const int ntw = n1 - n0;
    kfp_grid gw = *g;
    gw.nt = ntw;
    gw.T = ntw * dt;
    double *out = (w == W - 1) ? uT : b.tmp + (size_t)(w & 1) * field;
    if (use_guess)
      HIP_TRY(launch_u0_guess(start, g->nx, ntw, J, b.ab, tr, p, q, 2.0 / g->nv, b.lam, user));
    if (use_full)  // the window's levels of every plane, packed
      HIP_TRY(hipMemcpy2DAsync(b.lam, (size_t)ntw * g->nx * sizeof(double),
                               lam_full + (size_t)n0 * g->nx,
                               (size_t)g->nt * g->nx * sizeof(double),
                               (size_t)ntw * g->nx * sizeof(double), (size_t)2 * (J - 1),
                               hipMemcpyDeviceToDevice, user));
    kfp_swr_stats sw{};
    if (stats && stats->res_history) sw.res_history = stats->res_history + (size_t)w * max_iter;
    st = swr_solve_impl(&gw, start, f, s ? s + n0 : nullptr, J, o, tr, p, q, tol, max_iter,
                        (use_guess || use_full) ? b.lam : nullptr, out, nullptr, &sw, user);
    if (st != KFP_OK && st != KFP_ENOCONV) return st;
    if (st == KFP_ENOCONV) worst = KFP_ENOCONV;
    if (window_iters) window_iters[w] = sw.iters;
    agg.iters += sw.iters;
    agg.restarted |= sw.restarted;
    agg.residual = std::max(agg.residual, sw.residual);
    agg.device_seconds += sw.device_seconds;
    agg.step_seconds += sw.step_seconds;
    agg.step_launches += sw.step_launches;
    agg.cell_steps += sw.cell_steps;
    agg.alg_bytes += sw.alg_bytes;
    start = out;
  }
  // the window buffers are freed on return: the caller's stream must have
  // consumed them (the last window wrote uT itself)
  HIP_TRY(hipStreamSynchronize(user));
  if (stats) {
    double *h = stats->res_history;
    *stats = agg;
    stats->res_history = h;
    stats->seconds = now_s() - t_start;
  }
  if (worst) return fail(KFP_ENOCONV, "a window did not converge in %d iterations", max_iter);
  return KFP_OK;
}

kfp_status kfp_swr_solve_windows(const kfp_grid *g, const double *u0, const double *f,
                                 const double *s, int32_t J, int32_t overlap, int32_t tr,
                                 double p, double q, double tol, int32_t max_iter,
                                 int32_t n_windows, int32_t guess, double *uT,
                                 int32_t *window_iters, kfp_swr_stats *stats, void *stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  if (tr == KFP_ROBIN && !(q > 0.0 && std::isfinite(q)))
    return fail(KFP_EINVAL, "Robin transmission needs q > 0 (got %g)", q);
  return swr_windows_impl(g, u0, f, s, J, overlap, tr, p, q, tol, max_iter, n_windows, guess,
                          uT, window_iters, stats, (hipStream_t)stream);
}

kfp_status kfp_swr_solve_windows_init(const kfp_grid *g, const double *u0, const double *f,
                                      const double *s, int32_t J, int32_t overlap, int32_t tr,
                                      double p, double q, double tol, int32_t max_iter,
                                      int32_t n_windows, const double *lambda_init, double *uT,
                                      int32_t *window_iters, kfp_swr_stats *stats,
                                      void *stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  if (tr == KFP_ROBIN && !(q > 0.0 && std::isfinite(q)))
    return fail(KFP_EINVAL, "Robin transmission needs q > 0 (got %g)", q);
  if (!lambda_init && J > 1) return fail(KFP_EINVAL, "lambda_init must be non-NULL");
  return swr_windows_impl(g, u0, f, s, J, overlap, tr, p, q, tol, max_iter, n_windows, 0, uT,
                          window_iters, stats, (hipStream_t)stream, lambda_init);
}

kfp_status kfp_u0_guess(const kfp_grid *g, const double *u0, int32_t J, int32_t overlap,
                        int32_t tr, double p, double *lambda, void *stream) {
  return u0_guess_impl(g, u0, J, overlap, tr, p, p, lambda, stream);
}

kfp_status kfp_u0_guess_pq(const kfp_grid *g, const double *u0, int32_t J, int32_t overlap,
                           int32_t tr, double p, double q, double *lambda, void *stream) {
  if (tr == KFP_ROBIN && !(q > 0.0 && std::isfinite(q))) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    return fail(KFP_EINVAL, "Robin transmission needs q > 0 (got %g)", q);
  }
  return u0_guess_impl(g, u0, J, overlap, tr, p, q, lambda, stream);
}

static kfp_status u0_guess_impl(const kfp_grid *g, const double *u0, int32_t J, int32_t overlap,
                                int32_t tr, double p, double q, double *lambda, void *stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  Geo geo;
  kfp_status st = make_geo(g, J, overlap, tr, p, geo, g_scheme);
  if (st) return st;
  if (!u0 || (!lambda && J > 1)) return fail(KFP_EINVAL, "u0 and lambda must be non-NULL");
  if (J == 1) return KFP_OK;
  Plan *pl = nullptr;
  if ((st = get_plan(geo, choose_config(geo), &pl))) return st;
  if ((st = sync_in((hipStream_t)stream, *pl))) return st;
  HIP_TRY(launch_u0_guess(u0, geo.nx, geo.nt, J, pl->ab.p, tr, p, q, 2.0 / geo.nv, lambda,
                          pl->cs));
  return sync_out((hipStream_t)stream, *pl);
}

kfp_status kfp_swr_batch(int32_t n, const kfp_instance *inst, double tol, int32_t max_iter,
                         kfp_swr_stats *stats, void *stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  return swr_batch_impl(n, inst, tol, max_iter, stats, (hipStream_t)stream);
}

kfp_status kfp_tune(const kfp_grid *g, int32_t J, int32_t overlap, int32_t tr, double p,
                    int32_t *waves_out, int32_t *seg_max_out, int32_t *steps_out, void *stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  return tune_impl(g, J, overlap, tr, p, waves_out, seg_max_out, steps_out, (hipStream_t)stream);
}

kfp_status kfp_tune_batch(int32_t n, const kfp_instance *inst, int32_t iters,
                          int32_t *groups_out, void *stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  return tune_batch_impl(n, inst, iters, groups_out, (hipStream_t)stream);
}

kfp_status kfp_get_batch_launch(const kfp_instance *inst, int32_t *waves_out,
                                int32_t *groups_out, int32_t *seg_max_out, int32_t *steps_out,
                                int32_t *tiles_out) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  if (!inst) return fail(KFP_EINVAL, "inst is NULL");
  Geo geo;
  kfp_status st = make_geo(&inst->g, inst->J, inst->overlap, inst->tr, inst->p, geo, g_scheme);
  if (st) return st;
  const Config c = batch_config(geo.n_max);
  if (waves_out) *waves_out = c.waves;
  if (groups_out) *groups_out = c.groups;
  if (seg_max_out) *seg_max_out = c.seg;
  if (steps_out) *steps_out = c.steps;
  if (tiles_out) *tiles_out = c.tiles;
  return KFP_OK;
}

kfp_status kfp_reload_tune_cache(void) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  delete g_tune;
  g_tune = nullptr;
  return KFP_OK;
}

kfp_status kfp_set_kernel_timing(int32_t on) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  g_ktime = on != 0;
  return KFP_OK;
}

kfp_status kfp_set_ordering(int32_t order) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  if (order != 0 && order != 1) return fail(KFP_EINVAL, "order must be 0 or 1");
  g_order = order;
  return KFP_OK;
}

kfp_status kfp_set_scheme(int32_t scheme) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  if (scheme != KFP_SCHEME_FD && scheme != KFP_SCHEME_FEM)
    return fail(KFP_EINVAL, "scheme must be 0 (finite differences) or 1 (finite elements)");
  g_scheme = scheme;
  return KFP_OK;
}

kfp_status kfp_set_pipeline(int32_t inflight) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  if (inflight < -1 || inflight == 1) return fail(KFP_EINVAL, "inflight must be -1, 0 or >= 2");
  g_pipe = inflight;
  return KFP_OK;
}

kfp_status kfp_set_launch_tiles(int32_t waves, int32_t groups, int32_t seg_max, int32_t steps,
                                int32_t tiles) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  if (waves == 0) {
    g_forced = Config{};
    return KFP_OK;
  }
  const Config c{waves, seg_max, steps, groups, tiles};
  if (!config_supported(c))
    return fail(KFP_EINVAL,
                "configuration waves=%d groups=%d seg_max=%d steps=%d tiles=%d is not compiled",
                waves, groups, seg_max, steps, tiles);
  g_forced = c;
  return KFP_OK;
}

kfp_status kfp_set_launch(int32_t waves, int32_t groups, int32_t seg_max, int32_t steps) {
  return kfp_set_launch_tiles(waves, groups, seg_max, steps, 0);
}

kfp_status kfp_set_config(int32_t waves, int32_t seg_max, int32_t steps) {
  return kfp_set_launch(waves, 1, seg_max, steps);
}

kfp_status kfp_get_launch_tiles(const kfp_grid *g, int32_t J, int32_t overlap, int32_t tr,
                                int32_t *waves_out, int32_t *groups_out, int32_t *seg_max_out,
                                int32_t *steps_out, int32_t *tiles_out) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  Geo geo;
  kfp_status st = make_geo(g, J, overlap, tr, 1.0, geo, g_scheme);
  if (st) return st;
  const Config c = choose_config(geo, J > 1 ? g_order : 0);
  if (waves_out) *waves_out = c.waves;
  if (groups_out) *groups_out = c.groups;
  if (seg_max_out) *seg_max_out = c.seg;
  if (steps_out) *steps_out = c.steps;
  if (tiles_out) *tiles_out = c.tiles;
  return KFP_OK;
}

kfp_status kfp_get_launch(const kfp_grid *g, int32_t J, int32_t overlap, int32_t tr,
                          int32_t *waves_out, int32_t *groups_out, int32_t *seg_max_out,
                          int32_t *steps_out) {
  return kfp_get_launch_tiles(g, J, overlap, tr, waves_out, groups_out, seg_max_out, steps_out,
                              nullptr);
}

kfp_status kfp_get_config(const kfp_grid *g, int32_t J, int32_t overlap, int32_t tr,
                          int32_t *waves_out, int32_t *seg_max_out, int32_t *steps_out) {
  return kfp_get_launch(g, J, overlap, tr, waves_out, nullptr, seg_max_out, steps_out);
}

kfp_status kfp_subdomain_rows(const kfp_grid *g, int32_t J, int32_t overlap, int32_t tr,
                              int64_t *rows_out) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  Geo geo;
  kfp_status st = make_geo(g, J, overlap, tr, 1.0, geo, g_scheme);
  if (st) return st;
  if (!rows_out) return fail(KFP_EINVAL, "rows_out is NULL");
  *rows_out = geo.rows;
  return KFP_OK;
}

kfp_status kfp_bw_probe(const void *src, void *dst, int64_t bytes, void *stream) {
  g_err.clear();
  if (!src || !dst || bytes < 0 || bytes % 16) return fail(KFP_EINVAL, "bad probe arguments");
  HIP_TRY(launch_bw_probe(src, dst, (size_t)bytes, (hipStream_t)stream));
  return KFP_OK;
}

kfp_status kfp_tile_probe(const double *U, const double *F, double *V, int64_t rows, int32_t nx,
                          int32_t waves, int32_t rows_per_wave, void *stream) {
  g_err.clear();
  if (!U || !F || !V || rows < 0 || nx < 1)
    return fail(KFP_EINVAL, "bad tile probe arguments");
  if (!tile_probe_supported(waves, rows_per_wave))
    return fail(KFP_EINVAL, "tile probe shape (%d, %d) is not built", (int)waves,
                (int)rows_per_wave);
  if ((rows + (int64_t)waves * rows_per_wave - 1) / ((int64_t)waves * rows_per_wave) > 65535)
    return fail(KFP_EINVAL, "tile probe: too many rows");
  HIP_TRY(launch_tile_probe(U, F, V, (long)rows, nx, waves, rows_per_wave, (hipStream_t)stream));
  return KFP_OK;
}

void kfp_release_workspace(void) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_plans.clear();
  g_plan_lru.clear();
}

const char *kfp_last_error(void) { return g_err.c_str(); }

kfp_status kfp_debug_tables(const kfp_grid *g, int32_t J, int32_t overlap, int32_t tr, double p,
                            int32_t waves, int32_t *sub_info, double *rows, int32_t *segs,
                            double *reds, double *mat) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_err.clear();
  Geo geo;
  kfp_status st = make_geo(g, J, overlap, tr, p, geo, g_scheme);
  if (st) return st;
  if (waves < 1 || waves > 16) return fail(KFP_EINVAL, "waves must be in 1..16");
  if (!sub_info || !rows || !segs || !reds || !mat) return fail(KFP_EINVAL, "NULL output");
  HostTables h;
  add_instance(geo, p, p, waves, 0, h);
  const double hv = 2.0 / geo.nv, dt = geo.T / geo.nt, r = dt / (hv * hv);
  for (int j = 0; j < J; ++j) {
    const SubDev &d = h.subs[j];
    int32_t *o = sub_info + 8 * j;
    o[0] = d.n;
    o[1] = d.row_off;
    o[2] = d.g_lo;
    o[3] = d.P;
    o[4] = d.lo_kind;
    o[5] = d.hi_kind;
    o[6] = d.tab;
    o[7] = d.seg;
    std::vector<double> lo, di, up;
    any_row_matrix(geo.sub[j], geo.scheme, r, p, p, hv, lo, di, up);
    for (int k = 0; k < d.n; ++k) {
      mat[3 * (d.tab + k) + 0] = lo[k];
      mat[3 * (d.tab + k) + 1] = di[k];
      mat[3 * (d.tab + k) + 2] = up[k];
    }
  }
  for (size_t i = 0; i < h.rows.size(); ++i) {
    const RowCoef &c = h.rows[i];
    double *o = rows + 6 * i;
    o[0] = c.nu;
    o[1] = c.fa;
    o[2] = c.fb;
    o[3] = c.bc;
    o[4] = c.sl;
    o[5] = c.sr;
  }
  for (size_t i = 0; i < h.segs.size(); ++i) segs[i] = h.segs[i];
  for (size_t i = 0; i < h.reds.size(); ++i) {
    const RedCoef &c = h.reds[i];
    double *o = reds + 5 * i;
    o[0] = c.ra;
    o[1] = c.rc;
    o[2] = c.g1;
    o[3] = c.g2;
    o[4] = c.h;
  }
  return KFP_OK;
}

}  // extern "C"
