// Host runtime of the learned initial-trace network: parameter storage
// (FP32 masters, BF16 copies, Adam moments), the forward pass, the backward
// pass, Adam, the fused training step, checkpoints, and the data helpers
// (casts, standardisation) around it.  C ABI in include/kfpswr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/kfpswr.h"
#include "mlp_internal.h"

namespace kfp {

// the library's one error slot (kfp_last_error), defined in swr_runtime.cpp
extern thread_local std::string g_err;
#define m_err g_err

static kfp_status mfail(kfp_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  m_err = buf;
  return st;
}

#define MHIP(expr)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return mfail(e_ == hipErrorOutOfMemory ? KFP_ENOMEM : KFP_EDEVICE, "%s: %s (%s:%d)", \
                   #expr, hipGetErrorString(e_), __FILE__, __LINE__);                      \
  } while (0)

template <class T>
static hipError_t dmalloc(T **p, size_t n) {
  *p = nullptr;
  return hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
}

struct Layer {
  int in = 0;
  long out = 0;
  float *W = nullptr, *b = nullptr;      // FP32 masters: W [out][in]
  __bf16 *Wb = nullptr;                  // BF16 copy [out][in]
  float *mW = nullptr, *vW = nullptr, *mb = nullptr, *vb = nullptr;
  float *gW = nullptr;                   // weight gradient (allocated by the first backward)
  float *gb = nullptr;                   // bias gradient
};

struct Acts {
  int cap = 0;
  __bf16 *Xb = nullptr;                        // input [B][in0]
  std::vector<float *> Z;                      // pre-activations [B][h] (hidden layers)
  std::vector<__bf16 *> Ab;                    // GELU outputs [B][h]
  __bf16 *db = nullptr;                        // output gradient BF16 [B][out]
  float *PB = nullptr;                         // its column sums per 64 rows [2*ceil(B/128)][out]
  float *dA = nullptr, *dZ32 = nullptr;        // hidden gradients [B][h]
  __bf16 *dZb = nullptr;
  float *P = nullptr;                          // split-K partials
  size_t P_n = 0;
  double *loss = nullptr;       // sum of squared residuals of the last forward with targets
  double *loss_part = nullptr;  // its per-wavefront partials [4 * output-layer tiles]
  size_t loss_part_n = 0;
};

}  // namespace kfp

struct kfp_mlp {
  int in = 0, hidden = 0, depth = 0;
  int skip = 0;  // the output layer also reads the network input (depth >= 1)
  long out = 0;
  long long step = 0;
  std::vector<kfp::Layer> L;
  kfp::Acts A;
};

namespace kfp {

static std::recursive_mutex m_mu;

static void free_acts(Acts &a) {
  auto f = [](void *p) {
    if (p) (void)hipFree(p);
  };
  f(a.Xb);
  for (auto p : a.Z) f(p);
  for (auto p : a.Ab) f(p);
  f(a.db);
  f(a.PB);
  f(a.dA);
  f(a.dZ32);
  f(a.dZb);
  f(a.P);
  f(a.loss);
  f(a.loss_part);
  a = Acts{};
}

static void free_mlp(kfp_mlp *m) {
  for (auto &l : m->L) {
    for (void *p : {(void *)l.W, (void *)l.b, (void *)l.Wb, (void *)l.mW, (void *)l.vW,
                    (void *)l.mb, (void *)l.vb, (void *)l.gW, (void *)l.gb})
      if (p) (void)hipFree(p);
  }
  free_acts(m->A);
}

// rows of the per-64-row column sums of the output gradient (two per
// 128-row tile of the batch)
static int pb_rows(int B) { return 2 * ((B + 127) / 128); }

static kfp_status ensure_acts(kfp_mlp *m, int B) {
  if (m->A.cap >= B) return KFP_OK;
  free_acts(m->A);
  Acts &a = m->A;
  const int nh = m->depth;
  MHIP(dmalloc(&a.Xb, (size_t)B * m->in));
  a.Z.assign(nh, nullptr);
  a.Ab.assign(nh, nullptr);
  for (int l = 0; l < nh; ++l) {
    // the last hidden activations sit beside a copy of the input with skip
    const size_t w = (size_t)m->hidden + ((m->skip && l == nh - 1) ? m->in : 0);
    MHIP(dmalloc(&a.Z[l], (size_t)B * m->hidden));
    MHIP(dmalloc(&a.Ab[l], (size_t)B * w));
  }
  MHIP(dmalloc(&a.db, (size_t)B * m->out));
  MHIP(dmalloc(&a.PB, (size_t)pb_rows(B) * m->out));
  const size_t hmax = std::max(m->hidden, m->in);
  MHIP(dmalloc(&a.dA, (size_t)B * hmax));
  MHIP(dmalloc(&a.dZ32, (size_t)B * hmax));
  MHIP(dmalloc(&a.dZb, (size_t)B * hmax));
  MHIP(dmalloc(&a.loss, 1));
  a.loss_part_n = (size_t)4 * ((B + 127) / 128) * ((m->out + 127) / 128);
  MHIP(dmalloc(&a.loss_part, a.loss_part_n));
  a.cap = B;
  return KFP_OK;
}

static int cu_count() {
  static int n = 0;
  if (!n) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        v > 0)
      n = v;
    else
      n = 256;
  }
  return n;
}

// C = A B^T with the split-K decision: long reductions over few output
// tiles (the input gradient of the wide layer) and short ones over very few
// tiles (the hidden layers) are cut into chunks whose partials a second
// pass sums in order and hands to the epilogue (store or Adam; the
// squared-error epilogue takes the whole K per tile).
static kfp_status gemm(kfp_mlp *m, GemmArgs g, hipStream_t s) {
  if (g.K % 8 || g.lda % 8 || g.ldb % 8 || (g.a_kmajor && g.M % 8) || (g.b_kmajor && g.N % 8))
    return mfail(KFP_EINVAL,
                 "GEMM needs K, lda, ldb multiples of 8, and M (N) too for a K-major A (B) "
                 "(M=%d N=%d K=%d)",
                 g.M, g.N, g.K);
  if (g.epi != EPI_STORE && (g.N % 8 || g.ldt % 4 || g.ldcb % 4 || g.ldw % 4))
    return mfail(KFP_EINVAL, "fused GEMM epilogue needs N a multiple of 8 (N=%d)", g.N);
  const long tiles = (long)((g.M + 127) / 128) * ((g.N + 127) / 128);
  int splits = 1;
  if (g.epi != EPI_MSE) {
    // long reductions: one round of resident workgroups (three per compute
    // unit at this kernel's register use)
    if (tiles < 512 && g.K >= 4096)
      splits = (int)std::min<long>((g.K + 2047) / 2048,
                                   std::max<long>(1, 3L * cu_count() / tiles));
    else if (tiles < 64 && g.K >= 128)
      splits = (int)std::min<long>(g.K / 64, std::max<long>(1, 256 / tiles));
  }
  int kchunk = (g.K + splits - 1) / splits;
  kchunk = (kchunk + 63) / 64 * 64;  // whole K steps of the kernel
  splits = (g.K + kchunk - 1) / kchunk;
  g.kchunk = kchunk;
  if (splits > 1) {
    const size_t need = (size_t)splits * g.M * g.N;
    if (m->A.P_n < need) {
      if (m->A.P) (void)hipFree(m->A.P);
      m->A.P = nullptr;
      m->A.P_n = 0;
      MHIP(dmalloc(&m->A.P, need));
      m->A.P_n = need;
    }
    g.P = m->A.P;
  } else {
    g.P = nullptr;
  }
  MHIP(launch_gemm(g, splits, s));
  return KFP_OK;
}

static GemmArgs gargs(int M, int N, int K, const __bf16 *A, long lda, const __bf16 *B, long ldb) {
  GemmArgs g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A;
  g.lda = lda;
  g.B = B;
  g.ldb = ldb;
  return g;
}

// Forward pass.  Without targets the output goes to Y (FP32 [B][out]).
// With targets T the output layer's epilogue forms the squared-error
// gradient instead: A.db = BF16(scale (y - T)), its column sums per 64 rows
// in A.PB, and sum (y - T)^2 in A.loss; y itself is never stored.
static kfp_status forward(kfp_mlp *m, int B, const float *X, float *Y, hipStream_t s,
                          const float *T = nullptr, float scale = 0.f) {
  kfp_status st = ensure_acts(m, B);
  if (st) return st;
  Acts &a = m->A;
  MHIP(launch_f32_to_bf16(X, a.Xb, (size_t)B * m->in, s));
  const __bf16 *cur = a.Xb;
  int cur_w = m->in;
  const int nl = (int)m->L.size();
  for (int l = 0; l < nl; ++l) {
    Layer &L = m->L[l];
    GemmArgs g = gargs(B, (int)L.out, L.in, cur, cur_w, L.Wb, L.in);
    g.bias = L.b;
    const bool concat = m->skip && l == nl - 2;
    const long wcat = concat ? L.out + m->in : L.out;
    if (l < nl - 1) {
      g.C = a.Z[l];
      g.ldc = L.out;
      g.Cb = a.Ab[l];
      g.ldcb = wcat;
      g.gelu = 1;
    } else if (T) {
      g.epi = EPI_MSE;
      g.T = T;
      g.ldt = L.out;
      g.scale = scale;
      g.loss_part = a.loss_part;
      g.PB = a.PB;
      g.Cb = a.db;
      g.ldcb = L.out;
    } else {
      g.C = Y;
      g.ldc = L.out;
    }
    if ((st = gemm(m, g, s))) return st;
    if (l == nl - 1 && T) {
      // the slots this batch's tiles wrote (the buffer is sized for the capacity)
      const size_t parts = (size_t)4 * ((B + 127) / 128) * ((L.out + 127) / 128);
      MHIP(launch_sum_f64(a.loss_part, parts, a.loss, s));
    }
    if (concat) MHIP(launch_f32_to_bf16_cols(X, B, m->in, a.Ab[l] + L.out, wcat, s));
    if (l < nl - 1) {
      cur = a.Ab[l];
      cur_w = (int)wcat;
    }
  }
  return KFP_OK;
}

struct AdamStep {
  float lr, b1, b2, eps, c1, c2;
};

static AdamStep adam_next(kfp_mlp *m, float lr) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  m->step += 1;
  return AdamStep{lr,  b1, b2, eps, 1.f - std::pow(b1, (float)m->step),
                  1.f - std::pow(b2, (float)m->step)};
}

// Gradients of the mean squared error at (X, T).  With opt == nullptr they
// are stored in gW / gb; otherwise each layer's weight-gradient product
// applies the Adam step in its epilogue and the gradient is never stored.
// Per layer, from the output back: bias gradient; input gradient (it reads
// the layer's weights before their update); weight gradient (and update);
// GELU derivative into the next layer's output gradient.
static kfp_status backprop(kfp_mlp *m, int B, const float *X, const float *T, double *loss_out,
                           const AdamStep *opt, hipStream_t s) {
  kfp_status st = ensure_acts(m, B);
  if (st) return st;
  const int nl = (int)m->L.size();
  if (!opt) {
    for (auto &L : m->L)
      if (!L.gW) MHIP(dmalloc(&L.gW, (size_t)L.out * L.in));
  }
  Acts &a = m->A;
  const size_t nout = (size_t)B * m->out;
  if ((st = forward(m, B, X, nullptr, s, T, 2.0f / (float)nout))) return st;
  const __bf16 *dbf = a.db;  // output gradient of layer l, [B][out_l]
  for (int l = nl - 1; l >= 0; --l) {
    Layer &L = m->L[l];
    const int outw = (int)L.out;
    if (l == nl - 1)
      MHIP(launch_colsum(a.PB, pb_rows(B), outw, L.gb, s));
    else
      MHIP(launch_colsum(a.dZ32, B, outw, L.gb, s));
    // input gradient dA[b][i] = sum_o d[b][o] W[o][i] over the hidden inputs
    // only (the input columns of a skip layer end there); W read K-major
    const int hin = (m->skip && l == nl - 1) ? m->hidden : L.in;
    if (l > 0) {
      GemmArgs gx = gargs(B, hin, outw, dbf, outw, L.Wb, L.in);
      gx.b_kmajor = 1;
      gx.C = a.dA;
      gx.ldc = hin;
      if ((st = gemm(m, gx, s))) return st;
    }
    // weight gradient dW[o][i] = sum_b d[b][o] act[b][i]: both operands
    // K-major with K = batch
    const __bf16 *act = (l == 0) ? a.Xb : a.Ab[l - 1];
    GemmArgs gw = gargs(outw, L.in, B, dbf, outw, act, L.in);
    gw.a_kmajor = 1;
    gw.b_kmajor = 1;
    if (opt) {
      gw.epi = EPI_ADAM;
      gw.W = L.W;
      gw.Mo = L.mW;
      gw.Vo = L.vW;
      gw.Wb = L.Wb;
      gw.ldw = L.in;
      gw.lr = opt->lr;
      gw.b1 = opt->b1;
      gw.b2 = opt->b2;
      gw.eps = opt->eps;
      gw.c1 = opt->c1;
      gw.c2 = opt->c2;
    } else {
      gw.C = L.gW;
      gw.ldc = L.in;
    }
    if ((st = gemm(m, gw, s))) return st;
    if (opt)
      MHIP(launch_adam(L.b, L.gb, L.mb, L.vb, nullptr, (size_t)L.out, opt->lr, opt->b1, opt->b2,
                       opt->eps, opt->c1, opt->c2, s));
    if (l == 0) break;
    MHIP(launch_gelu_back(a.dA, a.Z[l - 1], a.dZ32, a.dZb, (size_t)B * hin, s));
    dbf = a.dZb;
  }
  if (loss_out) {
    double h = 0.0;
    MHIP(hipMemcpyAsync(&h, a.loss, sizeof(double), hipMemcpyDeviceToHost, s));
    MHIP(hipStreamSynchronize(s));
    *loss_out = h / (double)nout;
  }
  return KFP_OK;
}

static kfp_status adam(kfp_mlp *m, float lr, hipStream_t s) {
  for (auto &L : m->L)
    if (!L.gW) return mfail(KFP_EINVAL, "adam: no stored gradients (kfp_mlp_backward first)");
  const AdamStep o = adam_next(m, lr);
  for (auto &L : m->L) {
    const size_t nw = (size_t)L.out * L.in;
    MHIP(launch_adam(L.W, L.gW, L.mW, L.vW, L.Wb, nw, o.lr, o.b1, o.b2, o.eps, o.c1, o.c2, s));
    MHIP(launch_adam(L.b, L.gb, L.mb, L.vb, nullptr, (size_t)L.out, o.lr, o.b1, o.b2, o.eps, o.c1,
                     o.c2, s));
  }
  return KFP_OK;
}

static kfp_status refresh_copies(kfp_mlp *m, hipStream_t s) {
  for (auto &L : m->L) {
    const size_t nw = (size_t)L.out * L.in;
    MHIP(launch_f32_to_bf16(L.W, L.Wb, nw, s));
  }
  return KFP_OK;
}

static kfp_status create(int in, int hidden, int depth, long out, int flags,
                         unsigned long long seed, bool init, kfp_mlp **res) {
  if (in < 8 || in % 8 || hidden < 8 || hidden % 8 || depth < 0 || depth > 16 || out < 1 ||
      out % 8)
    return mfail(KFP_EINVAL,
                 "network shape: in, hidden and out must be positive multiples of 8, depth 0..16");
  if (flags & ~KFP_MLP_SKIP) return mfail(KFP_EINVAL, "unknown network flags %d", flags);
  std::unique_ptr<kfp_mlp> m(new kfp_mlp());
  m->in = in;
  m->hidden = hidden;
  m->depth = depth;
  m->out = out;
  m->skip = (flags & KFP_MLP_SKIP) && depth >= 1;
  const int nl = depth + 1;
  m->L.resize(nl);
  for (int l = 0; l < nl; ++l) {
    Layer &L = m->L[l];
    L.in = (l == 0) ? in : hidden;
    if (m->skip && l == nl - 1) L.in += in;
    L.out = (l == nl - 1) ? out : hidden;
    const size_t nw = (size_t)L.out * L.in;
    auto bad = [&](hipError_t e) {
      if (e != hipSuccess) {
        free_mlp(m.get());
        return true;
      }
      return false;
    };
    if (bad(dmalloc(&L.W, nw)) || bad(dmalloc(&L.b, L.out)) || bad(dmalloc(&L.Wb, nw)) ||
        bad(dmalloc(&L.mW, nw)) || bad(dmalloc(&L.vW, nw)) || bad(dmalloc(&L.mb, L.out)) ||
        bad(dmalloc(&L.vb, L.out)) || bad(dmalloc(&L.gb, L.out)))
      return mfail(KFP_ENOMEM, "device allocation of the network failed");
    hipError_t e = hipSuccess;
    if (init) {
      e = launch_init_normal(L.W, nw, 1.0f / std::sqrt((float)L.in), seed * 131 + l, nullptr);
      if (e == hipSuccess) e = hipMemset(L.b, 0, sizeof(float) * L.out);
    }
    if (e == hipSuccess) e = hipMemset(L.mW, 0, sizeof(float) * nw);
    if (e == hipSuccess) e = hipMemset(L.vW, 0, sizeof(float) * nw);
    if (e == hipSuccess) e = hipMemset(L.mb, 0, sizeof(float) * L.out);
    if (e == hipSuccess) e = hipMemset(L.vb, 0, sizeof(float) * L.out);
    if (e != hipSuccess) {
      free_mlp(m.get());
      return mfail(KFP_EDEVICE, "network initialisation: %s", hipGetErrorString(e));
    }
  }
  if (init) {
    kfp_status st = refresh_copies(m.get(), nullptr);
    if (st) {
      free_mlp(m.get());
      return st;
    }
    if (hipDeviceSynchronize() != hipSuccess) {
      free_mlp(m.get());
      return mfail(KFP_EDEVICE, "network initialisation failed");
    }
  }
  *res = m.release();
  return KFP_OK;
}

}  // namespace kfp

using namespace kfp;

extern "C" {

kfp_status kfp_mlp_create(int32_t in, int32_t hidden, int32_t depth, int64_t out, uint64_t seed,
                          kfp_mlp **mlp) {
  std::lock_guard<std::recursive_mutex> lk(m_mu);
  m_err.clear();
  if (!mlp) return mfail(KFP_EINVAL, "mlp is NULL");
  return create(in, hidden, depth, (long)out, 0, seed, true, mlp);
}

kfp_status kfp_mlp_create_ex(int32_t in, int32_t hidden, int32_t depth, int64_t out,
                             int32_t flags, uint64_t seed, kfp_mlp **mlp) {
  std::lock_guard<std::recursive_mutex> lk(m_mu);
  m_err.clear();
  if (!mlp) return mfail(KFP_EINVAL, "mlp is NULL");
  return create(in, hidden, depth, (long)out, flags, seed, true, mlp);
}

void kfp_mlp_destroy(kfp_mlp *m) {
  std::lock_guard<std::recursive_mutex> lk(m_mu);
  if (!m) return;
  (void)hipDeviceSynchronize();
  free_mlp(m);
  delete m;
}

kfp_status kfp_mlp_forward(kfp_mlp *m, int32_t B, const float *X, float *Y, void *stream) {
  std::lock_guard<std::recursive_mutex> lk(m_mu);
  m_err.clear();
  if (!m || !X || !Y || B < 1) return mfail(KFP_EINVAL, "forward: bad arguments");
  return forward(m, B, X, Y, (hipStream_t)stream);
}

kfp_status kfp_mlp_backward(kfp_mlp *m, int32_t B, const float *X, const float *T, double *loss,
                            void *stream) {
  std::lock_guard<std::recursive_mutex> lk(m_mu);
  m_err.clear();
  if (!m || !X || !T || B < 8 || B % 8)
    return mfail(KFP_EINVAL, "backward: bad arguments (batch must be a multiple of 8)");
  return backprop(m, B, X, T, loss, nullptr, (hipStream_t)stream);
}

kfp_status kfp_mlp_adam(kfp_mlp *m, float lr, void *stream) {
  std::lock_guard<std::recursive_mutex> lk(m_mu);
  m_err.clear();
  if (!m || !(lr >= 0.f)) return mfail(KFP_EINVAL, "adam: bad arguments");
  return adam(m, lr, (hipStream_t)stream);
}

kfp_status kfp_mlp_train_step(kfp_mlp *m, int32_t B, const float *X, const float *T, float lr,
                              double *loss, void *stream) {
  std::lock_guard<std::recursive_mutex> lk(m_mu);
  m_err.clear();
  if (!m || !X || !T || B < 8 || B % 8 || !(lr >= 0.f))
    return mfail(KFP_EINVAL, "train_step: bad arguments (batch must be a multiple of 8)");
  const AdamStep o = adam_next(m, lr);
  return backprop(m, B, X, T, loss, &o, (hipStream_t)stream);
}

kfp_status kfp_mlp_layer_shape(const kfp_mlp *m, int32_t layer, int32_t *in, int64_t *out) {
  m_err.clear();
  if (!m || layer < 0 || layer >= (int)m->L.size()) return mfail(KFP_EINVAL, "bad layer");
  if (in) *in = m->L[layer].in;
  if (out) *out = m->L[layer].out;
  return KFP_OK;
}

kfp_status kfp_mlp_param(kfp_mlp *m, int32_t layer, int32_t which, int32_t set, float *buf,
                         void *stream) {
  std::lock_guard<std::recursive_mutex> lk(m_mu);
  m_err.clear();
  if (!m || !buf || layer < 0 || layer >= (int)m->L.size() || which < 0 || which > 3)
    return mfail(KFP_EINVAL, "param: bad arguments");
  Layer &L = m->L[layer];
  float *p = which == 0 ? L.W : which == 1 ? L.b : which == 2 ? L.gW : L.gb;
  if (!p) return mfail(KFP_EINVAL, "param: no stored weight gradient (kfp_mlp_backward first)");
  const size_t n = (which == 0 || which == 2) ? (size_t)L.out * L.in : (size_t)L.out;
  hipStream_t s = (hipStream_t)stream;
  if (set) {
    if (which > 1) return mfail(KFP_EINVAL, "param: gradients are read-only");
    MHIP(hipMemcpyAsync(p, buf, n * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (which == 0) MHIP(launch_f32_to_bf16(L.W, L.Wb, n, s));
  } else {
    MHIP(hipMemcpyAsync(buf, p, n * sizeof(float), hipMemcpyDeviceToDevice, s));
  }
  return KFP_OK;
}

kfp_status kfp_mlp_save(const kfp_mlp *m, const char *path) {
  std::lock_guard<std::recursive_mutex> lk(m_mu);
  m_err.clear();
  if (!m || !path) return mfail(KFP_EINVAL, "save: bad arguments");
  FILE *fp = fopen(path, "wb");
  if (!fp) return mfail(KFP_EINVAL, "save: cannot open %s", path);
  const char magic[8] = {'K', 'F', 'P', 'M', 'L', 'P', '2', 0};
  long long hdr[6] = {m->in, m->hidden, m->depth, m->out, m->step, m->skip ? KFP_MLP_SKIP : 0};
  bool ok = fwrite(magic, 1, 8, fp) == 8 && fwrite(hdr, sizeof hdr, 1, fp) == 1;
  std::vector<float> h;
  for (const auto &L : m->L) {
    const size_t nw = (size_t)L.out * L.in;
    for (auto pr : {std::make_pair(L.W, nw), std::make_pair(L.b, (size_t)L.out),
                    std::make_pair(L.mW, nw), std::make_pair(L.vW, nw),
                    std::make_pair(L.mb, (size_t)L.out), std::make_pair(L.vb, (size_t)L.out)}) {
      if (!ok) break;
      h.resize(pr.second);
      ok = hipMemcpy(h.data(), pr.first, pr.second * sizeof(float), hipMemcpyDeviceToHost) ==
               hipSuccess &&
           fwrite(h.data(), sizeof(float), pr.second, fp) == pr.second;
    }
  }
  fclose(fp);
  return ok ? KFP_OK : mfail(KFP_EDEVICE, "save: write failed");
}

kfp_status kfp_mlp_load(const char *path, kfp_mlp **res) {
  std::lock_guard<std::recursive_mutex> lk(m_mu);
  m_err.clear();
  if (!path || !res) return mfail(KFP_EINVAL, "load: bad arguments");
  FILE *fp = fopen(path, "rb");
  if (!fp) return mfail(KFP_EINVAL, "load: cannot open %s", path);
  char magic[8];
  long long hdr[6] = {0, 0, 0, 0, 0, 0};
  // version 1 headers have no flags word
  const bool ok_magic = fread(magic, 1, 8, fp) == 8 &&
                        (memcmp(magic, "KFPMLP1", 8) == 0 || memcmp(magic, "KFPMLP2", 8) == 0);
  const size_t nh = (ok_magic && magic[6] == '2') ? 6 : 5;
  if (!ok_magic || fread(hdr, sizeof(long long), nh, fp) != nh) {
    fclose(fp);
    return mfail(KFP_EINVAL, "load: %s is not a network checkpoint", path);
  }
  kfp_mlp *m = nullptr;
  kfp_status st =
      create((int)hdr[0], (int)hdr[1], (int)hdr[2], (long)hdr[3], (int)hdr[5], 0, false, &m);
  if (st) {
    fclose(fp);
    return st;
  }
  m->step = hdr[4];
  bool ok = true;
  std::vector<float> h;
  for (auto &L : m->L) {
    const size_t nw = (size_t)L.out * L.in;
    for (auto pr : {std::make_pair(L.W, nw), std::make_pair(L.b, (size_t)L.out),
                    std::make_pair(L.mW, nw), std::make_pair(L.vW, nw),
                    std::make_pair(L.mb, (size_t)L.out), std::make_pair(L.vb, (size_t)L.out)}) {
      if (!ok) break;
      h.resize(pr.second);
      ok = fread(h.data(), sizeof(float), pr.second, fp) == pr.second &&
           hipMemcpy(pr.first, h.data(), pr.second * sizeof(float), hipMemcpyHostToDevice) ==
               hipSuccess;
    }
  }
  fclose(fp);
  if (ok) ok = refresh_copies(m, nullptr) == KFP_OK && hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    kfp_mlp_destroy(m);
    return mfail(KFP_EINVAL, "load: truncated or unreadable checkpoint %s", path);
  }
  *res = m;
  return KFP_OK;
}

kfp_status kfp_cast_f64_f32(const double *src, const double *base, float *dst, int64_t n,
                            void *stream) {
  m_err.clear();
  if (n < 0) return mfail(KFP_EINVAL, "cast: negative size");
  if ((!src || !dst) && n > 0) return mfail(KFP_EINVAL, "cast: NULL pointer");
  MHIP(launch_f64_to_f32(src, base, dst, (size_t)n, (hipStream_t)stream));
  return KFP_OK;
}

kfp_status kfp_axpy_f32(const float *x, float *y, float alpha, int64_t n, void *stream) {
  m_err.clear();
  if (n < 0 || ((!x || !y) && n > 0)) return mfail(KFP_EINVAL, "axpy: bad arguments");
  MHIP(launch_axpy(x, y, alpha, (size_t)n, (hipStream_t)stream));
  return KFP_OK;
}

kfp_status kfp_mul_f32(const float *a, float *y, int64_t n, void *stream) {
  m_err.clear();
  if (n < 0 || ((!a || !y) && n > 0)) return mfail(KFP_EINVAL, "mul: bad arguments");
  MHIP(launch_mul(a, y, (size_t)n, (hipStream_t)stream));
  return KFP_OK;
}

kfp_status kfp_column_stats(const float *X, int32_t rows, int64_t cols, float floor_,
                            float *mean, float *stdv, void *stream) {
  m_err.clear();
  if (!X || !mean || !stdv || rows < 1 || cols < 1) return mfail(KFP_EINVAL, "stats: bad args");
  MHIP(launch_colstats(X, rows, (size_t)cols, mean, stdv, floor_, (hipStream_t)stream));
  return KFP_OK;
}

kfp_status kfp_standardize(float *X, int32_t rows, int64_t cols, const float *mean,
                           const float *stdv, void *stream) {
  m_err.clear();
  if (!X || !mean || !stdv || rows < 1 || cols < 1) return mfail(KFP_EINVAL, "standardize: bad args");
  MHIP(launch_standardize(X, (size_t)cols, (size_t)rows * cols, mean, stdv, (hipStream_t)stream));
  return KFP_OK;
}

kfp_status kfp_destandardize(const float *Y, int32_t rows, int64_t cols, const float *mean,
                             const float *stdv, const double *base, double *lam, void *stream) {
  m_err.clear();
  if (!Y || !mean || !stdv || !lam || rows < 1 || cols < 1)
    return mfail(KFP_EINVAL, "destandardize: bad args");
  MHIP(launch_destandardize(Y, mean, stdv, base, (size_t)cols, (size_t)rows * cols, lam,
                            (hipStream_t)stream));
  return KFP_OK;
}

static kfp_status trace_modes_arg(int32_t nx, int32_t nmodes, const int32_t *modes,
                                  TraceModes *md) {
  if (nx < 1 || nmodes < 1 || nmodes > 8 || !modes)
    return mfail(KFP_EINVAL, "trace modes: nx >= 1 and 1..8 frequencies are required");
  md->n = nmodes;
  for (int k = 0; k < 8; ++k) md->m[k] = 0;
  for (int k = 0; k < nmodes; ++k) {
    if (modes[k] < 1 || 2 * modes[k] >= nx)
      return mfail(KFP_EINVAL, "trace modes: frequency %d outside 1 .. nx/2 - 1 (nx = %d)",
                   modes[k], nx);
    md->m[k] = modes[k];
  }
  return KFP_OK;
}

kfp_status kfp_trace_modes(const double *lam, int64_t rows, int32_t nx, int32_t nmodes,
                           const int32_t *modes, double *coef, void *stream) {
  m_err.clear();
  TraceModes md;
  kfp_status st = trace_modes_arg(nx, nmodes, modes, &md);
  if (st) return st;
  if (rows < 0 || ((!lam || !coef) && rows > 0))
    return mfail(KFP_EINVAL, "trace modes: bad arguments");
  MHIP(launch_trace_modes(lam, (long)rows, nx, md, coef, (hipStream_t)stream));
  return KFP_OK;
}

kfp_status kfp_trace_synth(const double *coef, int32_t planes, int32_t ntc, int32_t nmodes,
                           const int32_t *modes, int32_t nt, int32_t nx, double *lam,
                           void *stream) {
  m_err.clear();
  TraceModes md;
  kfp_status st = trace_modes_arg(nx, nmodes, modes, &md);
  if (st) return st;
  if (planes < 1 || ntc < 1 || nt < 1 || !coef || !lam)
    return mfail(KFP_EINVAL, "trace synth: bad arguments");
  MHIP(launch_trace_synth(coef, planes, ntc, nt, nx, md, lam, (hipStream_t)stream));
  return KFP_OK;
}

}  // extern "C"
