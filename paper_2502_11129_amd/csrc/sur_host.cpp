// C ABI of the learned fitness surrogate (include/sur.h): validation,
// workspace layout and the order of kernel launches of each call.
#include "sur.h"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <algorithm>
#include <vector>

#include "sur_launch.h"

using namespace surk;

namespace {

constexpr int64_t kPredictChunk = 65536;  // rows per forward pass of sur_predict
constexpr int kMaxSplitK = 16;            // layers of a weight-gradient product
constexpr int kSplitKRows = 256;          // batch rows per layer at least

struct Work {
  float *p, *m, *v, *g;
  uint16_t *wt1, *wt2, *wt3, *wb2, *wb3;
  float* w4f;
  // one batch (max(max_batch, kPredictChunk) rows for the hidden activations)
  float *z1, *z2, *z3;
  uint16_t *h1, *h2, *h3, *dza, *dzb;
  float *y, *r, *dy, *partial, *loss;
  // split-K layers of the weight-gradient products
  float* splitk;
  // top-k scratch
  uint32_t *hist, *state, *blocks;
  int64_t blocks_cap;
  double* stats;
};

}  // namespace

struct sur_handle {
  sur_config cfg{};
  int64_t rows = 0;  // activation rows held by the workspace
  size_t bytes = 0;
  char* base = nullptr;
  Work w{};
  int64_t t = 0;
  bool bound = false;
  bool sticky = false;
  std::string err;
};

static std::string g_create_err;

static int fail(sur_handle* h, int code, const std::string& msg) {
  if (h) {
    h->err = msg;
    if (code == SUR_E_DEVICE) h->sticky = true;
  } else {
    g_create_err = msg;
  }
  return code;
}

static int hip_fail(sur_handle* h, hipError_t e, const char* what) {
  return fail(h, SUR_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define SUR_HIP(h, call, what)               \
  do {                                       \
    hipError_t e_ = (call);                  \
    if (e_ != hipSuccess) return hip_fail(h, e_, what); \
  } while (0)

static int ready(sur_handle* h) {
  if (!h) return SUR_E_INVALID;
  if (h->sticky) return fail(h, SUR_E_DEVICE, "handle has a sticky device error: " + h->err);
  if (!h->bound) return fail(h, SUR_E_STATE, "sur_bind has not been called");
  return SUR_OK;
}

// Workspace layout: 256-byte aligned regions in a fixed order.
static size_t layout(const sur_handle* h, char* base, Work* w) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) & ~size_t(255);
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const int64_t R = h->rows;
  const int64_t nblk_cap = (int64_t(1) << 31) / kTopkBlock + 1;
  Work x{};
  x.p = (float*)take(sizeof(float) * kNParams);
  x.m = (float*)take(sizeof(float) * kNParams);
  x.v = (float*)take(sizeof(float) * kNParams);
  x.g = (float*)take(sizeof(float) * kNParams);
  x.wt1 = (uint16_t*)take(2 * kFeat * kHid);
  x.wt2 = (uint16_t*)take(2 * kHid * kHid);
  x.wt3 = (uint16_t*)take(2 * kHid * kHid);
  x.wb2 = (uint16_t*)take(2 * kHid * kHid);
  x.wb3 = (uint16_t*)take(2 * kHid * kHid);
  x.w4f = (float*)take(sizeof(float) * kHid);
  x.z1 = (float*)take(sizeof(float) * R * kHid);
  x.z2 = (float*)take(sizeof(float) * R * kHid);
  x.z3 = (float*)take(sizeof(float) * R * kHid);
  x.h1 = (uint16_t*)take(2 * R * kHid);
  x.h2 = (uint16_t*)take(2 * R * kHid);
  x.h3 = (uint16_t*)take(2 * R * kHid);
  x.dza = (uint16_t*)take(2 * R * kHid);
  x.dzb = (uint16_t*)take(2 * R * kHid);
  x.y = (float*)take(sizeof(float) * R);
  x.r = (float*)take(sizeof(float) * R);
  x.dy = (float*)take(sizeof(float) * R);
  x.partial = (float*)take(sizeof(float) * ((R + kHeadChunk - 1) / kHeadChunk) * (kHid + 2));
  x.loss = (float*)take(sizeof(float) * 4);
  x.splitk = (float*)take(sizeof(float) * kMaxSplitK * (kHid + 1) * kHid);
  x.hist = (uint32_t*)take(sizeof(uint32_t) * 256);
  x.state = (uint32_t*)take(sizeof(uint32_t) * 4);
  x.blocks = (uint32_t*)take(sizeof(uint32_t) * 3 * nblk_cap);
  x.blocks_cap = nblk_cap;
  x.stats = (double*)take(sizeof(double) * 2);
  if (w) *w = x;
  return (off + 255) & ~size_t(255);
}

extern "C" {

int sur_create(const sur_config* cfg, sur_handle** out) {
  if (!out) return fail(nullptr, SUR_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(nullptr, SUR_E_INVALID, "cfg is NULL");
  if (cfg->max_batch < 1 || cfg->max_batch > 65536)
    return fail(nullptr, SUR_E_INVALID, "max_batch must be in [1, 65536]");
  if (!(cfg->lr > 0.0) || !(cfg->beta1 >= 0.0 && cfg->beta1 < 1.0) || !(cfg->beta2 >= 0.0 && cfg->beta2 < 1.0) ||
      !(cfg->eps > 0.0))
    return fail(nullptr, SUR_E_INVALID, "Adam settings out of range (lr > 0, 0 <= beta < 1, eps > 0)");
  sur_handle* h = new sur_handle();
  h->cfg = *cfg;
  h->rows = cfg->max_batch > kPredictChunk ? cfg->max_batch : kPredictChunk;
  h->bytes = layout(h, nullptr, nullptr);
  *out = h;
  return SUR_OK;
}

int sur_workspace_bytes(const sur_handle* h, size_t* bytes) {
  if (!h || !bytes) return SUR_E_INVALID;
  *bytes = h->bytes;
  return SUR_OK;
}

int sur_bind(sur_handle* h, void* ws, size_t bytes, const float* init, void* stream) {
  if (!h) return SUR_E_INVALID;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return fail(h, SUR_E_INVALID, "workspace NULL or not 256-byte aligned");
  if (bytes < h->bytes) return fail(h, SUR_E_NOMEM, "workspace smaller than sur_workspace_bytes()");
  if (!init) return fail(h, SUR_E_INVALID, "init_params is NULL");
  hipStream_t s = (hipStream_t)stream;
  h->base = (char*)ws;
  layout(h, h->base, &h->w);
  const size_t pb = sizeof(float) * kNParams;
  SUR_HIP(h, hipMemcpyAsync(h->w.p, init, pb, hipMemcpyHostToDevice, s), "upload parameters");
  std::vector<float> zero(kNParams, 0.f);
  SUR_HIP(h, hipMemcpyAsync(h->w.m, zero.data(), pb, hipMemcpyHostToDevice, s), "zero m");
  SUR_HIP(h, hipMemcpyAsync(h->w.v, zero.data(), pb, hipMemcpyHostToDevice, s), "zero v");
  SUR_HIP(h, hipMemcpyAsync(h->w.g, zero.data(), pb, hipMemcpyHostToDevice, s), "zero grad");
  const Work& w = h->w;
  SUR_HIP(h, refresh_copies(w.p, w.wt1, w.wt2, w.wt3, w.wb2, w.wb3, w.w4f, s), "refresh copies");
  SUR_HIP(h, hipStreamSynchronize(s), "bind sync");
  h->t = 0;
  h->bound = true;
  return SUR_OK;
}

int sur_features(sur_handle* h, int64_t n, const int32_t* nh, const int8_t* parent, const int8_t* face,
                 const int8_t* axis, const float* cpg, uint16_t* X, void* stream) {
  int rc = ready(h);
  if (rc) return rc;
  if (n < 0) return fail(h, SUR_E_INVALID, "n < 0");
  if (n == 0) return SUR_OK;
  if (!nh || !parent || !face || !axis || !cpg || !X) return fail(h, SUR_E_INVALID, "NULL array");
  if ((reinterpret_cast<uintptr_t>(X) & 15) || (reinterpret_cast<uintptr_t>(cpg) & 3))
    return fail(h, SUR_E_INVALID, "X must be 16-byte aligned and cpg 4-byte aligned");
  SUR_HIP(h, features(n, nh, parent, face, axis, cpg, X, (hipStream_t)stream), "features");
  return SUR_OK;
}

// Forward pass over rows [0, n) of a chunk: layers into the workspace, then the head.
static int forward_rows(sur_handle* h, int n, const uint16_t* X, int64_t x_rows, const int32_t* idx, bool keep_z,
                        hipStream_t s) {
  const Work& w = h->w;
  GemmArgs a{};
  a.N = kHid;
  a.onesRow = -1;
  a.ldc = kHid;
  // layer 1: X[idx] (n x 128) * W1
  a.M = n;
  a.K = kFeat;
  a.A = X;
  a.lda = kFeat;
  a.gatherA = idx;
  a.rowsA = x_rows;
  a.B = w.wt1;
  a.ldb = kFeat;
  a.bias = w.p + kOffB1;
  a.zout = keep_z ? w.z1 : nullptr;
  a.hout = w.h1;
  SUR_HIP(h, gemm(kRowK, kRowK, kEpiGelu, a, s), "layer 1");
  // layers 2, 3
  a.K = kHid;
  a.lda = kHid;
  a.gatherA = nullptr;
  a.ldb = kHid;
  a.A = w.h1;
  a.B = w.wt2;
  a.bias = w.p + kOffB2;
  a.zout = keep_z ? w.z2 : nullptr;
  a.hout = w.h2;
  SUR_HIP(h, gemm(kRowK, kRowK, kEpiGelu, a, s), "layer 2");
  a.A = w.h2;
  a.B = w.wt3;
  a.bias = w.p + kOffB3;
  a.zout = keep_z ? w.z3 : nullptr;
  a.hout = w.h3;
  SUR_HIP(h, gemm(kRowK, kRowK, kEpiGelu, a, s), "layer 3");
  return SUR_OK;
}

int sur_predict(sur_handle* h, int64_t n, const uint16_t* X, int64_t x_rows, const int32_t* idx, float* y,
                void* stream) {
  int rc = ready(h);
  if (rc) return rc;
  if (n < 0) return fail(h, SUR_E_INVALID, "n < 0");
  if (n == 0) return SUR_OK;
  if (!X || !y) return fail(h, SUR_E_INVALID, "NULL array");
  if (reinterpret_cast<uintptr_t>(X) & 15) return fail(h, SUR_E_INVALID, "X must be 16-byte aligned");
  if (!idx && x_rows < n) return fail(h, SUR_E_INVALID, "x_rows < n without idx");
  hipStream_t s = (hipStream_t)stream;
  const Work& w = h->w;
  for (int64_t r0 = 0; r0 < n; r0 += h->rows) {
    const int rows = (int)((n - r0) < h->rows ? (n - r0) : h->rows);
    // without idx, the chunk's rows start at X + r0 rows
    const uint16_t* Xc = idx ? X : X + r0 * kFeat;
    const int32_t* ic = idx ? idx + r0 : nullptr;
    rc = forward_rows(h, rows, Xc, x_rows, ic, false, s);
    if (rc) return rc;
    SUR_HIP(h, head(rows, w.h3, w.w4f, w.p + kOffB4, y + r0, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, s),
            "head");
  }
  return SUR_OK;
}

int sur_adam_step(sur_handle* h, const float* grad, void* stream) {
  int rc = ready(h);
  if (rc) return rc;
  if (!grad) return fail(h, SUR_E_INVALID, "grad is NULL");
  const Work& w = h->w;
  h->t += 1;
  SUR_HIP(h, adam(w.p, w.m, w.v, grad, h->t, h->cfg.lr, h->cfg.beta1, h->cfg.beta2, h->cfg.eps, w.wt1, w.wt2, w.wt3,
                  w.wb2, w.wb3, w.w4f, (hipStream_t)stream),
          "adam");
  return SUR_OK;
}

static int train_step(sur_handle* h, int B, const uint16_t* X, int64_t x_rows, const float* target,
                      const int32_t* idx, float* loss, hipStream_t s) {
  const Work& w = h->w;
  int rc = forward_rows(h, B, X, x_rows, idx, true, s);
  if (rc) return rc;
  // head: y, dy, dz3; then grad W4, b4 and the loss
  SUR_HIP(h, head(B, w.h3, w.w4f, w.p + kOffB4, w.y, target, idx, x_rows, w.z3, w.r, w.dy, w.dza, s), "head");
  SUR_HIP(h, head_reduce(B, w.h3, w.dy, w.r, w.partial, w.g + kOffW4, w.g + kOffB4, loss ? loss : w.loss, s),
          "head reduce");
  GemmArgs a{};
  // grad [W3; b3] = [h2 | 1]^T dz3   (M = 257 rows: the last one sums dz3 for the bias)
  a.M = kHid + 1;
  a.N = kHid;
  a.K = B;
  a.A = w.h2;
  a.lda = kHid;
  a.onesRow = kHid;
  a.B = w.dza;
  a.ldb = kHid;
  a.fout = w.g + kOffW3;
  a.ldc = kHid;
  // the batch (the reduction) is long and M x N small: split it over layers
  a.ksplit = std::min(kMaxSplitK, std::max(1, B / kSplitKRows));
  a.partial = w.splitk;
  SUR_HIP(h, gemm(kRowM, kRowM, kEpiF32, a, s), "grad W3");
  // dz2 = bf16((dz3 W3^T) * GELU'(z2))
  GemmArgs d{};
  d.M = B;
  d.N = kHid;
  d.K = kHid;
  d.A = w.dza;
  d.lda = kHid;
  d.onesRow = -1;
  d.B = w.wb3;
  d.ldb = kHid;
  d.zin = w.z2;
  d.ldz = kHid;
  d.hout = w.dzb;
  d.ldc = kHid;
  SUR_HIP(h, gemm(kRowK, kRowK, kEpiGeluGrad, d, s), "dz2");
  a.A = w.h1;
  a.B = w.dzb;
  a.fout = w.g + kOffW2;
  SUR_HIP(h, gemm(kRowM, kRowM, kEpiF32, a, s), "grad W2");
  d.A = w.dzb;
  d.B = w.wb2;
  d.zin = w.z1;
  d.hout = w.dza;
  SUR_HIP(h, gemm(kRowK, kRowK, kEpiGeluGrad, d, s), "dz1");
  // grad [W1; b1] = [X[idx] | 1]^T dz1
  a.M = kFeat + 1;
  a.A = X;
  a.lda = kFeat;
  a.gatherA = idx;
  a.rowsA = x_rows;
  a.onesRow = kFeat;
  a.B = w.dza;
  a.fout = w.g + kOffW1;
  SUR_HIP(h, gemm(kRowM, kRowM, kEpiF32, a, s), "grad W1");
  h->t += 1;
  SUR_HIP(h, adam(w.p, w.m, w.v, w.g, h->t, h->cfg.lr, h->cfg.beta1, h->cfg.beta2, h->cfg.eps, w.wt1, w.wt2, w.wt3,
                  w.wb2, w.wb3, w.w4f, s),
          "adam");
  return SUR_OK;
}

int sur_train_step(sur_handle* h, int32_t batch, const uint16_t* X, int64_t x_rows, const float* target,
                   const int32_t* idx, float* loss, void* stream) {
  int rc = ready(h);
  if (rc) return rc;
  if (batch < 1 || batch > h->cfg.max_batch) return fail(h, SUR_E_INVALID, "batch out of [1, max_batch]");
  if (!X || !target || !idx) return fail(h, SUR_E_INVALID, "NULL array");
  if (reinterpret_cast<uintptr_t>(X) & 15) return fail(h, SUR_E_INVALID, "X must be 16-byte aligned");
  return train_step(h, batch, X, x_rows, target, idx, loss, (hipStream_t)stream);
}

int sur_train_epoch(sur_handle* h, int64_t n, const uint16_t* X, int64_t x_rows, const float* target,
                    const int32_t* perm, int32_t batch, float* losses, void* stream) {
  int rc = ready(h);
  if (rc) return rc;
  if (n < 0) return fail(h, SUR_E_INVALID, "n < 0");
  if (batch < 1 || batch > h->cfg.max_batch) return fail(h, SUR_E_INVALID, "batch out of [1, max_batch]");
  if (n == 0) return SUR_OK;
  if (!X || !target || !perm) return fail(h, SUR_E_INVALID, "NULL array");
  if (reinterpret_cast<uintptr_t>(X) & 15) return fail(h, SUR_E_INVALID, "X must be 16-byte aligned");
  int64_t bi = 0;
  for (int64_t r0 = 0; r0 < n; r0 += batch, ++bi) {
    const int B = (int)((n - r0) < batch ? (n - r0) : batch);
    rc = train_step(h, B, X, x_rows, target, perm + r0, losses ? losses + bi : nullptr, (hipStream_t)stream);
    if (rc) return rc;
  }
  return SUR_OK;
}

int sur_get_grad(const sur_handle* hc, float* out, int where, void* stream) {
  sur_handle* h = const_cast<sur_handle*>(hc);
  int rc = ready(h);
  if (rc) return rc;
  if (!out) return fail(h, SUR_E_INVALID, "out is NULL");
  hipStream_t s = (hipStream_t)stream;
  const size_t pb = sizeof(float) * kNParams;
  if (where == 1) {
    SUR_HIP(h, hipMemcpyAsync(out, h->w.g, pb, hipMemcpyDeviceToDevice, s), "grad copy");
    return SUR_OK;
  }
  if (where != 0) return fail(h, SUR_E_INVALID, "where must be 0 (host) or 1 (device)");
  SUR_HIP(h, hipMemcpyAsync(out, h->w.g, pb, hipMemcpyDeviceToHost, s), "grad download");
  SUR_HIP(h, hipStreamSynchronize(s), "grad sync");
  return SUR_OK;
}

int sur_get_state(const sur_handle* hc, float* params, float* m, float* v, int64_t* t, void* stream) {
  sur_handle* h = const_cast<sur_handle*>(hc);
  int rc = ready(h);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const size_t pb = sizeof(float) * kNParams;
  if (params) SUR_HIP(h, hipMemcpyAsync(params, h->w.p, pb, hipMemcpyDeviceToHost, s), "params download");
  if (m) SUR_HIP(h, hipMemcpyAsync(m, h->w.m, pb, hipMemcpyDeviceToHost, s), "m download");
  if (v) SUR_HIP(h, hipMemcpyAsync(v, h->w.v, pb, hipMemcpyDeviceToHost, s), "v download");
  SUR_HIP(h, hipStreamSynchronize(s), "state sync");
  if (t) *t = h->t;
  return SUR_OK;
}

int sur_set_state(sur_handle* h, const float* params, const float* m, const float* v, int64_t t, void* stream) {
  int rc = ready(h);
  if (rc) return rc;
  if (t < 0) return fail(h, SUR_E_INVALID, "t < 0");
  hipStream_t s = (hipStream_t)stream;
  const size_t pb = sizeof(float) * kNParams;
  if (params) SUR_HIP(h, hipMemcpyAsync(h->w.p, params, pb, hipMemcpyHostToDevice, s), "params upload");
  if (m) SUR_HIP(h, hipMemcpyAsync(h->w.m, m, pb, hipMemcpyHostToDevice, s), "m upload");
  if (v) SUR_HIP(h, hipMemcpyAsync(h->w.v, v, pb, hipMemcpyHostToDevice, s), "v upload");
  const Work& w = h->w;
  SUR_HIP(h, refresh_copies(w.p, w.wt1, w.wt2, w.wt3, w.wb2, w.wb3, w.w4f, s), "refresh copies");
  SUR_HIP(h, hipStreamSynchronize(s), "state sync");
  h->t = t;
  return SUR_OK;
}

int sur_topk(sur_handle* h, int64_t n, const float* scores, int64_t k, int32_t* out, void* stream) {
  int rc = ready(h);
  if (rc) return rc;
  if (n < 0 || k < 0 || k > n) return fail(h, SUR_E_INVALID, "need 0 <= k <= n");
  if (n > 0x7fffffffLL) return fail(h, SUR_E_INVALID, "n must fit int32 indices");
  if (k == 0) return SUR_OK;
  if (!scores || !out) return fail(h, SUR_E_INVALID, "NULL array");
  TopkScratch ws{h->w.hist, h->w.state, h->w.blocks};
  SUR_HIP(h, topk(n, scores, k, out, ws, (hipStream_t)stream), "topk");
  return SUR_OK;
}

int sur_topk_noalloc(int64_t n, const float* scores, int64_t k, int32_t* out, void* stream, char* err,
                     size_t err_len) {
  auto fail_msg = [&](int code, const char* msg) {
    if (err && err_len) std::snprintf(err, err_len, "%s", msg);
    return code;
  };
  if (err && err_len) err[0] = '\0';
  static_assert(SUR_TOPK_NOALLOC_MAX == kTopkStaticMax, "header and scratch size agree");
  if (n < 0 || k < 0 || k > n) return fail_msg(SUR_E_INVALID, "need 0 <= k <= n");
  if (n > SUR_TOPK_NOALLOC_MAX)
    return fail_msg(SUR_E_INVALID, "n exceeds SUR_TOPK_NOALLOC_MAX (16777216 scores), the size of the static scratch");
  if (k == 0) return SUR_OK;
  if (!scores || !out) return fail_msg(SUR_E_INVALID, "NULL array");
  const hipError_t e = topk_noalloc(n, scores, k, out, (hipStream_t)stream);
  if (e != hipSuccess) {
    char buf[256];
    std::snprintf(buf, sizeof(buf), "topk_noalloc: %s", hipGetErrorString(e));
    return fail_msg(SUR_E_DEVICE, buf);
  }
  return SUR_OK;
}

int sur_standardize(sur_handle* h, int64_t n, const float* y, float* z, double* stats, void* stream) {
  int rc = ready(h);
  if (rc) return rc;
  if (n < 1) return fail(h, SUR_E_INVALID, "n < 1");
  if (!y || !z) return fail(h, SUR_E_INVALID, "NULL array");
  hipStream_t s = (hipStream_t)stream;
  SUR_HIP(h, standardize(n, y, z, h->w.stats, s), "standardize");
  if (stats) {
    SUR_HIP(h, hipMemcpyAsync(stats, h->w.stats, 2 * sizeof(double), hipMemcpyDeviceToHost, s), "stats download");
    SUR_HIP(h, hipStreamSynchronize(s), "stats sync");
  }
  return SUR_OK;
}

void sur_destroy(sur_handle* h) { delete h; }

const char* sur_last_error(const sur_handle* h) { return h ? h->err.c_str() : g_create_err.c_str(); }

}  // extern "C"
