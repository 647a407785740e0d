// Host side of the warm-start network entry points (include/nmf.h): parameter
// blob layout, batched forward, loss/gradient of one batch through the
// library's own backward kernels, Adam, and minibatch training.
#include <algorithm>
#include <cstring>
#include <random>
#include <vector>

#include "plan_impl.hpp"

using namespace plnmf;

namespace {

nmf_mlp_layout layout_of(int K, int H) {
  nmf_mlp_layout L{};
  const size_t nm = (size_t)H * K + H + (size_t)K * H + K;
  Carver c(nullptr);
  L.n_master = nm;
  c.take<float>(nm);
  L.master = 0;
  L.adam_m = align_up(c.off);
  c.take<float>(nm);
  L.adam_v = align_up(c.off);
  c.take<float>(nm);
  L.w1_bf16 = align_up(c.off);
  c.take<__bf16>((size_t)H * K);
  L.w2_bf16 = align_up(c.off);
  c.take<__bf16>((size_t)K * H);
  L.step = align_up(c.off);
  c.take<int64_t>(1);
  L.total = align_up(c.off);
  return L;
}

struct Params {
  float *W1, *b1, *W2, *b2;  // masters
  float *m, *v;
  __bf16 *W1b, *W2b;
  int64_t* step;
  size_t n;
};

Params view(void* blob, int K, int H) {
  const nmf_mlp_layout L = layout_of(K, H);
  char* b = (char*)blob;
  Params p;
  p.W1 = (float*)(b + L.master);
  p.b1 = p.W1 + (size_t)H * K;
  p.W2 = p.b1 + H;
  p.b2 = p.W2 + (size_t)K * H;
  p.m = (float*)(b + L.adam_m);
  p.v = (float*)(b + L.adam_v);
  p.W1b = (__bf16*)(b + L.w1_bf16);
  p.W2b = (__bf16*)(b + L.w2_bf16);
  p.step = (int64_t*)(b + L.step);
  p.n = L.n_master;
  return p;
}

struct Ws {
  __bf16* xb;
  float* z1;
  __bf16* gb;
  float* z2;
  float* yhat;
  __bf16* dz2b;
  float* dz2f;
  float* dz1f;
  __bf16* dz1b;
  float* partial;
  double* red;
  double* scal;
  double* csum;  // column-sum partials [kColSlices][max(K, H)]
  float* grads;
  float* xbat;
  float* ybat;
  int32_t* idx;
  size_t off;
};

int splits_for(int K, int H, int64_t B, int64_t* kps) {
  const int64_t m = std::max(K, H);
  (void)m;
  return gemm_pick_splits(K, H, B, kps);  // the weight-gradient products are K x H and H x K
}

Ws ws_layout(void* base, int K, int H, int64_t B) {
  Carver c(base);
  Ws w;
  w.xb = c.take<__bf16>((size_t)(B * K));
  w.z1 = c.take<float>((size_t)(B * H));
  w.gb = c.take<__bf16>((size_t)(B * H));
  w.z2 = c.take<float>((size_t)(B * K));
  w.yhat = c.take<float>((size_t)(B * K));
  w.dz2b = c.take<__bf16>((size_t)(B * K));
  w.dz2f = c.take<float>((size_t)(B * K));
  w.dz1f = c.take<float>((size_t)(B * H));
  w.dz1b = c.take<__bf16>((size_t)(B * H));
  int64_t kps;
  const int sp = splits_for(K, H, B, &kps);
  w.partial = c.take<float>((size_t)std::max(sp, 1) * K * H);
  w.red = c.take<double>(1024);
  w.scal = c.take<double>(8);
  w.csum = c.take<double>((size_t)kColSlices * std::max(K, H));
  w.grads = c.take<float>((size_t)H * K + H + (size_t)K * H + K);
  w.xbat = c.take<float>((size_t)(B * K));
  w.ybat = c.take<float>((size_t)(B * K));
  w.idx = c.take<int32_t>((size_t)B);
  c.take<char>(kAlign);
  w.off = c.off;
  return w;
}

// largest batch the workspace holds
int64_t batch_of(int K, int H, size_t bytes) {
  const size_t f0 = ws_layout(nullptr, K, H, 1).off;
  if (bytes < f0) return 0;
  int64_t lo = 1, hi = 1;
  while (ws_layout(nullptr, K, H, hi * 2).off <= bytes && hi < ((int64_t)1 << 40)) hi *= 2;
  hi *= 2;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) / 2;
    if (ws_layout(nullptr, K, H, mid).off <= bytes) lo = mid; else hi = mid;
  }
  return lo;
}

int check_dims(int K, int H) {
  if (K < 1 || K > NMF_MAX_K || H < 1 || H > 4096)
    return fail(NMF_E_SHAPE, "network dims K=%d hidden=%d out of range", K, H);
  return NMF_OK;
}

#define MLPCHECK(expr)                                                                    \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(NMF_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

hipError_t refresh(const Params& p, int K, int H, hipStream_t s) {
  hipError_t e = cast_bf16(p.W1, p.W1b, (int64_t)H * K, s);
  if (e != hipSuccess) return e;
  return cast_bf16(p.W2, p.W2b, (int64_t)K * H, s);
}

// forward of b rows of X (FP32) into yhat (FP32); leaves z1, gb, z2, xb in ws
int forward_rows(const Params& p, int K, int H, const float* X, float* yhat, int64_t b,
                 const Ws& w, hipStream_t s) {
  MLPCHECK(cast_bf16(X, w.xb, b * K, s));
  GemmArgs g{};
  g.A = w.xb;
  g.lda = K;
  g.B = p.W1b;  // B(k,j) = W1[j*K + k]
  g.ldb = K;
  g.M = b;
  g.N = H;
  g.Kd = K;
  g.C = w.z1;
  g.ldc = H;
  g.epi = EPI_BIAS_GELU;
  g.bias = p.b1;
  g.C2 = w.gb;
  g.splits = 1;
  MLPCHECK(gemm(Elem::BF16, false, true, g, s));
  GemmArgs g2{};
  g2.A = w.gb;
  g2.lda = H;
  g2.B = p.W2b;  // B(j,k) = W2[k*H + j]
  g2.ldb = H;
  g2.M = b;
  g2.N = K;
  g2.Kd = H;
  g2.C = w.z2;
  g2.ldc = K;
  g2.epi = EPI_BIAS_SOFTPLUS;
  g2.bias = p.b2;
  g2.C2 = yhat;
  g2.splits = 1;
  MLPCHECK(gemm(Elem::BF16, false, true, g2, s));
  return NMF_OK;
}

// loss (device scal[0], mean over b*K) and gradients into `grads`
int loss_grad_rows(const Params& p, int K, int H, const float* X, const float* Y, int64_t b,
                   float* grads, const Ws& w, hipStream_t s) {
  int rc = forward_rows(p, K, H, X, w.yhat, b, w, s);
  if (rc) return rc;
  const int64_t n = b * K;
  const int nb = reduce_blocks(n);
  MLPCHECK(mlp_out_grad(w.z2, w.yhat, Y, n, (float)(2.0 / (double)n), w.dz2b, w.dz2f, w.red, nb, s));
  MLPCHECK(finish_f64(w.red, nb, w.scal, s));
  float* gW1 = grads;
  float* gb1 = gW1 + (size_t)H * K;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + (size_t)K * H;
  // gW2 [K,H] = dz2^T g
  GemmArgs a{};
  a.A = w.dz2b;  // A(k, r) = dz2[r*K + k]
  a.lda = K;
  a.B = w.gb;    // B(r, j) = g[r*H + j]
  a.ldb = H;
  a.M = K;
  a.N = H;
  a.Kd = b;
  a.C = gW2;
  a.ldc = H;
  a.epi = EPI_STORE;
  a.splits = gemm_pick_splits(a.M, a.N, a.Kd, &a.k_per_split);
  a.partial = w.partial;
  MLPCHECK(gemm(Elem::BF16, true, false, a, s));
  MLPCHECK(col_sum(w.dz2f, b, K, gb2, w.csum, s));
  // dz1 [b,H] = (dz2 W2) * GELU'(z1)
  GemmArgs d{};
  d.A = w.dz2b;
  d.lda = K;
  d.B = p.W2b;  // B(k, j) = W2[k*H + j]
  d.ldb = H;
  d.M = b;
  d.N = H;
  d.Kd = K;
  d.C = w.dz1f;
  d.ldc = H;
  d.epi = EPI_GELU_GRAD;
  d.D = w.z1;
  d.ldd = H;
  d.C2 = w.dz1b;
  d.splits = 1;
  MLPCHECK(gemm(Elem::BF16, false, false, d, s));
  // gW1 [H,K] = dz1^T x
  GemmArgs c{};
  c.A = w.dz1b;  // A(j, r) = dz1[r*H + j]
  c.lda = H;
  c.B = w.xb;    // B(r, k) = x[r*K + k]
  c.ldb = K;
  c.M = H;
  c.N = K;
  c.Kd = b;
  c.C = gW1;
  c.ldc = K;
  c.epi = EPI_STORE;
  c.splits = gemm_pick_splits(c.M, c.N, c.Kd, &c.k_per_split);
  c.partial = w.partial;
  MLPCHECK(gemm(Elem::BF16, true, false, c, s));
  MLPCHECK(col_sum(w.dz1f, b, H, gb1, w.csum, s));
  return NMF_OK;
}

}  // namespace

namespace plnmf {
// used by fold-in: forward over N rows in workspace-sized batches
// Inference needs only the BF16 input and hidden activations (no FP32
// pre-activations, no backward buffers): about (K + H) * 2 bytes per row.
struct WsI {
  __bf16* xb;  // [B, K]
  __bf16* gb;  // [B, H]
  size_t off;
};
WsI ws_infer_layout(void* base, int K, int H, int64_t B) {
  Carver c(base);
  WsI w;
  w.xb = c.take<__bf16>((size_t)(B * K));
  w.gb = c.take<__bf16>((size_t)(B * H));
  c.take<char>(kAlign);
  w.off = c.off;
  return w;
}
int64_t batch_infer_of(int K, int H, size_t bytes) {
  const size_t per = ws_infer_layout(nullptr, K, H, 2).off - ws_infer_layout(nullptr, K, H, 1).off;
  const size_t f0 = ws_infer_layout(nullptr, K, H, 1).off;
  if (bytes < f0) return 0;
  int64_t b = 1 + (int64_t)((bytes - f0) / std::max<size_t>(per, 1));
  while (b > 1 && ws_infer_layout(nullptr, K, H, b).off > bytes) b--;
  return b;
}

int mlp_forward_impl(const void* params, int K, int H, const float* X, float* Y, int64_t N,
                     void* ws, size_t bytes, hipStream_t s) {
  const int64_t B = batch_infer_of(K, H, bytes);
  if (B < 1) return fail(NMF_E_WORKSPACE, "network workspace too small");
  const WsI w = ws_infer_layout(ws, K, H, B);
  const Params p = view((void*)params, K, H);
  for (int64_t r = 0; r < N; r += B) {
    const int64_t b = std::min(B, N - r);
    MLPCHECK(cast_bf16(X + r * K, w.xb, b * K, s));
    GemmArgs g{};
    g.A = w.xb;
    g.lda = K;
    g.B = p.W1b;  // B(k,j) = W1[j*K + k]
    g.ldb = K;
    g.M = b;
    g.N = H;
    g.Kd = K;
    g.epi = EPI_BIAS_GELU;  // the pre-activation (C) is not kept
    g.bias = p.b1;
    g.C2 = w.gb;
    g.ldc = H;
    g.splits = 1;
    MLPCHECK(gemm(Elem::BF16, false, true, g, s));
    GemmArgs g2{};
    g2.A = w.gb;
    g2.lda = H;
    g2.B = p.W2b;  // B(j,k) = W2[k*H + j]
    g2.ldb = H;
    g2.M = b;
    g2.N = K;
    g2.Kd = H;
    g2.epi = EPI_BIAS_SOFTPLUS;
    g2.bias = p.b2;
    g2.C2 = Y + r * K;
    g2.ldc = K;
    g2.splits = 1;
    MLPCHECK(gemm(Elem::BF16, false, true, g2, s));
  }
  return NMF_OK;
}
size_t mlp_ws_bytes(int K, int H, int64_t B) { return ws_infer_layout(nullptr, K, H, B).off; }

// The warm start of fold-in: Ht_new = max(eps, ||r|| mlp(r / ||r||)) per row r of
// R.  One fused kernel where the shape allows it, else normalisation, the two
// GEMMs and the rescaling as separate launches (xn, norms, y: [N, K], [N],
// [N, K] scratch for that route).
int mlp_warm_start(const void* params, int K, int H, const float* R, int64_t N, float eps,
                   float* out, float* xn, float* norms, float* y, void* ws, size_t bytes,
                   hipStream_t s) {
  if (mlp_infer_fused_ok(K, H)) {
    const Params p = view((void*)params, K, H);
    MLPCHECK(mlp_infer_fused(R, N, K, H, p.W1b, p.b1, p.W2b, p.b2, eps, out, s));
    return NMF_OK;
  }
  MLPCHECK(row_normalize(R, N, K, xn, norms, s));
  int rc = mlp_forward_impl(params, K, H, xn, y, N, ws, bytes, s);
  if (rc) return rc;
  MLPCHECK(rescale_clip_rows(y, norms, N, K, eps, out, s));
  return NMF_OK;
}
}  // namespace plnmf

extern "C" {

int nmf_mlp_param_bytes(int K, int hidden, nmf_mlp_layout* layout) {
  if (!layout) return fail(NMF_E_ARG, "layout is NULL");
  int rc = check_dims(K, hidden);
  if (rc) return rc;
  *layout = layout_of(K, hidden);
  return NMF_OK;
}

int nmf_mlp_init(void* params, int K, int hidden, uint64_t seed, void* stream) {
  int rc = check_dims(K, hidden);
  if (rc) return rc;
  if (!params || ((uintptr_t)params % kAlign)) return fail(NMF_E_ARG, "params must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const Params p = view(params, K, hidden);
  MLPCHECK(mlp_init_params(p.W1, (int64_t)p.n, K, hidden, seed, s));
  MLPCHECK(hipMemsetAsync(p.m, 0, p.n * sizeof(float), s));
  MLPCHECK(hipMemsetAsync(p.v, 0, p.n * sizeof(float), s));
  MLPCHECK(hipMemsetAsync(p.step, 0, sizeof(int64_t), s));
  MLPCHECK(refresh(p, K, hidden, s));
  return NMF_OK;
}

int nmf_mlp_refresh(void* params, int K, int hidden, void* stream) {
  int rc = check_dims(K, hidden);
  if (rc) return rc;
  if (!params || ((uintptr_t)params % kAlign)) return fail(NMF_E_ARG, "params must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const Params p = view(params, K, hidden);
  MLPCHECK(hipMemsetAsync(p.m, 0, p.n * sizeof(float), s));
  MLPCHECK(hipMemsetAsync(p.v, 0, p.n * sizeof(float), s));
  MLPCHECK(hipMemsetAsync(p.step, 0, sizeof(int64_t), s));
  MLPCHECK(refresh(p, K, hidden, s));
  return NMF_OK;
}

int nmf_mlp_workspace_bytes(int K, int hidden, int64_t batch, size_t* bytes) {
  int rc = check_dims(K, hidden);
  if (rc) return rc;
  if (!bytes || batch < 1) return fail(NMF_E_ARG, "bad batch or NULL bytes");
  *bytes = ws_layout(nullptr, K, hidden, batch).off;
  return NMF_OK;
}

int nmf_mlp_predict(const void* params, int K, int hidden, const float* X, float* Yhat, int64_t N,
                    void* workspace, size_t workspace_bytes, void* stream) {
  int rc = check_dims(K, hidden);
  if (rc) return rc;
  if (!params || !X || !Yhat || !workspace) return fail(NMF_E_ARG, "NULL argument");
  if (N < 0) return fail(NMF_E_ARG, "N < 0");
  return mlp_forward_impl(params, K, hidden, X, Yhat, N, workspace, workspace_bytes,
                          (hipStream_t)stream);
}

int nmf_mlp_loss_grad(const void* params, int K, int hidden, const float* X, const float* Y,
                      int64_t N, float* grads, double* loss, void* workspace,
                      size_t workspace_bytes, void* stream) {
  int rc = check_dims(K, hidden);
  if (rc) return rc;
  if (!params || !X || !Y || !grads || !workspace) return fail(NMF_E_ARG, "NULL argument");
  const int64_t B = batch_of(K, hidden, workspace_bytes);
  if (N < 1 || N > B) return fail(NMF_E_WORKSPACE, "batch of %lld rows exceeds the workspace (%lld)",
                                  (long long)N, (long long)B);
  hipStream_t s = (hipStream_t)stream;
  const Ws w = ws_layout(workspace, K, hidden, B);
  const Params p = view((void*)params, K, hidden);
  rc = loss_grad_rows(p, K, hidden, X, Y, N, grads, w, s);
  if (rc) return rc;
  if (loss) {
    double v = 0.0;
    MLPCHECK(hipMemcpyAsync(&v, w.scal, sizeof(double), hipMemcpyDeviceToHost, s));
    MLPCHECK(hipStreamSynchronize(s));
    *loss = v / (double)(N * K);
  }
  return NMF_OK;
}

int nmf_mlp_adam_step(void* params, int K, int hidden, const float* grads, float lr, void* stream) {
  int rc = check_dims(K, hidden);
  if (rc) return rc;
  if (!params || !grads) return fail(NMF_E_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const Params p = view(params, K, hidden);
  MLPCHECK(mlp_adam(p.W1, p.m, p.v, grads, (int64_t)p.n, lr, p.step, s));
  MLPCHECK(refresh(p, K, hidden, s));
  return NMF_OK;
}

int nmf_mlp_train(void* params, int K, int hidden, const float* X, const float* Y, int64_t N,
                  int epochs, int batch, float lr, uint64_t seed, void* workspace,
                  size_t workspace_bytes, double* epoch_loss, void* stream) {
  int rc = check_dims(K, hidden);
  if (rc) return rc;
  if (!params || !X || !Y || !workspace) return fail(NMF_E_ARG, "NULL argument");
  if (N < 1 || epochs < 0 || batch < 1) return fail(NMF_E_ARG, "bad N, epochs or batch");
  const int64_t B = batch_of(K, hidden, workspace_bytes);
  if (batch > B) return fail(NMF_E_WORKSPACE, "batch %d exceeds the workspace (%lld)", batch,
                             (long long)B);
  hipStream_t s = (hipStream_t)stream;
  const Ws w = ws_layout(workspace, K, hidden, B);
  const Params p = view(params, K, hidden);
  std::vector<int32_t> perm((size_t)N);
  for (int64_t i = 0; i < N; i++) perm[(size_t)i] = (int32_t)i;
  std::mt19937_64 rng(seed);
  for (int ep = 0; ep < epochs; ep++) {
    for (int64_t i = N - 1; i > 0; i--) {  // Fisher-Yates
      const int64_t j = (int64_t)(rng() % (uint64_t)(i + 1));
      std::swap(perm[(size_t)i], perm[(size_t)j]);
    }
    MLPCHECK(hipMemsetAsync(w.scal + 1, 0, sizeof(double), s));
    int64_t nbatches = 0;
    for (int64_t r = 0; r < N; r += batch) {
      const int64_t b = std::min<int64_t>(batch, N - r);
      MLPCHECK(hipMemcpyAsync(w.idx, perm.data() + r, (size_t)b * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
      MLPCHECK(gather_rows(X, w.idx, b, K, w.xbat, s));
      MLPCHECK(gather_rows(Y, w.idx, b, K, w.ybat, s));
      rc = loss_grad_rows(p, K, hidden, w.xbat, w.ybat, b, w.grads, w, s);
      if (rc) return rc;
      MLPCHECK(acc_scaled(w.scal + 1, w.scal, 1.0 / (double)(b * K), s));
      MLPCHECK(mlp_adam(p.W1, p.m, p.v, w.grads, (int64_t)p.n, lr, p.step, s));
      MLPCHECK(refresh(p, K, hidden, s));
      nbatches++;
    }
    // the index uploads read `perm`, which the next epoch reshuffles
    MLPCHECK(hipStreamSynchronize(s));
    if (epoch_loss) {
      double v = 0.0;
      MLPCHECK(hipMemcpyAsync(&v, w.scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
      MLPCHECK(hipStreamSynchronize(s));
      epoch_loss[ep] = v / (double)nbatches;
    }
  }
  return NMF_OK;
}

}  // extern "C"
