// Host side of nmf_foldin: H-only FAST-HALS for new documents with the plan's
// W fixed -- the H half of Alg. 1 (R' = A_new^T W and S = W^T W formed once,
// then the H loop repeated), optionally warm-started by the network.
#include <algorithm>
#include <cmath>
#include <vector>

#include "plan_impl.hpp"

using namespace plnmf;

namespace plnmf {
int mlp_forward_impl(const void* params, int K, int H, const float* X, float* Y, int64_t N,
                     void* ws, size_t bytes, hipStream_t s);
size_t mlp_ws_bytes(int K, int H, int64_t B);
int mlp_warm_start(const void* params, int K, int H, const float* R, int64_t N, float eps,
                   float* out, float* xn, float* norms, float* y, void* ws, size_t bytes,
                   hipStream_t s);
}  // namespace plnmf

namespace {

constexpr int kTraceChunk = 1024;
constexpr int64_t kMlpBatch = 131072;  // rows per network inference pass

struct FoldWs {
  float* R;       // [D',K]
  float* S;       // [K,K]
  float* Qn;      // [K,K]
  float* partial;
  float* gpart;   // Gram partials
  float* panel;   // tile panels of the H update
  double* red;
  double* scal;   // [0] a2 [1] wp [2] sq [3] half [4] rel
  double* trace;  // [kTraceChunk]
  int4* items;
  int32_t* item_slot;
  int32_t* fix;
  float* carry;
  int32_t* counter;
  float* xn;      // MLP input [D',K]
  float* norms;   // [D']
  float* y;       // MLP output [D',K]
  void* mlp_ws;
  size_t mlp_ws_bytes;
  size_t off;
  int L;
};

FoldWs fold_layout(void* base, int64_t Dn, int64_t V, int K, const nmf_matrix* AnewT, int hidden) {
  Carver c(base);
  FoldWs f{};
  f.R = c.take<float>((size_t)(Dn * K));
  f.S = c.take<float>((size_t)K * K);
  f.Qn = c.take<float>((size_t)K * K);
  size_t part = 1;
  int64_t kps;
  if (AnewT->format == NMF_DENSE) {
    const int sp = gemm_pick_splits(Dn, K, V, &kps);
    if (sp > 1) part = std::max(part, (size_t)sp * Dn * K);
  }
  f.partial = c.take<float>(part);
  f.gpart = c.take<float>(gram_partial_floats(K, gram_max_chunks()));
  f.panel = c.take<float>(std::max(std::max(hals_panel_floats(K, 16), hals_panel_floats(K, 32)),
                                    hals_panel_floats(K, 64)));
  f.red = c.take<double>(1024);
  f.scal = c.take<double>(8);
  f.trace = c.take<double>(kTraceChunk);
  if (AnewT->format == NMF_CSR) {
    f.L = spmm_item_nnz(AnewT->nnz);
    const SpmmSizes z = spmm_sizes(Dn, AnewT->nnz, f.L);
    f.items = c.take<int4>((size_t)z.items);
    f.item_slot = c.take<int32_t>((size_t)z.items);
    f.fix = c.take<int32_t>((size_t)(3 * z.fix));
    f.carry = c.take<float>((size_t)(z.seg * K));
    f.counter = c.take<int32_t>(4);
  }
  if (hidden > 0) {
    f.xn = c.take<float>((size_t)(Dn * K));
    f.norms = c.take<float>((size_t)Dn);
    f.y = c.take<float>((size_t)(Dn * K));
    f.mlp_ws_bytes = mlp_ws_bytes(K, hidden, std::min<int64_t>(Dn, kMlpBatch));
    f.mlp_ws = c.take<char>(f.mlp_ws_bytes);
  }
  c.take<char>(kAlign);
  f.off = c.off;
  return f;
}

hipError_t gram_with(const float* X, int64_t rows, int K, float* out, float* gpart, int cus,
                     hipStream_t s, float* panel = nullptr, int tile = 32, bool rows_layout = false) {
  return gram_xtx(X, rows, K, out, K, gpart, gram_chunks(rows, cus), s, panel, 1, tile, rows_layout);
}

#define FCHECK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(NMF_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int fold_objective(nmf_plan_s* p, const FoldWs& f, float* Ht, int64_t Dn, double* dst,
                   hipStream_t s) {
  const int K = p->K;
  FCHECK(gram_with(Ht, Dn, K, f.Qn, f.gpart, p->cus, s));
  int nb = reduce_blocks(Dn * K);
  FCHECK(dot_f64(Ht, f.R, Dn * K, f.red, nb, s));
  FCHECK(finish_f64(f.red, nb, f.scal + 1, s));
  nb = reduce_blocks((int64_t)K * K);
  FCHECK(dot_f64(f.S, f.Qn, (int64_t)K * K, f.red, nb, s));
  FCHECK(finish_f64(f.red, nb, f.scal + 2, s));
  FCHECK(combine_objective(f.scal + 0, f.scal + 1, f.scal + 2, f.scal + 3, dst, s));
  return NMF_OK;
}

int check_anew(nmf_plan_s* p, const nmf_matrix* AnewT) {
  int rc = check_matrix(AnewT);
  if (rc) return rc;
  if (AnewT->cols != p->V)
    return fail(NMF_E_SHAPE, "new documents have %lld terms, plan has V=%lld",
                (long long)AnewT->cols, (long long)p->V);
  return NMF_OK;
}

}  // namespace

extern "C" {

int nmf_foldin_workspace_bytes(nmf_plan p, const nmf_matrix* AnewT, int mlp_hidden,
                               size_t* bytes) {
  if (!p || !bytes) return fail(NMF_E_ARG, "NULL argument");
  int rc = check_anew(p, AnewT);
  if (rc) return rc;
  *bytes = fold_layout(nullptr, AnewT->rows, p->V, p->K, AnewT, mlp_hidden).off;
  return NMF_OK;
}

int nmf_foldin(nmf_plan p, const nmf_matrix* AnewT, float* Ht_new, int init_mode,
               const void* mlp_params, int mlp_hidden, int max_sweeps, double tol,
               int* sweeps_done, double* rel_trace, void* workspace, size_t workspace_bytes) {
  return foldin_run(p, AnewT, Ht_new, init_mode, mlp_params, mlp_hidden, max_sweeps, tol,
                    sweeps_done, rel_trace, workspace, workspace_bytes);
}

}  // extern "C"

// The body of nmf_foldin, shared with the entry point whose workspace is the
// library's own device array.
int plnmf::foldin_run(nmf_plan p, const nmf_matrix* AnewT, float* Ht_new, int init_mode,
                      const void* mlp_params, int mlp_hidden, int max_sweeps, double tol,
                      int* sweeps_done, double* rel_trace, void* workspace,
                      size_t workspace_bytes) {
  if (sweeps_done) *sweeps_done = 0;
  if (!p || !Ht_new || !workspace) return fail(NMF_E_ARG, "NULL argument");
  if (!(tol >= 0.0) || std::isinf(tol)) return fail(NMF_E_ARG, "tol must be finite and >= 0");
  const int n_sweeps = max_sweeps;
  if (p->poisoned) return fail(p->poisoned, "plan is poisoned by an earlier error");
  int rc = check_anew(p, AnewT);
  if (rc) return rc;
  if (init_mode < NMF_FOLDIN_GIVEN || init_mode > NMF_FOLDIN_MLP)
    return fail(NMF_E_ARG, "unknown init mode %d", init_mode);
  if (init_mode == NMF_FOLDIN_MLP && (!mlp_params || mlp_hidden < 1))
    return fail(NMF_E_ARG, "MLP init needs parameters and hidden > 0");
  if (n_sweeps < 0) return fail(NMF_E_ARG, "max_sweeps < 0");
  if (((uintptr_t)Ht_new & 15) || ((uintptr_t)workspace % kAlign))
    return fail(NMF_E_ARG, "misaligned Ht_new or workspace");
  const int64_t Dn = AnewT->rows;
  const int K = p->K;
  const int hid = init_mode == NMF_FOLDIN_MLP ? mlp_hidden : 0;
  FoldWs f = fold_layout(workspace, Dn, p->V, K, AnewT, hid);
  if (workspace_bytes < f.off)
    return fail(NMF_E_WORKSPACE, "fold-in workspace %zu < %zu", workspace_bytes, f.off);
  hipStream_t s = p->stream;

  // validate and build the product plan for the new documents
  FCHECK(hipMemsetAsync(f.scal, 0, 8 * sizeof(double), s));
  if (AnewT->format == NMF_CSR) {
    FCHECK(hipMemsetAsync(f.counter, 0, 4 * sizeof(int32_t), s));
    FCHECK(csr_validate(Dn, p->V, AnewT->nnz, AnewT->rowptr, AnewT->colidx, AnewT->values,
                        f.counter + 1, s));
    int32_t flag = 0;
    FCHECK(hipMemcpyAsync(&flag, f.counter + 1, sizeof(flag), hipMemcpyDeviceToHost, s));
    FCHECK(hipStreamSynchronize(s));
    if (flag & 3) return fail(NMF_E_SHAPE, "new-document CSR structure invalid (code %d)", flag);
    if (flag & 4) return fail(NMF_E_NUMERIC, "new documents have a negative, NaN or Inf entry");
    SpmmPlan sp{};
    sp.rows = Dn;
    sp.nnz = AnewT->nnz;
    sp.L = f.L;
    sp.rowptr = AnewT->rowptr;
    sp.col = AnewT->colidx;
    sp.val = AnewT->values;
    sp.items = f.items;
    sp.item_slot = f.item_slot;
    sp.fix = f.fix;
    sp.carry = f.carry;
    FCHECK(spmm_build(&sp, s));
    FCHECK(spmm(sp, Elem::F32, p->W, K, f.R, s));
    const int nb = reduce_blocks(AnewT->nnz);
    FCHECK(sumsq_f64(AnewT->values, AnewT->nnz, f.red, nb, s));
    FCHECK(finish_f64(f.red, nb, f.scal + 0, s));
  } else {
    GemmArgs g{};
    g.A = AnewT->dense;
    g.lda = p->V;
    g.B = p->W;
    g.ldb = K;
    g.M = Dn;
    g.N = K;
    g.Kd = p->V;
    g.C = f.R;
    g.ldc = K;
    g.epi = EPI_STORE;
    g.splits = gemm_pick_splits(g.M, g.N, g.Kd, &g.k_per_split);
    g.partial = f.partial;
    FCHECK(gemm(Elem::F32, false, false, g, s));
    const int nb = reduce_blocks(Dn * p->V);
    FCHECK(sumsq_f64(AnewT->dense, Dn * p->V, f.red, nb, s));
    FCHECK(finish_f64(f.red, nb, f.scal + 0, s));
  }
  FCHECK(hipMemsetAsync(f.panel, 0,
                        std::max(std::max(hals_panel_floats(K, 16), hals_panel_floats(K, 32)),
                                 hals_panel_floats(K, 64)) * sizeof(float), s));
  const bool rl = hals_h_rows_layout(Dn, K, p->cus, p->h_tile);
  FCHECK(gram_with(p->W, p->V, K, f.S, f.gpart, p->cus, s, f.panel, p->h_tile, rl));

  // initialisation of H for the new documents
  if (init_mode == NMF_FOLDIN_WTA) {
    FCHECK(clip_min(f.R, Dn * K, p->eps, Ht_new, s));
  } else if (init_mode == NMF_FOLDIN_MLP) {
    rc = mlp_warm_start(mlp_params, K, mlp_hidden, f.R, Dn, p->eps, Ht_new, f.xn, f.norms, f.y,
                        f.mlp_ws, f.mlp_ws_bytes, s);
    if (rc) return rc;
  }

  HalsArgs a{};
  a.X = Ht_new;
  a.Bterm = f.R;
  a.G = f.S;
  a.rows = Dn;
  a.K = K;
  a.eps = p->eps;
  a.diag_one = 1;
  a.panel = f.panel;
  a.tile = p->h_tile;
  a.rows_layout = rl;
  int filled = 0;  // trace entries waiting in f.trace
  int written = 0; // trace entries copied to the host
  auto flush = [&]() -> int {
    if (filled == 0) return NMF_OK;
    FCHECK(hipMemcpyAsync(rel_trace + written, f.trace, (size_t)filled * sizeof(double),
                          hipMemcpyDeviceToHost, s));
    FCHECK(hipStreamSynchronize(s));
    written += filled;
    filled = 0;
    return NMF_OK;
  };
  if (tol > 0.0) {
    // stop at the first sweep whose decrease of the relative objective is
    // below tol: the objective is read back after every sweep (one 8-byte copy
    // and one synchronisation per sweep)
    double prev = 0.0, cur = 0.0;
    rc = fold_objective(p, f, Ht_new, Dn, f.trace, s);
    if (rc) return rc;
    FCHECK(hipMemcpyAsync(&prev, f.trace, sizeof(double), hipMemcpyDeviceToHost, s));
    FCHECK(hipStreamSynchronize(s));
    if (!std::isfinite(prev)) return fail(NMF_E_NUMERIC, "fold-in objective is not finite");
    if (rel_trace) rel_trace[0] = prev;
    int done = 0;
    while (done < n_sweeps) {
      FCHECK(hals_update(a, s));
      rc = fold_objective(p, f, Ht_new, Dn, f.trace, s);
      if (rc) return rc;
      FCHECK(hipMemcpyAsync(&cur, f.trace, sizeof(double), hipMemcpyDeviceToHost, s));
      FCHECK(hipStreamSynchronize(s));
      if (!std::isfinite(cur)) return fail(NMF_E_NUMERIC, "fold-in objective is not finite");
      done++;
      if (rel_trace) rel_trace[done] = cur;
      if (sweeps_done) *sweeps_done = done;
      if (prev - cur < tol) break;
      prev = cur;
    }
    return NMF_OK;
  }
  if (rel_trace) {
    rc = fold_objective(p, f, Ht_new, Dn, f.trace + filled, s);
    if (rc) return rc;
    filled++;
  }
  for (int i = 0; i < n_sweeps; i++) {
    FCHECK(hals_update(a, s));
    if (rel_trace) {
      if (filled == kTraceChunk) {
        rc = flush();
        if (rc) return rc;
      }
      rc = fold_objective(p, f, Ht_new, Dn, f.trace + filled, s);
      if (rc) return rc;
      filled++;
    }
  }
  if (rel_trace) {
    rc = flush();
    if (rc) return rc;
  }
  if (sweeps_done) *sweeps_done = n_sweeps;
  return NMF_OK;
}
