// Private host-side declarations shared by the C-ABI implementation files.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "../../include/nmf.h"
#include "internal.hpp"

namespace plnmf {

int fail(int code, const char* fmt, ...);

#define HIPCHECK(plan, expr)                                                              \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) {                                                               \
      if (plan) (plan)->poisoned = NMF_E_HIP;                                             \
      return ::plnmf::fail(NMF_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    }                                                                                     \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kDenseRowsMax = 256;  // rows of A multiplied as a dense block in P = A H^T
constexpr int64_t kDenseRowsMinDK = (int64_t)32 << 20;  // ... when D K reaches this
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Sequential carve of a workspace: with base == nullptr it only sizes.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t count) {
    off = align_up(off);
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

int device_check(int* dev, int* cus);
int check_matrix(const nmf_matrix* A);

}  // namespace plnmf

struct nmf_plan_s {
  int device = 0, cus = 0;
  hipStream_t stream = nullptr;
  int64_t V = 0, D = 0, nnz = 0;
  int K = 0, fmt = 0, prec = 0;
  float eps = 0.f;
  float* W = nullptr;
  float* Ht = nullptr;
  const float* A_dense = nullptr;
  const int32_t* a_rowptr = nullptr;
  const int32_t* a_col = nullptr;
  const float* a_val = nullptr;
  int32_t* t_rowptr = nullptr;
  int32_t* t_col = nullptr;
  float* t_val = nullptr;
  __bf16* a_val_bf = nullptr;
  __bf16* t_val_bf = nullptr;
  __bf16* A_bf = nullptr;   // dense [V,D]
  __bf16* At_bf = nullptr;  // dense [D,V]
  __bf16* X_bf = nullptr;   // per-sweep BF16 cast of W or Ht
  plnmf::SpmmPlan sp_A{}, sp_At{};
  plnmf::SpmmPlan sp_A_f32{};  // FP32 values of A (objective of BF16 plans)
  float* a_top = nullptr;       // [n_top, D] the densest rows of A, dense (CSR plans)
  __bf16* a_top_bf = nullptr;   // the same in BF16 (CSR plans with BF16 products)
  float* c_top = nullptr;       // [n_top, K] their rows of P
  int32_t* top_idx = nullptr;   // [n_top] their row indices
  int n_top = 0;
  int h_panel_order = -1;       // order of panel_h's entries: -1 all zero, 0 plain, 1 rows kernel's
  float* P = nullptr;
  float* Q = nullptr;
  float* R = nullptr;
  float* S = nullptr;
  float* S2 = nullptr;
  float* P2 = nullptr;      // FP32 A H^T for the objective of BF16 plans
  float* partial = nullptr;
  float* gram_part = nullptr;   // per-chunk partial Grams
  float* panel = nullptr;       // precomputed tile panels of the W update (32 wide)
  float* panel_h = nullptr;     // those of the H update (h_tile wide)
  size_t panel_h_floats = 0;
  int h_tile = 32;              // tile width of the H update
  size_t partial_floats = 0;
  double* colsq = nullptr;
  double* red = nullptr;
  int red_n = 0;
  double* scal = nullptr;   // [0] ||A||^2 [1] <W,P> [2] sum sq [3] half [4] rel
  unsigned long long* slots = nullptr;
  unsigned* w_flags = nullptr;
  float* w_handoff = nullptr;  // [ceil(K/kTile)][V][kTile] tile products
  float* w_new = nullptr;      // [ceil(K/kTile)][V][kTile] finished tiles
  int32_t* status = nullptr;
  int w_grid = 0;
  int w_groups = 0;            // column groups of the W kernel
  int w_rows_per_group = 0;
  int tr_blocks = 1;
  unsigned epoch = 1;
  int64_t sweeps_done = 0;
  bool pq_valid = false;
  int poisoned = 0;
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof[NMF_STEP_COUNT];
};

namespace plnmf {
// out = X^T X; with panel_diag 1 also the H update's tile panels (p->panel_h,
// p->h_tile wide), with 0 the W update's (p->panel, 32 wide)
hipError_t gram(nmf_plan_s* p, const float* X, int64_t rows, float* out, int panel_diag = -1,
                bool rows_layout = false);
int enqueue_objective(nmf_plan_s* p);
// nmf_foldin on a given workspace (also serves the entry point that brings none)
int foldin_run(nmf_plan p, const nmf_matrix* AnewT, float* Ht_new, int init_mode,
               const void* mlp_params, int mlp_hidden, int max_sweeps, double tol,
               int* sweeps_done, double* rel_trace, void* workspace, size_t workspace_bytes);
}  // namespace plnmf
