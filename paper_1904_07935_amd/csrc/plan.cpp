// Host side of the C ABI declared in include/nmf.h: plan creation and
// validation, the workspace layout, and the per-sweep launch sequence of
// FAST-HALS (Alg. 1): H half = R = A^T W, S = W^T W, tiled H update; W half =
// P = A H^T, Q = H H^T, persistent tiled W update with in-kernel column
// normalisation.  All device memory is caller-owned; this file only carves the
// caller's workspace and enqueues kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "plan_impl.hpp"

using namespace plnmf;

namespace plnmf {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

}  // namespace plnmf

namespace {

struct ShapeInfo {
  int64_t V, D, nnz;
  int K;
  int fmt, prec;
};

// blocks of the deterministic CSR transpose: >= 32 source rows each, and the
// count table (blocks + 1) x D must fit in the P/R region it borrows
int tr_blocks_for(int64_t V, int64_t D, int64_t pr_floats) {
  int64_t nb = V / 32;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  while (nb > 1 && (nb + 1) * D > pr_floats) nb /= 2;
  return (int)nb;
}

}  // namespace

namespace {

void layout(const ShapeInfo& s, Carver& c, nmf_plan_s* p) {
  const int64_t V = s.V, D = s.D, K = s.K, nnz = s.nnz;
  const int64_t p_floats = (int64_t)(align_up((size_t)(V * K) * 4) / 4);
  int64_t pr_floats = p_floats + D * K;
  int nblk = 1;
  if (s.fmt == NMF_CSR) {
    nblk = tr_blocks_for(V, D, std::max<int64_t>(pr_floats, (int64_t)16 << 20));
    pr_floats = std::max<int64_t>(pr_floats, (int64_t)(nblk + 1) * D);
  }
  float* P = c.take<float>((size_t)pr_floats);
  float* R = P ? P + p_floats : nullptr;
  if (p) p->tr_blocks = nblk;
  float* Q = c.take<float>((size_t)(K * K));
  float* S = c.take<float>((size_t)(K * K));
  float* S2 = c.take<float>((size_t)(K * K));
  if (p) { p->P = P; p->R = R; p->Q = Q; p->S = S; p->S2 = S2; }
  // split-K partials: the largest of the GEMMs a sweep launches
  size_t part = 0;
  auto need = [&](int64_t M, int64_t N, int64_t Kd) {
    int64_t kps;
    int sp = gemm_pick_splits(M, N, Kd, &kps);
    if (sp > 1) part = std::max(part, (size_t)(sp * M * N));
  };
  if (s.fmt == NMF_DENSE) {
    need(D, K, V);
    need(V, K, D);
  }
  if (s.fmt == NMF_CSR) need(kDenseRowsMax, K, D);  // the dense rows of A in P
  float* partial = c.take<float>(std::max<size_t>(part, 1));
  float* gpart = c.take<float>(gram_partial_floats((int)K, gram_max_chunks()));
  float* panel = c.take<float>(hals_panel_floats((int)K));
  // the H update's panels, sized for every supported tile width
  const size_t ph = std::max(std::max(hals_panel_floats((int)K, 16), hals_panel_floats((int)K, 32)),
                             hals_panel_floats((int)K, 64));
  float* panel_h = c.take<float>(ph);
  const int64_t resid_tiles = ((V + 127) / 128) * ((D + 127) / 128);
  const int red_n = (int)std::max<int64_t>(std::max<int64_t>(resid_tiles, 1024), 1);
  double* red = c.take<double>((size_t)red_n);
  double* scal = c.take<double>(16);
  unsigned long long* slots = c.take<unsigned long long>(kSlotWords);
  unsigned* wflags = c.take<unsigned>(kWFlagWords);
  const int64_t wtiles = (K + kTile - 1) / kTile;
  float* whand = c.take<float>((size_t)(wtiles * V * kTile));
  float* wnew = c.take<float>((size_t)(wtiles * V * kTile));
  int32_t* status = c.take<int32_t>(16);
  double* colsq = c.take<double>((size_t)1024 * K);
  if (p) {
    p->colsq = colsq;
    p->partial = partial;
    p->gram_part = gpart;
    p->panel = panel;
    p->panel_h = panel_h;
    p->panel_h_floats = ph;
    p->partial_floats = std::max<size_t>(part, 1);
    p->red = red;
    p->red_n = red_n;
    p->scal = scal;
    p->slots = slots;
    p->w_flags = wflags;
    p->w_handoff = whand;
    p->w_new = wnew;
    p->status = status;
  }
  if (s.fmt == NMF_CSR) {
    int32_t* t_rowptr = c.take<int32_t>((size_t)(D + 1));
    int32_t* t_col = c.take<int32_t>((size_t)std::max<int64_t>(nnz, 1));
    float* t_val = c.take<float>((size_t)std::max<int64_t>(nnz, 1));
    const int L = spmm_item_nnz(nnz);
    const SpmmSizes zA = spmm_sizes(V, nnz, L), zT = spmm_sizes(D, nnz, L);
    int4* itA = c.take<int4>((size_t)zA.items);
    int32_t* slA = c.take<int32_t>((size_t)zA.items);
    int32_t* fixA = c.take<int32_t>((size_t)(3 * zA.fix));
    float* carryA = c.take<float>((size_t)(zA.seg * K));
    int4* itT = c.take<int4>((size_t)zT.items);
    int32_t* slT = c.take<int32_t>((size_t)zT.items);
    int32_t* fixT = c.take<int32_t>((size_t)(3 * zT.fix));
    float* carryT = c.take<float>((size_t)(zT.seg * K));
    float* a_top = c.take<float>((size_t)kDenseRowsMax * D);
    float* c_top = c.take<float>((size_t)kDenseRowsMax * K);
    int32_t* top_idx = c.take<int32_t>((size_t)kDenseRowsMax);
    __bf16 *avb = nullptr, *tvb = nullptr, *xb = nullptr, *atb = nullptr;
    float* P2 = nullptr;
    if (s.prec == NMF_BF16_PRODUCTS) {
      atb = c.take<__bf16>((size_t)kDenseRowsMax * D);
      avb = c.take<__bf16>((size_t)std::max<int64_t>(nnz, 1));
      tvb = c.take<__bf16>((size_t)std::max<int64_t>(nnz, 1));
      xb = c.take<__bf16>((size_t)(std::max(V, D) * K));
      P2 = c.take<float>((size_t)(V * K));
    }
    if (p) {
      p->t_rowptr = t_rowptr;
      p->t_col = t_col;
      p->t_val = t_val;
      p->sp_A.L = p->sp_At.L = L;
      p->sp_A.items = itA;
      p->sp_A.item_slot = slA;
      p->sp_A.fix = fixA;
      p->sp_A.carry = carryA;
      p->sp_At.items = itT;
      p->sp_At.item_slot = slT;
      p->sp_At.fix = fixT;
      p->sp_At.carry = carryT;
      p->a_top = a_top;
      p->a_top_bf = atb;
      p->c_top = c_top;
      p->top_idx = top_idx;
      p->a_val_bf = avb;
      p->t_val_bf = tvb;
      p->X_bf = xb;
      p->P2 = P2;
    }
  } else if (s.prec == NMF_BF16_PRODUCTS) {
    __bf16* Ab = c.take<__bf16>((size_t)(V * D));
    __bf16* Atb = c.take<__bf16>((size_t)(V * D));
    __bf16* xb = c.take<__bf16>((size_t)(std::max(V, D) * K));
    if (p) {
      p->A_bf = Ab;
      p->At_bf = Atb;
      p->X_bf = xb;
    }
  }
  c.take<char>(kAlign);
}

}  // namespace

int plnmf::check_matrix(const nmf_matrix* A) {
  if (!A) return fail(NMF_E_ARG, "A is NULL");
  if (A->rows <= 0 || A->cols <= 0) return fail(NMF_E_SHAPE, "A has an empty dimension");
  if (A->format == NMF_DENSE) {
    if (!A->dense) return fail(NMF_E_ARG, "dense A without data pointer");
    if (((uintptr_t)A->dense) & 15) return fail(NMF_E_ARG, "dense A must be 16-byte aligned");
  } else if (A->format == NMF_CSR) {
    if (!A->rowptr || (A->nnz > 0 && (!A->colidx || !A->values)))
      return fail(NMF_E_ARG, "CSR A with a NULL array");
    if (A->nnz < 0 || A->nnz > (int64_t)INT32_MAX) return fail(NMF_E_SHAPE, "nnz out of range");
    if (A->rows > (int64_t)INT32_MAX - 1 || A->cols > (int64_t)INT32_MAX - 1)
      return fail(NMF_E_SHAPE, "CSR dimension exceeds int32 indexing");
  } else {
    return fail(NMF_E_ARG, "unknown matrix format %d", (int)A->format);
  }
  return NMF_OK;
}

namespace {

int check_shape(const nmf_matrix* A, int K, int precision) {
  int rc = check_matrix(A);
  if (rc) return rc;
  if (precision != NMF_FP32 && precision != NMF_BF16_PRODUCTS)
    return fail(NMF_E_ARG, "unknown precision %d", precision);
  if (K < 1 || K > NMF_MAX_K) return fail(NMF_E_SHAPE, "K=%d outside [1, %d]", K, NMF_MAX_K);
  if (K > A->rows || K > A->cols)
    return fail(NMF_E_SHAPE, "K=%d exceeds min(V, D) = %lld", K,
                (long long)std::min(A->rows, A->cols));
  return NMF_OK;
}

ShapeInfo shape_of(const nmf_matrix* A, int K, int precision) {
  ShapeInfo s;
  s.V = A->rows;
  s.D = A->cols;
  s.nnz = A->format == NMF_CSR ? A->nnz : A->rows * A->cols;
  s.K = K;
  s.fmt = A->format;
  s.prec = precision;
  return s;
}

}  // namespace

int plnmf::device_check(int* dev, int* cus) {
  hipError_t e = hipGetDevice(dev);
  if (e != hipSuccess) return fail(NMF_E_HIP, "no HIP device: %s", hipGetErrorString(e));
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, *dev);
  if (e != hipSuccess) return fail(NMF_E_HIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(NMF_E_HIP, "device %s is not gfx950 (library built for gfx950 only)",
                prop.gcnArchName);
  *cus = prop.multiProcessorCount;
  return NMF_OK;
}

// ------------------------------------------------------- step launchers ----
hipError_t plnmf::gram(nmf_plan_s* p, const float* X, int64_t rows, float* out, int panel_diag,
                       bool rows_layout) {
  // panel_diag 1: the H update's panels (its own buffer and tile width, in
  // the order of the kernel that will read them); 0: the W update's (32 wide)
  float* panel = panel_diag == 1 ? p->panel_h : panel_diag == 0 ? p->panel : nullptr;
  return gram_xtx(X, rows, p->K, out, p->K, p->gram_part, gram_chunks(rows, p->cus), p->stream,
                  panel, panel_diag, panel_diag == 1 ? p->h_tile : kTile, panel_diag == 1 && rows_layout);
}

namespace {

// R = A^T W  (D x K)
hipError_t product_R(nmf_plan_s* p) {
  const int K = p->K;
  if (p->fmt == NMF_CSR) {
    if (p->prec == NMF_BF16_PRODUCTS) {
      hipError_t e = cast_bf16(p->W, p->X_bf, p->V * K, p->stream);
      if (e != hipSuccess) return e;
      return spmm(p->sp_At, Elem::BF16, p->X_bf, K, p->R, p->stream);
    }
    if (K > 256) {
      // two column slices of W: twice as many of the popular terms' rows fit
      // in an XCD's L2 (each column's sums keep their nonzero order, so the
      // result is the same).  Measured on 10^5 x 3*10^5 at K = 400: 3.20 ->
      // 3.05 ms; four slices 3.71 ms.
      const int kh = (K / 2) / 4 * 4;
      hipError_t e = spmm_slice(p->sp_At, Elem::F32, p->W, K, 0, kh, p->R, K, p->stream);
      if (e != hipSuccess) return e;
      return spmm_slice(p->sp_At, Elem::F32, p->W, K, kh, K - kh, p->R, K, p->stream);
    }
    return spmm(p->sp_At, Elem::F32, p->W, K, p->R, p->stream);
  }
  GemmArgs g{};
  g.M = p->D;
  g.N = K;
  g.Kd = p->V;
  g.C = p->R;
  g.ldc = K;
  g.epi = EPI_STORE;
  g.splits = gemm_pick_splits(g.M, g.N, g.Kd, &g.k_per_split);
  g.partial = p->partial;
  if (p->prec == NMF_BF16_PRODUCTS) {
    hipError_t e = cast_bf16_transpose(p->W, p->X_bf, p->V, K, p->stream);  // W^T [K,V]
    if (e != hipSuccess) return e;
    g.A = p->At_bf;  // [D,V]
    g.lda = p->V;
    g.B = p->X_bf;   // B(v,k) = WT[k*V + v]
    g.ldb = p->V;
    return gemm(Elem::BF16, false, true, g, p->stream);
  }
  g.A = p->A_dense;  // A(d,v) = A[v*D + d]
  g.lda = p->D;
  g.B = p->W;
  g.ldb = K;
  return gemm(Elem::F32, true, false, g, p->stream);
}

// NMF_DENSE_ROWS=0 keeps every row of A in the sparse P product, =1 takes the
// dense rows whatever the size (measurement, tests); unset: by size.
int dense_rows_mode() {
  const char* e = getenv("NMF_DENSE_ROWS");
  if (e && e[0] == '0') return 0;
  if (e && e[0] == '1') return 1;
  return -1;
}

// P = A H^T  (V x K), from Ht [D,K]
hipError_t product_P(nmf_plan_s* p, bool force_fp32, float* out) {
  const int K = p->K;
  const bool bf = p->prec == NMF_BF16_PRODUCTS && !force_fp32;
  if (p->fmt == NMF_CSR) {
    hipError_t e;
    if (bf) {
      e = cast_bf16(p->Ht, p->X_bf, p->D * K, p->stream);
      if (e == hipSuccess) e = spmm(p->sp_A, Elem::BF16, p->X_bf, K, out, p->stream);
    } else {
      e = spmm(p->prec == NMF_BF16_PRODUCTS ? p->sp_A_f32 : p->sp_A, Elem::F32, p->Ht, K, out,
               p->stream);
    }
    if (e != hipSuccess || p->n_top == 0) return e;
    // the dense rows: C_top [n_top, K] = A_top [n_top, D] H^T on the matrix
    // cores (in the precision of the other products), then into their rows of P
    GemmArgs g{};
    g.A = bf ? (const void*)p->a_top_bf : (const void*)p->a_top;
    g.lda = p->D;
    g.B = bf ? (const void*)p->X_bf : (const void*)p->Ht;  // B(d,k) = Ht[d*K + k]
    g.ldb = K;
    g.M = p->n_top;
    g.N = K;
    g.Kd = p->D;
    g.C = p->c_top;
    g.ldc = K;
    g.epi = EPI_STORE;
    g.splits = gemm_pick_splits(g.M, g.N, g.Kd, &g.k_per_split);
    g.partial = p->partial;
    e = gemm(bf ? Elem::BF16 : Elem::F32, false, false, g, p->stream);
    if (e != hipSuccess) return e;
    return scatter_rows(p->c_top, p->top_idx, p->n_top, K, out, p->stream);
  }
  GemmArgs g{};
  g.M = p->V;
  g.N = K;
  g.Kd = p->D;
  g.C = out;
  g.ldc = K;
  g.epi = EPI_STORE;
  g.splits = gemm_pick_splits(g.M, g.N, g.Kd, &g.k_per_split);
  g.partial = p->partial;
  if (bf) {
    hipError_t e = cast_bf16_transpose(p->Ht, p->X_bf, p->D, K, p->stream);  // H [K,D]
    if (e != hipSuccess) return e;
    g.A = p->A_bf;  // [V,D]
    g.lda = p->D;
    g.B = p->X_bf;  // B(d,k) = H[k*D + d]
    g.ldb = p->D;
    return gemm(Elem::BF16, false, true, g, p->stream);
  }
  g.A = p->A_dense;
  g.lda = p->D;
  g.B = p->Ht;  // B(d,k) = Ht[d*K + k]
  g.ldb = K;
  return gemm(Elem::F32, false, false, g, p->stream);
}

unsigned next_epoch(nmf_plan_s* p) {
  unsigned e = p->epoch & 0x3FFFFFu;
  if (e == 0) e = 1;
  p->epoch = e + 1;
  return e;
}

// event pair around one step on the plan's stream (profiling only)
hipEvent_t prof_begin(nmf_plan_s* p) {
  if (!p->profiling) return nullptr;
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  if (hipEventRecord(e, p->stream) != hipSuccess) {
    (void)hipEventDestroy(e);
    return nullptr;
  }
  return e;
}

void prof_end(nmf_plan_s* p, int step, hipEvent_t e0) {
  if (!e0) return;
  hipEvent_t e1 = nullptr;
  if (hipEventCreate(&e1) != hipSuccess || hipEventRecord(e1, p->stream) != hipSuccess) {
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return;
  }
  p->prof[step].push_back({e0, e1});
}

#define TIMED(p, step, expr)                 \
  do {                                       \
    hipEvent_t ev0_ = prof_begin(p);         \
    HIPCHECK(p, expr);                       \
    prof_end(p, step, ev0_);                 \
  } while (0)

void prof_clear(nmf_plan_s* p) {
  for (auto& v : p->prof) {
    for (auto& e : v) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    v.clear();
  }
}

int half_h(nmf_plan_s* p) {
  const bool rl = hals_h_rows_layout(p->D, p->K, p->cus, p->h_tile);
  if (p->h_panel_order >= 0 && p->h_panel_order != (rl ? 1 : 0)) {
    // the kernel choice changed (NMF_H_KERNEL): the other order's entries go
    const hipError_t e = hipMemsetAsync(p->panel_h, 0, p->panel_h_floats * sizeof(float), p->stream);
    if (e != hipSuccess) return fail(NMF_E_HIP, "hipMemsetAsync: %s", hipGetErrorString(e));
  }
  p->h_panel_order = rl ? 1 : 0;
  TIMED(p, NMF_STEP_GRAM_S, gram(p, p->W, p->V, p->S, 1, rl));  // + the H update's panels
  TIMED(p, NMF_STEP_PRODUCT_R, product_R(p));
  HalsArgs a{};
  a.X = p->Ht;
  a.Bterm = p->R;
  a.G = p->S;
  a.rows = p->D;
  a.K = p->K;
  a.eps = p->eps;
  a.diag_one = 1;
  a.panel = p->panel_h;
  a.tile = p->h_tile;
  a.rows_layout = rl;
  TIMED(p, NMF_STEP_UPDATE_H, hals_update(a, p->stream));
  p->pq_valid = false;
  return NMF_OK;
}

int half_w(nmf_plan_s* p) {
  TIMED(p, NMF_STEP_PRODUCT_P, product_P(p, false, p->P));
  TIMED(p, NMF_STEP_GRAM_Q, gram(p, p->Ht, p->D, p->Q, 0));  // + the W update's panels
  HalsWArgs a{};
  a.X = p->W;
  a.Bterm = p->P;
  a.G = p->Q;
  a.rows = p->V;
  a.K = p->K;
  a.eps = p->eps;
  a.Y = p->w_handoff;
  a.Wn = p->w_new;
  a.panel = p->panel;
  a.slots = p->slots;
  a.flags = p->w_flags;
  a.n_col = p->w_groups;
  a.rows_per_group = p->w_rows_per_group;
  a.epoch = next_epoch(p);
  a.status = p->status;
  TIMED(p, NMF_STEP_UPDATE_W, hals_w_update(a, p->w_grid, p->stream));
  p->pq_valid = p->prec == NMF_FP32;
  return NMF_OK;
}

// Multiplicative update (the MU baseline): X <- X * N / (X G + delta) with
// N = R, G = S (H rule, X = Ht) or N = P, G = Q (W rule, X = W).  The
// denominator is the matrix-core product X G, whose epilogue writes the new
// values over N (each element read, then written, by one thread: X, the
// product's operand, is left intact); they are then copied into X.
hipError_t mu_update(nmf_plan_s* p, float* X, int64_t rows, float* N, const float* G) {
  const int K = p->K;
  GemmArgs g{};
  g.A = X;
  g.lda = K;
  g.B = G;
  g.ldb = K;
  g.M = rows;
  g.N = K;
  g.Kd = K;
  g.C = N;
  g.ldc = K;
  g.epi = EPI_MU;
  g.D = N;
  g.ldd = K;
  g.C2 = X;
  g.splits = 1;
  g.mu_delta = p->eps;
  hipError_t e = gemm(Elem::F32, false, false, g, p->stream);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(X, N, (size_t)rows * K * sizeof(float), hipMemcpyDeviceToDevice, p->stream);
}

int mu_half_h(nmf_plan_s* p) {
  TIMED(p, NMF_STEP_GRAM_S, gram(p, p->W, p->V, p->S));
  TIMED(p, NMF_STEP_PRODUCT_R, product_R(p));
  TIMED(p, NMF_STEP_UPDATE_H, mu_update(p, p->Ht, p->D, p->R, p->S));
  p->pq_valid = false;
  return NMF_OK;
}

int mu_half_w(nmf_plan_s* p) {
  TIMED(p, NMF_STEP_PRODUCT_P, product_P(p, false, p->P));
  TIMED(p, NMF_STEP_GRAM_Q, gram(p, p->Ht, p->D, p->Q));
  TIMED(p, NMF_STEP_UPDATE_W, mu_update(p, p->W, p->V, p->P, p->Q));
  p->pq_valid = false;  // P now holds the new W
  return NMF_OK;
}

int read_status(nmf_plan_s* p) {
  int32_t st = 0;
  HIPCHECK(p, hipMemcpyAsync(&st, p->status, sizeof(st), hipMemcpyDeviceToHost, p->stream));
  HIPCHECK(p, hipStreamSynchronize(p->stream));
  if (st & 256) {
    p->poisoned = NMF_E_TIMEOUT;
    return fail(NMF_E_TIMEOUT, "a device-side wait of the W update timed out");
  }
  return NMF_OK;
}

}  // namespace

// enqueue the objective into scal[3] (half) and scal[4] (rel)
int plnmf::enqueue_objective(nmf_plan_s* p) {
  double* sc = p->scal;
  if (p->fmt == NMF_DENSE) {
    GemmArgs g{};
    g.A = p->W;
    g.lda = p->K;
    g.B = p->Ht;  // B(k,d) = Ht[d*K + k]
    g.ldb = p->K;
    g.M = p->V;
    g.N = p->D;
    g.Kd = p->K;
    g.epi = EPI_RESID_SQ;
    g.D = p->A_dense;
    g.ldd = p->D;
    g.red_out = p->red;
    g.splits = 1;
    HIPCHECK(p, gemm(Elem::F32, false, true, g, p->stream));
    const int tiles = (int)(((p->V + 127) / 128) * ((p->D + 127) / 128));
    HIPCHECK(p, finish_f64(p->red, tiles, sc + 2, p->stream));
    HIPCHECK(p, combine_objective(sc + 0, nullptr, sc + 2, sc + 3, sc + 4, p->stream));
    return NMF_OK;
  }
  float* Puse = p->P;
  if (!p->pq_valid) {
    Puse = p->prec == NMF_BF16_PRODUCTS ? p->P2 : p->P;
    HIPCHECK(p, product_P(p, true, Puse));
    HIPCHECK(p, gram(p, p->Ht, p->D, p->Q));
  }
  HIPCHECK(p, gram(p, p->W, p->V, p->S2));
  const int64_t n1 = p->V * p->K;
  int nb = reduce_blocks(n1);
  HIPCHECK(p, dot_f64(p->W, Puse, n1, p->red, nb, p->stream));
  HIPCHECK(p, finish_f64(p->red, nb, sc + 1, p->stream));
  const int64_t n2 = (int64_t)p->K * p->K;
  nb = reduce_blocks(n2);
  HIPCHECK(p, dot_f64(p->S2, p->Q, n2, p->red, nb, p->stream));
  HIPCHECK(p, finish_f64(p->red, nb, sc + 2, p->stream));
  HIPCHECK(p, combine_objective(sc + 0, sc + 1, sc + 2, sc + 3, sc + 4, p->stream));
  return NMF_OK;
}

extern "C" {

const char* nmf_last_error(void) { return g_last_error.c_str(); }

int nmf_workspace_bytes(const nmf_matrix* A, int K, int precision, size_t* bytes) {
  if (!bytes) return fail(NMF_E_ARG, "bytes is NULL");
  int rc = check_shape(A, K, precision);
  if (rc) return rc;
  Carver c(nullptr);
  layout(shape_of(A, K, precision), c, nullptr);
  *bytes = c.off;
  return NMF_OK;
}

int nmf_init(nmf_plan* out, const nmf_matrix* A, int K, float eps, int precision, float* W,
             float* Ht, void* workspace, size_t workspace_bytes, void* stream) {
  if (!out) return fail(NMF_E_ARG, "out is NULL");
  *out = nullptr;
  int rc = check_shape(A, K, precision);
  if (rc) return rc;
  if (!(eps > 0.0f) || std::isinf(eps)) return fail(NMF_E_ARG, "eps must be finite and > 0");
  if (!W || !Ht || !workspace) return fail(NMF_E_ARG, "W, Ht and workspace must be non-NULL");
  if (((uintptr_t)W & 15) || ((uintptr_t)Ht & 15))
    return fail(NMF_E_ARG, "W and Ht must be 16-byte aligned");
  if ((uintptr_t)workspace % kAlign) return fail(NMF_E_ARG, "workspace must be 256-byte aligned");
  const ShapeInfo s = shape_of(A, K, precision);
  Carver probe(nullptr);
  layout(s, probe, nullptr);
  if (workspace_bytes < probe.off)
    return fail(NMF_E_WORKSPACE, "workspace %zu bytes < required %zu", workspace_bytes, probe.off);
  int dev = 0, cus = 0;
  rc = device_check(&dev, &cus);
  if (rc) return rc;

  nmf_plan_s* p = new (std::nothrow) nmf_plan_s();
  if (!p) return fail(NMF_E_ARG, "out of host memory");
  p->device = dev;
  p->cus = cus;
  p->stream = (hipStream_t)stream;
  p->V = s.V;
  p->D = s.D;
  p->nnz = s.nnz;
  p->K = K;
  p->fmt = s.fmt;
  p->prec = precision;
  p->eps = eps;
  p->W = W;
  p->Ht = Ht;
  Carver c(workspace);
  layout(s, c, p);
  hipStream_t st = p->stream;
  auto bail = [&](int code) {
    delete p;
    return code;
  };
#define INITCHECK(expr)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return bail(fail(NMF_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_))); \
  } while (0)

  // W kernel: one group per CU; column groups of at most
  // hals_w_max_rows_per_group() rows each (a count set on request, at least
  // what the rows need)
  int ncol = hals_w_column_groups(s.V, cus);
  if (const char* env = getenv("NMF_W_COLUMN_GROUPS")) {
    const int need = (int)((s.V + hals_w_max_rows_per_group() - 1) / hals_w_max_rows_per_group());
    const int v = atoi(env);
    if (v > 0) ncol = (int)std::min<int64_t>(std::min(std::max(v, need), hals_w_max_column_groups()), s.V);
  }
  const int64_t rpg = hals_w_rows_per_group(s.V, ncol);
  ncol = (int)((s.V + rpg - 1) / rpg);
  if (ncol > hals_w_max_column_groups())
    return bail(fail(NMF_E_UNSUPPORTED, "V=%lld exceeds the W kernel's %d x %d rows",
                     (long long)s.V, hals_w_max_column_groups(), hals_w_max_rows_per_group()));
  const int grid = hals_w_grid(cus, s.V, K, ncol);
  if (grid == 0)
    return bail(fail(NMF_E_UNSUPPORTED,
                     "the W kernel cannot be made resident for V=%lld, K=%d on %d CUs",
                     (long long)s.V, K, cus));
  p->w_grid = grid;
  p->w_groups = ncol;
  p->w_rows_per_group = (int)rpg;

  INITCHECK(hipMemsetAsync(p->status, 0, 16 * sizeof(int32_t), st));
  INITCHECK(hipMemsetAsync(p->slots, 0, kSlotWords * sizeof(unsigned long long), st));
  INITCHECK(hipMemsetAsync(p->w_flags, 0, kWFlagWords * sizeof(unsigned), st));
  INITCHECK(hipMemsetAsync(p->panel, 0, hals_panel_floats(K) * sizeof(float), st));
  INITCHECK(hipMemsetAsync(p->panel_h, 0, p->panel_h_floats * sizeof(float), st));
  // the H update's tile width: NMF_TILE_T = 16, 32 or 64 where supported, else 32
  p->h_tile = kTile;
  if (const char* e = getenv("NMF_TILE_T")) {
    const int t = atoi(e);
    if (hals_tile_supported(K, t)) p->h_tile = t;
  }
  // input checks: W, Ht finite and non-negative; A structure and values
  INITCHECK(check_finite_nonneg(W, s.V * K, p->status, 1, st));
  INITCHECK(check_finite_nonneg(Ht, s.D * K, p->status, 2, st));
  if (s.fmt == NMF_DENSE) {
    p->A_dense = A->dense;
    INITCHECK(check_finite_nonneg(A->dense, s.V * s.D, p->status, 4, st));
  } else {
    p->a_rowptr = A->rowptr;
    p->a_col = A->colidx;
    p->a_val = A->values;
    INITCHECK(csr_validate(s.V, s.D, s.nnz, A->rowptr, A->colidx, A->values, p->status + 1, st));
  }
  int32_t flags[2] = {0, 0};
  INITCHECK(hipMemcpyAsync(flags, p->status, sizeof(flags), hipMemcpyDeviceToHost, st));
  INITCHECK(hipStreamSynchronize(st));
  if (flags[1] & 3) return bail(fail(NMF_E_SHAPE, "CSR structure invalid (code %d)", flags[1]));
  if ((flags[1] & 4) || (flags[0] & 4))
    return bail(fail(NMF_E_NUMERIC, "A has a negative, NaN or Inf entry"));
  if (flags[0] & 3) return bail(fail(NMF_E_NUMERIC, "W or Ht has a negative, NaN or Inf entry"));
  INITCHECK(hipMemsetAsync(p->status, 0, 16 * sizeof(int32_t), st));

  if (s.fmt == NMF_CSR) {
    // CSR of A^T; the count scratch borrows P and R (unused until the first sweep)
    INITCHECK(csr_transpose(s.V, s.D, s.nnz, A->rowptr, A->colidx, A->values, p->t_rowptr, p->t_col,
                            p->t_val, (int32_t*)p->P, p->tr_blocks, st));
    p->sp_A.rows = s.V;
    p->sp_A.nnz = s.nnz;
    p->sp_A.rowptr = A->rowptr;
    p->sp_A.col = A->colidx;
    p->sp_A.val = A->values;
    p->sp_At.rows = s.D;
    p->sp_At.nnz = s.nnz;
    p->sp_At.rowptr = p->t_rowptr;
    p->sp_At.col = p->t_col;
    p->sp_At.val = p->t_val;
    std::vector<uint8_t> skip;
    const int drm = dense_rows_mode();
    if (drm == 1 || (drm < 0 && s.D * (int64_t)K >= kDenseRowsMinDK)) {
      // the densest rows of A (longer than one work item and at least 1/24
      // dense; at most kDenseRowsMax, longest first) are multiplied as a dense
      // block on the matrix cores; the sparse product skips them.  Only when
      // H^T is large (D K >= 32M floats): then each gathered row mostly comes
      // from HBM, and the dense block reads H^T once instead; for a smaller
      // H^T the gathers hit the caches and the split-K product costs more
      // than it saves (measured: 26,000 x 11,000 at K = 200, P 82 -> 147 us)
      std::vector<int32_t> rp((size_t)s.V + 1);
      INITCHECK(hipMemcpyAsync(rp.data(), A->rowptr, rp.size() * sizeof(int32_t),
                               hipMemcpyDeviceToHost, st));
      INITCHECK(hipStreamSynchronize(st));
      std::vector<int32_t> cand;
      for (int64_t r = 0; r < s.V; r++) {
        const int64_t len = (int64_t)rp[r + 1] - rp[r];
        if (len > p->sp_A.L && len * 24 >= s.D) cand.push_back((int32_t)r);
      }
      std::stable_sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) {
        return rp[a + 1] - rp[a] > rp[b + 1] - rp[b];
      });
      if ((int)cand.size() > kDenseRowsMax) cand.resize(kDenseRowsMax);
      std::sort(cand.begin(), cand.end());
      p->n_top = (int)cand.size();
      if (p->n_top > 0) {
        skip.assign((size_t)s.V, 0);
        for (int32_t r : cand) skip[r] = 1;
        INITCHECK(hipMemcpyAsync(p->top_idx, cand.data(), cand.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, st));
        INITCHECK(csr_dense_rows(A->rowptr, A->colidx, A->values, p->top_idx, p->n_top, s.D,
                                 p->a_top, st));
        if (precision == NMF_BF16_PRODUCTS)
          INITCHECK(cast_bf16(p->a_top, p->a_top_bf, (int64_t)p->n_top * s.D, st));
        INITCHECK(hipStreamSynchronize(st));  // cand is a host buffer
      }
    }
    INITCHECK(spmm_build(&p->sp_A, st, skip.empty() ? nullptr : skip.data()));
    INITCHECK(spmm_build(&p->sp_At, st));
    if (precision == NMF_BF16_PRODUCTS) {
      p->sp_A_f32 = p->sp_A;
      INITCHECK(cast_bf16(A->values, p->a_val_bf, s.nnz, st));
      INITCHECK(cast_bf16(p->t_val, p->t_val_bf, s.nnz, st));
      p->sp_A.val = p->a_val_bf;
      p->sp_At.val = p->t_val_bf;
    }
    const int nb = reduce_blocks(s.nnz);
    INITCHECK(sumsq_f64(A->values, s.nnz, p->red, nb, st));
    INITCHECK(finish_f64(p->red, nb, p->scal + 0, st));
  } else {
    if (precision == NMF_BF16_PRODUCTS) {
      INITCHECK(cast_bf16(A->dense, p->A_bf, s.V * s.D, st));
      INITCHECK(cast_bf16_transpose(A->dense, p->At_bf, s.V, s.D, st));
    }
    const int nb = reduce_blocks(s.V * s.D);
    INITCHECK(sumsq_f64(A->dense, s.V * s.D, p->red, nb, st));
    INITCHECK(finish_f64(p->red, nb, p->scal + 0, st));
  }
  // unit-norm columns of W before the first sweep (a column of zero norm has
  // no direction to keep: rejected)
  INITCHECK(normalize_columns(W, s.V, K, p->colsq, 1024, p->status, 8, st));
  INITCHECK(hipStreamSynchronize(st));
  double a2 = 0.0;
  INITCHECK(hipMemcpy(&a2, p->scal, sizeof(double), hipMemcpyDeviceToHost));
  if (!(a2 > 0.0)) return bail(fail(NMF_E_NUMERIC, "A is all zeros"));
  int32_t st0 = 0;
  INITCHECK(hipMemcpy(&st0, p->status, sizeof(st0), hipMemcpyDeviceToHost));
  if (st0 & 8) return bail(fail(NMF_E_NUMERIC, "a column of W has zero norm"));
#undef INITCHECK
  *out = p;
  return NMF_OK;
}

int nmf_half(nmf_plan p, int which) {
  if (!p) return fail(NMF_E_ARG, "plan is NULL");
  if (p->poisoned) return fail(p->poisoned, "plan is poisoned by an earlier error");
  if (which == NMF_HALF_H) return half_h(p);
  if (which == NMF_HALF_W) return half_w(p);
  return fail(NMF_E_ARG, "unknown half %d", which);
}

int nmf_sweep(nmf_plan p, int n_sweeps, double* rel_obj) {
  if (!p) return fail(NMF_E_ARG, "plan is NULL");
  if (p->poisoned) return fail(p->poisoned, "plan is poisoned by an earlier error");
  if (n_sweeps < 0) return fail(NMF_E_ARG, "n_sweeps < 0");
  std::vector<double> host;
  for (int i = 0; i < n_sweeps; i++) {
    int rc = half_h(p);
    if (rc) return rc;
    rc = half_w(p);
    if (rc) return rc;
    p->sweeps_done++;
    if (rel_obj) {
      rc = enqueue_objective(p);
      if (rc) return rc;
      HIPCHECK(p, hipMemcpyAsync(rel_obj + i, p->scal + 4, sizeof(double), hipMemcpyDeviceToHost,
                                 p->stream));
    }
  }
  // the device status word once per call (one 4-byte copy and one
  // synchronisation): a timed-out wait of the W update, here or in an earlier
  // nmf_half, poisons the plan now
  int rc = read_status(p);
  if (rc) return rc;
  if (rel_obj) {
    for (int i = 0; i < n_sweeps; i++)
      if (!std::isfinite(rel_obj[i])) return fail(NMF_E_NUMERIC, "objective is not finite");
  }
  return NMF_OK;
}

int nmf_mu_sweep(nmf_plan p, int n_sweeps, double* rel_obj) {
  if (!p) return fail(NMF_E_ARG, "plan is NULL");
  if (p->poisoned) return fail(p->poisoned, "plan is poisoned by an earlier error");
  if (n_sweeps < 0) return fail(NMF_E_ARG, "n_sweeps < 0");
  for (int i = 0; i < n_sweeps; i++) {
    int rc = mu_half_h(p);
    if (rc) return rc;
    rc = mu_half_w(p);
    if (rc) return rc;
    p->sweeps_done++;
    if (rel_obj) {
      rc = enqueue_objective(p);
      if (rc) return rc;
      HIPCHECK(p, hipMemcpyAsync(rel_obj + i, p->scal + 4, sizeof(double), hipMemcpyDeviceToHost,
                                 p->stream));
    }
  }
  int rc = read_status(p);
  if (rc) return rc;
  if (rel_obj) {
    for (int i = 0; i < n_sweeps; i++)
      if (!std::isfinite(rel_obj[i])) return fail(NMF_E_NUMERIC, "objective is not finite");
  }
  return NMF_OK;
}

int nmf_objective(nmf_plan p, double* half_sq_frob, double* rel_obj) {
  if (!p) return fail(NMF_E_ARG, "plan is NULL");
  if (p->poisoned) return fail(p->poisoned, "plan is poisoned by an earlier error");
  int rc = enqueue_objective(p);
  if (rc) return rc;
  double v[2];
  HIPCHECK(p, hipMemcpyAsync(v, p->scal + 3, sizeof(v), hipMemcpyDeviceToHost, p->stream));
  rc = read_status(p);
  if (rc) return rc;
  if (half_sq_frob) *half_sq_frob = v[0];
  if (rel_obj) *rel_obj = v[1];
  if (!std::isfinite(v[0]) || !std::isfinite(v[1]))
    return fail(NMF_E_NUMERIC, "objective is not finite");
  return NMF_OK;
}

int nmf_intermediates(nmf_plan p, const float** P, const float** Q, const float** R,
                      const float** S) {
  if (!p) return fail(NMF_E_ARG, "plan is NULL");
  if (P) *P = p->P;
  if (Q) *Q = p->Q;
  if (R) *R = p->R;
  if (S) *S = p->S;
  return NMF_OK;
}

int nmf_plan_info(nmf_plan p, nmf_info* info) {
  if (!p || !info) return fail(NMF_E_ARG, "NULL argument");
  info->V = p->V;
  info->D = p->D;
  info->nnz = p->nnz;
  info->K = p->K;
  info->format = p->fmt;
  info->precision = p->prec;
  info->tile = p->h_tile;
  info->w_groups = p->w_groups;
  info->h_groups = (int)((p->D + hals_rows_per_group_h() - 1) / hals_rows_per_group_h());
  info->sweeps_done = p->sweeps_done;
  return NMF_OK;
}

int nmf_inject_status(nmf_plan p, int32_t bits) {
  if (!p) return fail(NMF_E_ARG, "plan is NULL");
  if (bits != NMF_STATUS_TIMEOUT) return fail(NMF_E_ARG, "unknown status bits %d", bits);
  HIPCHECK(p, or_bits(p->status, bits, p->stream));
  return NMF_OK;
}

int nmf_set_stream(nmf_plan p, void* stream) {
  if (!p) return fail(NMF_E_ARG, "plan is NULL");
  p->stream = (hipStream_t)stream;
  return NMF_OK;
}

int nmf_profile(nmf_plan p, int enable) {
  if (!p) return fail(NMF_E_ARG, "plan is NULL");
  p->profiling = enable != 0;
  return NMF_OK;
}

int nmf_profile_read(nmf_plan p, double* ms_total, int64_t* launches) {
  if (!p || !ms_total || !launches) return fail(NMF_E_ARG, "NULL argument");
  HIPCHECK(p, hipStreamSynchronize(p->stream));
  for (int s = 0; s < NMF_STEP_COUNT; s++) {
    double tot = 0.0;
    for (auto& e : p->prof[s]) {
      float ms = 0.0f;
      HIPCHECK(p, hipEventElapsedTime(&ms, e.first, e.second));
      tot += ms;
    }
    ms_total[s] = tot;
    launches[s] = (int64_t)p->prof[s].size();
  }
  prof_clear(p);
  return NMF_OK;
}

int nmf_destroy(nmf_plan p) {
  if (p) prof_clear(p);
  delete p;
  return NMF_OK;
}

}  // extern "C"
