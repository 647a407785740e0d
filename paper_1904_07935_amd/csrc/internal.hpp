// Internal declarations shared by the host plan code and the kernel files.
// Not part of the public ABI (include/nmf.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace plnmf {

// Activations of the warm-start network, shared by the GEMM epilogues and the
// fused inference kernel.
// erf(x) by Abramowitz and Stegun's rational approximation 7.1.26
// (|error| <= 1.5e-7), branch-free with the hardware exponential: the GELU
// epilogue runs on every hidden activation, and its outputs are rounded to
// BF16 (2^-9) right after.
__device__ __forceinline__ float erf_as(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * ax);  // hardware reciprocal, 1 ulp
  const float poly =
      t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f +
                                                                        t * 1.061405429f))));
  const float y = 1.0f - poly * __expf(-ax * ax);
  return copysignf(y, x);
}
__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.0f + erf_as(z * 0.70710678118654752f));
}
// softplus(z) = max(z, 0) + log1p(exp(-|z|)), with log1p(u) = log(w) u / (w - 1),
// w = 1 + u rounded (exact to a few ulp; Goldberg's correction), on the
// hardware exponential and logarithm: the library log1pf expands to a long
// compensated sequence, and this runs on every output of the network.
__device__ __forceinline__ float softplus_f(float z) {
  const float u = __expf(-fabsf(z));
  const float w = 1.0f + u;
  const float l = w == 1.0f ? u : __logf(w) * u * __builtin_amdgcn_rcpf(w - 1.0f);
  return fmaxf(z, 0.0f) + l;
}


typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxK = 512;
constexpr int kTile = 32;          // tile width T of the column-update kernels
constexpr int kSpinLimit = 1 << 21; // bounded waits: a few seconds of polling at most
constexpr int kSlotReplicas = 1;    // copies of the column-norm exchange slots
constexpr int kSlotStride = 2 * 1024 + 16;  // u64 elements between replicas
constexpr int kSlotWords = kSlotReplicas * kSlotStride;

// ------------------------------------------------------------------ GEMM ----
// C[M,N] = sum_k A(m,k) B(k,n) with FP32 accumulation on the matrix cores.
// A(m,k) = A[m*lda + k] (a_trans = false) or A[k*lda + m] (a_trans = true);
// B(k,n) = B[k*ldb + n] (b_trans = false) or B[n*ldb + k] (b_trans = true).
enum GemmEpi : int {
  EPI_STORE = 0,      // C = acc (+ bias[n])
  EPI_RESID_SQ = 1,   // red_out[tile] = sum (D - acc)^2 over the tile (FP64)
  EPI_BIAS_GELU = 2,  // C = acc + bias (pre-activation, FP32; skipped if C is NULL); C2 (bf16) = GELU(C)
  EPI_BIAS_SOFTPLUS = 3, // C = acc + bias (FP32; skipped if NULL); C2 (float) = softplus(C)
  EPI_GELU_GRAD = 4,  // C (FP32, if set) and C2 (bf16) = acc * GELU'(D), D = z1
  EPI_MU = 5,         // C = D * X / (acc + mu_delta), X = (const float*)C2 (ld = ldc);
                      // C may be D (each element is read, then written, by one thread)
};

struct GemmArgs {
  const void* A;
  const void* B;
  int64_t M, N, Kd;
  int64_t lda, ldb;
  float* C;
  int64_t ldc;
  int epi;
  const float* bias;
  const float* D;  // EPI_RESID_SQ: reference matrix; EPI_GELU_GRAD: z1
  int64_t ldd;
  void* C2;        // secondary output (ld = ldc)
  double* red_out; // EPI_RESID_SQ partials, one per tile
  int splits;      // split-K factor (EPI_STORE only); >1 needs `partial`
  int64_t k_per_split;
  float* partial;  // [splits][M][N]
  int sym;         // 1: C is symmetric (M == N, op(A) = op(B)^T): upper tiles, mirrored
  float mu_delta;  // EPI_MU: added to the denominator
};

enum class Elem { F32, BF16 };

// Launch one GEMM.  Chooses tile/vector variants; returns hipError.
hipError_t gemm(Elem t, bool a_trans, bool b_trans, const GemmArgs& g, hipStream_t s);
// Pick a split-K factor and return partial-buffer floats needed (0 if none).
int gemm_pick_splits(int64_t M, int64_t N, int64_t Kd, int64_t* k_per_split);
// C[M,N] (ldc) = sum_z partial[z] (+ bias[n])
hipError_t splitk_reduce(const float* partial, int splits, int64_t M, int64_t N, float* C,
                         int64_t ldc, const float* bias, int sym, hipStream_t s);

// ------------------------------------------------------------------ Gram ----
// C[K][K] (ldc) = X^T X for X [rows, K] row-major, K <= kMaxK; deterministic.
int gram_chunks(int64_t rows, int device_cus);  // <= gram_max_chunks()
int gram_max_chunks();
size_t gram_partial_floats(int K, int chunks);
// With `panel` set, also writes the tile panels of the column updates derived
// from C (hals_panel_floats(K) floats; entries that never depend on C -- rows
// >= K, and outside the last tile -- must have been zeroed once), in the
// [tile][row][column] order with the tiles' G blocks after them, or with
// `rows_layout` in the H rows kernel's staging order (hals_h_rows_layout).
hipError_t gram_xtx(const float* X, int64_t rows, int K, float* C, int64_t ldc, float* partial,
                    int chunks, hipStream_t s, float* panel = nullptr, int diag_one = 0,
                    int tile = 32, bool rows_layout = false);

// ------------------------------------------------------------------ SpMM ----
// out[r, 0:K] = sum_j val[j] X[col[j], 0:K] over the rows of a CSR matrix.
// Work items (one wave each), planned on the host by spmm_build: runs of short
// rows holding about L nonzeros, or one segment of L nonzeros of a long row;
// segments leave partial rows in `carry` that a fixed-order pass adds up.
struct SpmmPlan {
  int64_t rows, nnz;
  const int32_t* rowptr;
  const int32_t* col;
  const void* val;        // float or bf16 (elem)
  int L;                  // target nonzeros per work item
  int4* items;            // [n_items] (first row, end row, first nz, end nz)
  int32_t* item_slot;     // [n_items] carry row of a segment, or -1
  int64_t n_items;
  int32_t* fix;           // [n_fix][3] (row, first segment, segments)
  int64_t n_fix;
  float* carry;           // [n_seg][K]
  int64_t n_seg;
};
struct SpmmSizes {
  int64_t items, fix, seg;  // upper bounds for any row structure
};
int spmm_item_nnz(int64_t nnz);
SpmmSizes spmm_sizes(int64_t rows, int64_t nnz, int L);
// Copies the row pointers to the host, plans the items, uploads them
// (synchronises the stream).  Device buffers must be sized by spmm_sizes.
// Rows r with skip[r] != 0 (host array, optional) that are longer than L get
// no items: their output rows are left to the caller.
hipError_t spmm_build(SpmmPlan* p, hipStream_t s, const uint8_t* skip = nullptr);
// Dense copy of selected CSR rows: out[i][:] = row rows[i] of the CSR
// (out [n, cols] zeroed first); and the scatter of product rows back:
// dst[rows[i]][:] = src[i][:] (K columns).
hipError_t csr_dense_rows(const int32_t* rowptr, const int32_t* col, const float* val,
                          const int32_t* rows, int n, int64_t cols, float* out, hipStream_t s);
hipError_t scatter_rows(const float* src, const int32_t* rows, int n, int K, float* dst,
                        hipStream_t s);
hipError_t spmm(const SpmmPlan& p, Elem t, const void* X, int K, float* out, hipStream_t s);
// Columns [k0, k0 + K) only: out[r, k0 + c] = sum_j a[r, j] X[col_j, k0 + c],
// X rows ldx apart, out rows ldo apart.
hipError_t spmm_slice(const SpmmPlan& p, Elem t, const void* X, int64_t ldx, int k0, int K,
                      float* out, int64_t ldo, hipStream_t s);

// CSR transpose (rows x cols -> cols x rows), deterministic, rows sorted.
// scratch: int32 [nblk * cols] (nblk from csr_transpose_blocks).
int csr_transpose_blocks(int64_t rows, int64_t cols, size_t scratch_ints);
hipError_t csr_transpose(int64_t rows, int64_t cols, int64_t nnz, const int32_t* rowptr,
                         const int32_t* col, const float* val, int32_t* t_rowptr, int32_t* t_col,
                         float* t_val, int32_t* scratch, int nblk, hipStream_t s);
// Structure check: sets flag bits (1 rowptr, 2 col range/order, 4 value) in *flag.
hipError_t csr_validate(int64_t rows, int64_t cols, int64_t nnz, const int32_t* rowptr,
                        const int32_t* col, const float* val, int32_t* flag, hipStream_t s);

// ----------------------------------------------------------- elementwise ----
// Scales every column of X [rows, K] to unit L2 norm; a column of zero norm
// is left as it is and sets `bit` in *flag.
hipError_t normalize_columns(float* X, int64_t rows, int K, double* part, int nblk_max,
                             int32_t* flag, int bit, hipStream_t s);
hipError_t cast_bf16(const float* x, __bf16* y, int64_t n, hipStream_t s);
// y[c][r] = bf16(x[r][c]) for x [rows, cols]
hipError_t cast_bf16_transpose(const float* x, __bf16* y, int64_t rows, int64_t cols,
                               hipStream_t s);
hipError_t check_finite_nonneg(const float* x, int64_t n, int32_t* flag, int bit, hipStream_t s);
// *word |= bits, on the device, in stream order.
hipError_t or_bits(int32_t* word, int32_t bits, hipStream_t s);

// FP64 fixed-order reductions.  partial buffers are [nblk] doubles.
int reduce_blocks(int64_t n);
hipError_t sumsq_f64(const float* x, int64_t n, double* partial, int nblk, hipStream_t s);
hipError_t dot_f64(const float* x, const float* y, int64_t n, double* partial, int nblk,
                   hipStream_t s);
hipError_t finish_f64(const double* partial, int n, double* out, hipStream_t s);
// out[0] = a2 + c1 * x[0] + c2 * y[0] ... combine for the sparse identity
hipError_t combine_objective(const double* a2, const double* wp, const double* sq,
                             double* out_half, double* out_rel, hipStream_t s);

// --------------------------------------------------------- HALS updates ----
// One tiled half-sweep over the rows of X [rows, K] (in place):
//   acc[r,t] = Bterm[r,t] + X[r,t] * cdiag(t) - sum_{l != t} Xcur[r,l] G[l,t]
//   X[r,t]   = max(eps, acc[r,t])       (W half: then divided by the column norm)
// cdiag = 1 - G[t,t] for the H update and 0 for the W update.
struct HalsArgs {
  float* X;
  const float* Bterm;
  const float* G;
  int64_t rows;
  int K;
  float eps;
  int diag_one;          // 1: H update (cdiag = 1 - G_tt); 0: no diagonal term
  const float* panel;    // tile panels of G (gram_xtx with panel output, diag_one and tile as here)
  const float* gblk;     // set by hals_update
  int tile;              // tile width: 32 (0 = 32), 16 or 64 (see hals_tile_supported)
  int rows_layout;       // panel written in the rows kernel's order: that kernel runs
};
// Row-independent update (no normalisation): the H half and fold-in.
hipError_t hals_update(const HalsArgs& a, hipStream_t s);
size_t hals_panel_floats(int K, int tile = 32);
// Whether the H update of `rows` rows takes the rows-in-registers kernel (so
// its Gram writes the panel in that kernel's staging order): decided once by
// the caller, passed to gram_xtx and to hals_update (HalsArgs::rows_layout).
bool hals_h_rows_layout(int64_t rows, int K, int cus, int tile);
// Tile widths of the H update: 32 always; 16 and 64 when K % 4 == 0 and the
// rows-in-registers kernel's double-buffered panel fits the LDS.
bool hals_tile_supported(int K, int tile);
int hals_rows_per_group_h();

constexpr int kWFlagCol = 1024;  // column-group flags follow the product-group flags
constexpr int kWFlagWords = 2 * kWFlagCol;

// The W half: column groups (phase 2, norm exchange) and product groups in one
// cooperative launch of `grid` groups (see hals_w_grid).
struct HalsWArgs {
  float* X;                   // W [rows, K], in place
  const float* Bterm;         // P [rows, K]
  const float* G;             // Q [K, K]
  int64_t rows;
  int K;
  float eps;
  float* Y;                   // [ceil(K/32)][rows][32] hand-off: each tile's product
  float* Wn;                  // [ceil(K/32)][rows][32] hand-off: each tile's new columns
  unsigned long long* slots;  // kSlotWords tagged partials of the norm exchange
  unsigned* flags;            // kWFlagWords tile flags (product, then column groups)
  int n_col;                  // column groups, 1 <= n_col <= grid / 2
  int rows_per_group;         // rows per column group (hals_w_rows_per_group)
  unsigned epoch;             // distinct per launch (tags of slots and flags)
  int32_t* status;            // bit 8 set on a wait timeout
  const float* panel;         // tile panels of Q (gram_xtx with panel output, diag_one 0)
  int jobs_per_wave;          // set by hals_w_update
  int jobs_parked;            // of those, parked in LDS before the wait (set by hals_w_update)
};
hipError_t hals_w_update(const HalsWArgs& a, int grid, hipStream_t s);
int hals_w_max_rows_per_group();
int hals_w_column_groups(int64_t rows, int device_cus);
// Rows per column group for n_col groups: a multiple of 32.
int hals_w_rows_per_group(int64_t rows, int n_col);
int hals_w_max_column_groups();
// Cooperative grid for this shape (one group per CU), or 0 if the kernel
// cannot be made resident (LDS or occupancy).
int hals_w_grid(int device_cus, int64_t rows, int K, int n_col);

// ----------------------------------------------------------------- MLP ----
hipError_t mlp_init_params(float* master, int64_t n, int K, int hidden, uint64_t seed,
                           hipStream_t s);
hipError_t mlp_adam(float* master, float* m, float* v, const float* g, int64_t n, float lr,
                    int64_t* step, hipStream_t s);
hipError_t acc_scaled(double* acc, const double* v, double scale, hipStream_t s);
hipError_t mlp_out_grad(const float* z2, const float* yhat, const float* y, int64_t n,
                        float scale, __bf16* dz2_bf16, float* dz2_f32, double* loss_partial,
                        int nblk, hipStream_t s);
constexpr int kColSlices = 32;  // row slices of a column sum (part: kColSlices x cols doubles)
hipError_t col_sum(const float* x, int64_t rows, int64_t cols, float* out, double* part,
                   hipStream_t s);

hipError_t gather_rows(const float* x, const int32_t* idx, int64_t n, int64_t cols, float* out,
                       hipStream_t s);
hipError_t row_normalize(const float* x, int64_t rows, int64_t cols, float* xn, float* norms,
                         hipStream_t s);
// The network's fused inference for fold-in: out = max(eps, ||r|| softplus(W2
// GELU(W1 r/||r|| + b1) + b2)) per row r of R [N, K]; BF16 weights.  Only for
// K % 8 == 0, K <= 208, hidden % 32 == 0 (mlp_infer_fused_ok).
bool mlp_infer_fused_ok(int K, int H);
hipError_t mlp_infer_fused(const float* R, int64_t N, int K, int H, const __bf16* W1b,
                           const float* b1, const __bf16* W2b, const float* b2, float eps,
                           float* out, hipStream_t s);
hipError_t rescale_clip_rows(const float* y, const float* norms, int64_t rows, int64_t cols,
                             float eps, float* out, hipStream_t s);
hipError_t clip_min(const float* x, int64_t n, float eps, float* out, hipStream_t s);

}  // namespace plnmf
