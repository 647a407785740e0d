/*
 * nmf.h -- C ABI of the MI355X FAST-HALS library (PL-NMF hot path).
 *
 * The library factorises a non-negative A (V x D, dense or CSR) as A ~= W H with
 * W (V x K) and H (K x D) by FAST-HALS (Alg. 1 of arXiv 1904.07935), with the
 * K-sequential column updates reordered into tiles (Sec. 3.3, Alg. 2, Eq. 4-6)
 * so that all cross-tile work runs as matrix products on the matrix cores.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - All matrix pointers are DEVICE pointers (memory of the current HIP device),
 *   caller-allocated and caller-owned.  The library never allocates or frees
 *   device memory; it keeps raw pointers inside a plan, so they must outlive it.
 * - Layouts are row-major.  W is [V, K]; the library stores H transposed as
 *   Ht [D, K] (row d holds document d's K weights), so that every row of both
 *   factors is K-contiguous.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is
 *   enqueued on it; only calls that return host values, and nmf_sweep (which
 *   reads the device status word once per call), synchronise it.
 * - Every call returns an int status (nmf_status).  No exception crosses the
 *   ABI.  On error, nmf_last_error() returns a thread-local message.  After a
 *   HIP runtime error or a device-side timeout a plan is poisoned and every
 *   later call on it returns the same status.
 * - Floating-point: products, Gram matrices and updates in FP32 (or BF16
 *   inputs with FP32 accumulation for the two products when the plan's
 *   precision is NMF_BF16_PRODUCTS); objective reductions in FP64.  All
 *   reductions are fixed-order: results are bitwise reproducible for a given
 *   device, shape and precision.
 */
#ifndef PLNMF_NMF_H
#define PLNMF_NMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NMF_MAX_K 512

typedef enum nmf_status {
  NMF_OK = 0,
  NMF_E_ARG = -1,         /* null pointer, bad enum, eps <= 0, misaligned pointer   */
  NMF_E_SHAPE = -2,       /* K outside [1, min(V, D, NMF_MAX_K)], bad CSR structure  */
  NMF_E_WORKSPACE = -3,   /* workspace smaller than the size query returned          */
  NMF_E_HIP = -4,         /* HIP runtime error, or no usable device                  */
  NMF_E_NUMERIC = -5,     /* NaN/Inf in an input or an objective                     */
  NMF_E_UNSUPPORTED = -6, /* valid request this build does not implement             */
  NMF_E_TIMEOUT = -7      /* a device-side bounded wait expired (co-residency lost)  */
} nmf_status;

typedef enum nmf_format { NMF_DENSE = 0, NMF_CSR = 1 } nmf_format;

typedef enum nmf_precision {
  NMF_FP32 = 0,          /* every step in FP32                                      */
  NMF_BF16_PRODUCTS = 1  /* A^T W and A H^T with BF16 inputs, FP32 accumulation     */
} nmf_precision;

typedef enum nmf_half_kind { NMF_HALF_H = 0, NMF_HALF_W = 1 } nmf_half_kind;

/* A matrix handed across the boundary (device memory, caller-owned).
 * DENSE: `dense` is [rows, cols] row-major, 16-byte aligned, leading dim = cols.
 * CSR:   `rowptr` [rows+1] (rowptr[0] = 0, non-decreasing, rowptr[rows] = nnz),
 *        `colidx` [nnz] in [0, cols), strictly increasing within each row,
 *        `values` [nnz]; entries must be finite and >= 0.                        */
typedef struct nmf_matrix {
  int64_t rows;
  int64_t cols;
  int64_t nnz;
  int32_t format; /* nmf_format */
  const float* dense;
  const int32_t* rowptr;
  const int32_t* colidx;
  const float* values;
} nmf_matrix;

typedef struct nmf_plan_s* nmf_plan;

/* Read-only facts about a plan (host struct filled by nmf_plan_info). */
typedef struct nmf_info {
  int64_t V, D, nnz;
  int32_t K, format, precision;
  int32_t tile;           /* tile width T of the column-update kernels              */
  int32_t w_groups;       /* column groups (phase 2, norm exchange) of the W kernel  */
  int32_t h_groups;       /* workgroups of the H-update kernel                      */
  int64_t sweeps_done;
} nmf_info;

/* Bytes of device workspace nmf_init needs for this problem (no device work). */
int nmf_workspace_bytes(const nmf_matrix* A, int K, int precision, size_t* bytes);

/* Create a plan for A ~= W H (Alg. 1, initialisation step).
 *   A          problem matrix (V x D), read at every sweep; not modified.
 *   W [V,K]    in: random non-negative init; out: columns scaled to unit L2 norm
 *              (the reading that makes Alg. 1's H update an exact minimiser).
 *   Ht [D,K]   in: random non-negative init of H, transposed; not modified here.
 *   eps        the clip value of Alg. 1 (> 0, finite).
 *   workspace  >= nmf_workspace_bytes(), 256-byte aligned; holds P, Q, R, S, the
 *              transposed CSR, BF16 copies and reduction scratch; owned by the
 *              caller and bound to the plan until nmf_destroy.
 * Validates shapes, alignment and (for CSR) the index structure on the device,
 * builds the CSR of A^T, computes ||A||_F^2.  Synchronises `stream`.
 * Errors: NMF_E_NUMERIC for a negative/NaN/Inf entry of A, W or Ht, for an
 * all-zero A, or for a column of W with zero norm (it cannot be normalised);
 * NMF_E_UNSUPPORTED when the W update cannot hold V rows with all its
 * workgroups resident: at most 128 column groups of 1,792 rows, each with at
 * least one product group, one workgroup per CU (V <= 229,376 on 256 CUs).  */
int nmf_init(nmf_plan* out, const nmf_matrix* A, int K, float eps, int precision,
             float* W, float* Ht, void* workspace, size_t workspace_bytes, void* stream);

/* Run n_sweeps outer iterations of Alg. 1 (H half, then W half) in place on the
 * plan's W and Ht.  If rel_obj is non-NULL it receives, per sweep, the relative
 * objective sqrt(sum (A-WH)^2 / sum A^2) of Sec. 6.2 after that sweep.  Every
 * call ends by reading the device status word (one 4-byte copy, one stream
 * synchronisation): a W update whose device-side wait timed out -- in this
 * call or in an earlier nmf_half -- returns NMF_E_TIMEOUT and poisons the
 * plan.  A non-finite objective returns NMF_E_NUMERIC.                       */
int nmf_sweep(nmf_plan plan, int n_sweeps, double* rel_obj);

/* The multiplicative-update baseline (MU; Sec. 2.1 names it, after Lee and
 * Seung, as the simplest NMF algorithm and the slower-converging comparator of
 * Sec. 6.3): n_sweeps iterations of
 *   H <- H * (W^T A) / (W^T W H + eps),   then   W <- W * (A H^T) / (W H H^T + eps)
 * (elementwise; eps is the plan's) on the plan's W and Ht, with the same
 * products, Grams, precision and objective as nmf_sweep and the same
 * synchronisation and error behaviour.  W is not normalised (MU does not need
 * it); a plan may mix nmf_sweep and nmf_mu_sweep.                            */
int nmf_mu_sweep(nmf_plan plan, int n_sweeps, double* rel_obj);

/* Run one half of a sweep: NMF_HALF_H forms R = A^T W and S = W^T W and updates
 * every row of H (Alg. 1, H loop); NMF_HALF_W forms P = A H^T and Q = H H^T and
 * updates every column of W with normalisation (Alg. 1, W loop).  Enqueue only:
 * a device-side timeout of its W update is reported by the next nmf_sweep or
 * nmf_objective on the plan.                                                  */
int nmf_half(nmf_plan plan, int which);

/* Objective of Eq. 2, 0.5 ||A - W H||_F^2, and the relative objective of
 * Sec. 6.2 for the plan's current W, Ht.  Dense A: explicit residual, FP32
 * terms, FP64 sums.  CSR A: ||A||^2 - 2<W, A H^T> + <W^T W, H H^T> with FP64
 * sums.  Either output pointer may be NULL.  Synchronises the stream.         */
int nmf_objective(nmf_plan plan, double* half_sq_frob, double* rel_obj);

/* Device pointers to the products and Gram matrices of the last half-sweeps:
 * P [V,K] = A H^T and Q [K,K] = H H^T (last W half), R [D,K] = A^T W and
 * S [K,K] = W^T W (last H half).  Valid until the next call on the plan.      */
int nmf_intermediates(nmf_plan plan, const float** P, const float** Q, const float** R,
                      const float** S);

int nmf_plan_info(nmf_plan plan, nmf_info* info);

/* Per-step timing with HIP events recorded on the plan's stream around each
 * step of nmf_sweep / nmf_half.  Steps: */
#define NMF_STEP_GRAM_S 0    /* S = W^T W                       (H half)       */
#define NMF_STEP_PRODUCT_R 1 /* R = A^T W, incl. BF16 operand cast            */
#define NMF_STEP_UPDATE_H 2  /* tiled H update: one kernel launch             */
#define NMF_STEP_PRODUCT_P 3 /* P = A H^T, incl. BF16 operand cast   (W half) */
#define NMF_STEP_GRAM_Q 4    /* Q = H H^T                                     */
#define NMF_STEP_UPDATE_W 5  /* persistent tiled W update: one kernel launch  */
#define NMF_STEP_COUNT 6
/* enable != 0 starts recording (events are created by the library and freed
 * by nmf_profile_read or nmf_destroy); enable == 0 stops.                    */
int nmf_profile(nmf_plan plan, int enable);
/* Sum of event-timed milliseconds and number of recorded launches per step
 * (host arrays of NMF_STEP_COUNT) since the last read; synchronises the
 * stream and resets the record.                                              */
int nmf_profile_read(nmf_plan plan, double* ms_total, int64_t* launches);
int nmf_set_stream(nmf_plan plan, void* stream);
/* Fault injection for tests of the error paths: ORs `bits` into the plan's
 * device status word, in stream order.  The only accepted value is
 * NMF_STATUS_TIMEOUT, the bit a timed-out device-side wait sets: the next W
 * update's bounded waits then give up at once (every kernel still runs to its
 * end; the factors are left unspecified) and the next nmf_sweep or
 * nmf_objective returns NMF_E_TIMEOUT and poisons the plan.                  */
#define NMF_STATUS_TIMEOUT 256
int nmf_inject_status(nmf_plan plan, int32_t bits);
int nmf_destroy(nmf_plan plan);
const char* nmf_last_error(void);

/* ------------------------------------------------------------- fold-in ----
 * H-only FAST-HALS for new documents with the plan's W fixed (the H half of
 * Alg. 1 repeated with R' = A_new^T W and S = W^T W formed once).
 *   AnewT     the new documents as a matrix with one ROW per document:
 *             D' x V (CSR or dense).
 *   Ht_new    [D', K] inout.  Initialised according to init_mode:
 *               NMF_FOLDIN_GIVEN  use Ht_new as passed (e.g. a cold U[0,1) draw)
 *               NMF_FOLDIN_WTA    max(eps, A_new^T W)   (non-learned warm start)
 *               NMF_FOLDIN_MLP    ||r|| * mlp(r / ||r||), r = row of A_new^T W,
 *                                 with the network in `mlp_params`
 *   max_sweeps  H-only sweeps to run at most after the initialisation.
 *   tol       0: run exactly max_sweeps sweeps (no per-sweep synchronisation).
 *             > 0: stop after the first sweep that lowers the relative
 *             objective of the fold-in problem by less than tol (absolute, in
 *             relative-objective units); the objective is then computed and
 *             read back after every sweep (one synchronisation per sweep).
 *   sweeps_done  host int or NULL: the number of sweeps run.
 *   rel_trace host [max_sweeps+1] or NULL: relative objective of the fold-in
 *             problem after initialisation (index 0) and after each sweep run
 *             (entries past *sweeps_done are left untouched); computed on the
 *             device (synchronises).
 *   workspace >= nmf_foldin_workspace_bytes().
 * Errors: NMF_E_ARG (tol < 0 or not finite, bad mode), NMF_E_SHAPE (the new
 * documents' CSR structure or V), NMF_E_NUMERIC (negative/NaN entries, or a
 * non-finite objective when tol > 0).                                        */
#define NMF_FOLDIN_GIVEN 0
#define NMF_FOLDIN_WTA 1
#define NMF_FOLDIN_MLP 2
int nmf_foldin_workspace_bytes(nmf_plan plan, const nmf_matrix* AnewT, int mlp_hidden,
                               size_t* bytes);
int nmf_foldin(nmf_plan plan, const nmf_matrix* AnewT, float* Ht_new, int init_mode,
               const void* mlp_params, int mlp_hidden, int max_sweeps, double tol,
               int* sweeps_done, double* rel_trace, void* workspace, size_t workspace_bytes);

/* nmf_foldin without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation).  The workspace is a device array owned by the library:
 * NMF_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, reserved when the library's code
 * is loaded on that GPU and held until the process ends; its address is looked
 * up on the first call on each device.  Arguments, results and errors are those
 * of nmf_foldin, plus:
 *   NMF_E_WORKSPACE  nmf_foldin_workspace_bytes() for these documents exceeds
 *                    NMF_NOALLOC_SCRATCH_BYTES (fold the documents in smaller
 *                    batches, or call nmf_foldin);
 *   NMF_E_ARG        the current device is not the plan's.
 * The call allocates no device memory.  Every call on a GPU uses the same
 * array and leaves its contents behind (each call clears what it needs
 * zeroed): calls that overlap on one GPU -- on different streams, or from
 * different host threads -- race and give unspecified results.             */
#define NMF_NOALLOC_SCRATCH_BYTES (64ull << 20)
int nmf_foldin_noalloc(nmf_plan plan, const nmf_matrix* AnewT, float* Ht_new, int init_mode,
                       const void* mlp_params, int mlp_hidden, int max_sweeps, double tol,
                       int* sweeps_done, double* rel_trace);

/* ------------------------------------------------- warm-start network ----
 * y = softplus(W2 GELU(W1 x + b1) + b2), x in R^K, hidden units `hidden`
 * (GELU erf form; softplus(z) = z for z > 20).  Parameter blob (device, caller
 * allocated, nmf_mlp_param_bytes), byte offsets in nmf_mlp_layout:
 *   FP32 masters W1 [hidden,K], b1 [hidden], W2 [K,hidden], b2 [K] (contiguous,
 *   in this order), Adam moments m and v (same layout), BF16 working copies of
 *   W1 and W2 used by the forward/backward products, and the Adam step count.
 * Training: mean-squared error over all N*K outputs, Adam (beta 0.9/0.999,
 * eps 1e-8), gradients from the library's own backward kernels.            */
typedef struct nmf_mlp_layout {
  size_t master, n_master;     /* byte offset of FP32 masters, float count   */
  size_t adam_m, adam_v;       /* byte offsets (n_master floats each)        */
  size_t w1_bf16, w2_bf16;     /* byte offsets of BF16 working copies        */
  size_t step;                 /* byte offset of the int64 Adam step count   */
  size_t total;
} nmf_mlp_layout;

int nmf_mlp_param_bytes(int K, int hidden, nmf_mlp_layout* layout);
/* Seeded fan-in uniform init U(-1/sqrt(fan_in), 1/sqrt(fan_in)) of masters from a
 * counter-based generator (SplitMix64 of seed and element index); zero Adam. */
int nmf_mlp_init(void* params, int K, int hidden, uint64_t seed, void* stream);
/* Re-derive the BF16 working copies from the FP32 masters (round to nearest
 * even) and zero the Adam state; call after writing masters directly.        */
int nmf_mlp_refresh(void* params, int K, int hidden, void* stream);
int nmf_mlp_workspace_bytes(int K, int hidden, int64_t batch, size_t* bytes);
/* Yhat [N,K] = network(X [N,K]); FP32 in/out, batched internally.            */
int nmf_mlp_predict(const void* params, int K, int hidden, const float* X, float* Yhat,
                    int64_t N, void* workspace, size_t workspace_bytes, void* stream);
/* Loss and gradients of one batch (N <= the batch the workspace was sized for):
 * grads has the layout of the FP32 masters.  *loss (host) synchronises.      */
int nmf_mlp_loss_grad(const void* params, int K, int hidden, const float* X, const float* Y,
                      int64_t N, float* grads, double* loss, void* workspace,
                      size_t workspace_bytes, void* stream);
/* One Adam step on the masters with `grads`, then refresh the BF16 copies.    */
int nmf_mlp_adam_step(void* params, int K, int hidden, const float* grads, float lr,
                      void* stream);
/* `epochs` passes of minibatch Adam over (X [N,K], Y [N,K]) in a seeded shuffled
 * order; epoch_loss (host [epochs] or NULL) gets the mean batch loss.         */
int nmf_mlp_train(void* params, int K, int hidden, const float* X, const float* Y, int64_t N,
                  int epochs, int batch, float lr, uint64_t seed, void* workspace,
                  size_t workspace_bytes, double* epoch_loss, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PLNMF_NMF_H */
