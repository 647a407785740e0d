/* PL-NMF-cpu: the paper's tiled FAST-HALS on the host, in FP64 with OpenMP
 * threads (Sec. 4.1, Alg. 2, Eq. 4-6; the CPU implementation of Sec. 6 and
 * Table 5).  A comparison baseline beside the GPU library (libplnmf.so): it is
 * a separate library (libplnmf_cpu.so) with its own entry points, and nothing
 * in the GPU library calls it.
 *
 * One sweep is Alg. 1's H half then W half.  Each half forms its product (R =
 * A^T W over a CSR of A^T built here, or P = A H^T) and its Gram matrix, then
 * updates the factor in the three phases of Alg. 2: with tiles of T columns,
 * phase 1 (Eq. 4) subtracts every tile's old values from the columns left of
 * it, phase 2 (Eq. 5, +P as in Alg. 2) walks the tile column by column (clip
 * at eps; for W also normalise the column over all rows), phase 3 (Eq. 6)
 * subtracts the finished tile from the columns right of it.  The H half is
 * the same without normalisation (Sec. 4.1).  Rows are processed in blocks so
 * that each Gram row is streamed once per block.  Reductions (Gram matrices,
 * column norms, objective) use a fixed number of row chunks summed in chunk
 * order, so results do not depend on the thread count.
 *
 * Layouts: W [V, K] and Ht = H^T [D, K] row-major FP64, owned by the caller and
 * updated in place; A is copied (FP64) at init.  All calls are synchronous.
 * Status: 0 ok, -1 bad argument, -2 bad shape/structure, -5 numeric.       */
#ifndef PLNMF_CPU_H
#define PLNMF_CPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nmf_cpu_plan_s* nmf_cpu_plan;

/* A as CSR (rowptr [V+1], col [nnz] sorted per row, val [nnz]) or, with
 * rowptr == NULL, dense [V, D] row-major in `val`.  FP32 values (the library's
 * input type), read once and widened.  K in [1, min(V, D)], eps > 0, tile in
 * [1, K] (0: the Sec. 5 model's choice, the nearest integer to sqrt(K)),
 * threads >= 1 (0: all available).  W's columns are normalised here (the same
 * initialisation reading as the GPU library).                                */
int nmf_cpu_init(nmf_cpu_plan* out, int64_t V, int64_t D, const int32_t* rowptr,
                 const int32_t* col, const float* val, int K, double eps, int tile, int threads,
                 double* W, double* Ht);
/* n_sweeps sweeps; rel_obj (host [n_sweeps] or NULL) receives the relative
 * objective sqrt(sum (A-WH)^2 / sum A^2) after each sweep.                   */
int nmf_cpu_sweep(nmf_cpu_plan plan, int n_sweeps, double* rel_obj);
/* The tile width and thread count in use.                                    */
int nmf_cpu_info(nmf_cpu_plan plan, int* tile, int* threads);
int nmf_cpu_destroy(nmf_cpu_plan plan);

#ifdef __cplusplus
}
#endif
#endif
