// Sparse products of the sweep on CSR inputs: R = A^T W (over the CSR of A^T,
// gathering rows of W) and P = A H^T (over the CSR of A, gathering rows of
// Ht); the sparse-matrix/dense-matrix products of Alg. 1 (R and P statements)
// and of the GPU implementation in Sec. 4.2.
//
// Design: the nnz range is cut into equal chunks, one wave per chunk, so the
// Zipf-skewed row lengths of a term-by-document matrix do not unbalance the
// grid.  Each nnz gathers one K-contiguous factor row with 16-byte (FP32) or
// 8-byte (BF16) lane loads; several nnz are in flight per wave.  Rows that cross
// a chunk boundary leave per-chunk partials in a carry buffer that a second,
// fixed-order pass adds up, and that pass also zeroes empty rows: no atomics,
// bitwise-reproducible results.
#include "internal.hpp"

namespace plnmf {
namespace {

struct SpmmKArgs {
  const int32_t* rowptr;
  const int32_t* col;
  const void* val;
  const int32_t* chunk_row;
  const void* X;
  float* out;
  float* carry;
  int64_t nnz;
  int64_t nchunks;
  int chunk;
  int K;
};

template <typename T>
__device__ __forceinline__ float ld_val(const void* p, int64_t j) {
  return (float)((const T*)p)[j];
}

// Load 4 consecutive elements of a factor row (columns c..c+3) as floats.
template <typename TX, bool VEC>
__device__ __forceinline__ floatx4 ld_x4(const TX* row, int c, int K) {
  floatx4 r;
  if constexpr (VEC) {
    if (c < K) {
      if constexpr (sizeof(TX) == 4) {
        r = *(const floatx4*)(row + c);
      } else {
        bf16x4 b = *(const bf16x4*)(row + c);
        r = floatx4{(float)b[0], (float)b[1], (float)b[2], (float)b[3]};
      }
    } else {
      r = floatx4{0, 0, 0, 0};
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; e++) r[e] = (c + e < K) ? (float)row[c + e] : 0.0f;
  }
  return r;
}

template <int VPL, int LPN, typename TV, typename TX, bool VEC>
__global__ __launch_bounds__(256) void spmm_chunks(SpmmKArgs a) {
  constexpr int NPAR = 64 / LPN;
  constexpr int UNR = 4;
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= a.nchunks) return;
  const int grp = lane / LPN, q = lane % LPN;
  const int K = a.K;
  const TX* X = (const TX*)a.X;
  const int64_t j0 = c * a.chunk;
  const int64_t j1 = j0 + a.chunk < a.nnz ? j0 + a.chunk : a.nnz;
  int64_t r = a.chunk_row[c];
  int64_t j = j0;
  while (j < j1) {
    const int64_t rs = a.rowptr[r], re = a.rowptr[r + 1];
    const int64_t se = re < j1 ? re : j1;
    floatx4 acc[VPL];
#pragma unroll
    for (int v = 0; v < VPL; v++) acc[v] = floatx4{0, 0, 0, 0};
    int64_t jj = j + grp;
    for (; jj + (UNR - 1) * NPAR < se; jj += UNR * NPAR) {
      int32_t cc[UNR];
      float vv[UNR];
#pragma unroll
      for (int u = 0; u < UNR; u++) {
        cc[u] = a.col[jj + u * NPAR];
        vv[u] = ld_val<TV>(a.val, jj + u * NPAR);
      }
      floatx4 x[UNR][VPL];
#pragma unroll
      for (int u = 0; u < UNR; u++)
#pragma unroll
        for (int v = 0; v < VPL; v++) x[u][v] = ld_x4<TX, VEC>(X + (int64_t)cc[u] * K, 4 * (q + LPN * v), K);
#pragma unroll
      for (int u = 0; u < UNR; u++)
#pragma unroll
        for (int v = 0; v < VPL; v++) acc[v] += vv[u] * x[u][v];
    }
    for (; jj < se; jj += NPAR) {
      const int32_t cc = a.col[jj];
      const float vv = ld_val<TV>(a.val, jj);
#pragma unroll
      for (int v = 0; v < VPL; v++) acc[v] += vv * ld_x4<TX, VEC>(X + (int64_t)cc * K, 4 * (q + LPN * v), K);
    }
    // combine the NPAR lane groups (fixed butterfly order)
#pragma unroll
    for (int off = LPN; off < 64; off <<= 1)
#pragma unroll
      for (int v = 0; v < VPL; v++)
#pragma unroll
        for (int e = 0; e < 4; e++) acc[v][e] += __shfl_xor(acc[v][e], off);
    float* dst;
    if (rs >= j0 && re <= j1) dst = a.out + r * K;                     // whole row here
    else if (rs < j0) dst = a.carry + (c * 2 + 0) * K;                 // head partial
    else dst = a.carry + (c * 2 + 1) * K;                              // tail partial
    if (grp == 0) {
#pragma unroll
      for (int v = 0; v < VPL; v++) {
        const int cb = 4 * (q + LPN * v);
#pragma unroll
        for (int e = 0; e < 4; e++)
          if (cb + e < K) dst[cb + e] = acc[v][e];
      }
    }
    j = se;
    if (j < j1) {
      r++;
      while (a.rowptr[r + 1] <= j) r++;  // skip empty rows (zeroed by the fixup)
    }
  }
}

// One wave per listed row: zero an empty row, or add the chunk partials of a
// row split across chunks in chunk order.
__global__ __launch_bounds__(256) void spmm_fixup(const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ fix_rows,
                                                  int64_t n_fix, const float* __restrict__ carry,
                                                  float* __restrict__ out, int K, int chunk) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n_fix) return;
  const int lane = threadIdx.x & 63;
  const int64_t r = fix_rows[i];
  const int64_t rs = rowptr[r], re = rowptr[r + 1];
  if (rs == re) {
    for (int k = lane; k < K; k += 64) out[r * K + k] = 0.0f;
    return;
  }
  const int64_t c0 = rs / chunk, c1 = (re - 1) / chunk;
  for (int k = lane; k < K; k += 64) {
    float s = carry[(c0 * 2 + 1) * K + k];
    for (int64_t c = c0 + 1; c <= c1; c++) s += carry[(c * 2 + 0) * K + k];
    out[r * K + k] = s;
  }
}

__global__ void spmm_chunk_rows(const int32_t* __restrict__ rowptr, int64_t rows, int64_t nchunks,
                                int chunk, int32_t* __restrict__ chunk_row) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nchunks) return;
  const int64_t j = c * chunk;
  // first row whose end exceeds j
  int64_t lo = 0, hi = rows - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (rowptr[mid + 1] > j) hi = mid; else lo = mid + 1;
  }
  chunk_row[c] = (int32_t)lo;
}

__global__ void spmm_find_fix(const int32_t* __restrict__ rowptr, int64_t rows, int chunk,
                              int32_t* __restrict__ fix_rows, int32_t* __restrict__ counter) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int64_t rs = rowptr[r], re = rowptr[r + 1];
  const bool need = (rs == re) || (rs / chunk != (re - 1) / chunk);
  if (need) {
    const int slot = atomicAdd(counter, 1);
    fix_rows[slot] = (int32_t)r;
  }
}

template <int VPL, int LPN, typename TV, typename TX>
hipError_t launch_t(const SpmmKArgs& a, bool vec, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.nchunks + 3) / 4);
  if (blocks == 0) return hipSuccess;
  if (vec) spmm_chunks<VPL, LPN, TV, TX, true><<<blocks, 256, 0, s>>>(a);
  else spmm_chunks<VPL, LPN, TV, TX, false><<<blocks, 256, 0, s>>>(a);
  return hipGetLastError();
}

template <typename TV, typename TX>
hipError_t launch_k(const SpmmKArgs& a, bool vec, hipStream_t s) {
  const int n4 = (a.K + 3) / 4;
  if (n4 <= 1) return launch_t<1, 1, TV, TX>(a, vec, s);
  if (n4 <= 2) return launch_t<1, 2, TV, TX>(a, vec, s);
  if (n4 <= 4) return launch_t<1, 4, TV, TX>(a, vec, s);
  if (n4 <= 8) return launch_t<1, 8, TV, TX>(a, vec, s);
  if (n4 <= 16) return launch_t<1, 16, TV, TX>(a, vec, s);
  if (n4 <= 32) return launch_t<1, 32, TV, TX>(a, vec, s);
  if (n4 <= 64) return launch_t<1, 64, TV, TX>(a, vec, s);
  return launch_t<2, 64, TV, TX>(a, vec, s);  // K <= 512
}

}  // namespace

hipError_t spmm_build(SpmmPlan* p, int K, int32_t* chunk_row_buf, int32_t* fix_rows_buf,
                      int32_t* counter, hipStream_t s) {
  p->chunk_row = chunk_row_buf;
  p->fix_rows = fix_rows_buf;
  if (p->nchunks > 0) {
    spmm_chunk_rows<<<(unsigned)((p->nchunks + 255) / 256), 256, 0, s>>>(
        p->rowptr, p->rows, p->nchunks, p->chunk, chunk_row_buf);
  }
  hipError_t e = hipMemsetAsync(counter, 0, sizeof(int32_t), s);
  if (e != hipSuccess) return e;
  if (p->rows > 0)
    spmm_find_fix<<<(unsigned)((p->rows + 255) / 256), 256, 0, s>>>(p->rowptr, p->rows, p->chunk,
                                                                     fix_rows_buf, counter);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  int32_t n = 0;
  e = hipMemcpyAsync(&n, counter, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  p->n_fix = n;
  (void)K;
  return e;
}

hipError_t spmm(const SpmmPlan& p, Elem t, const void* X, int K, float* out, hipStream_t s) {
  SpmmKArgs a;
  a.rowptr = p.rowptr;
  a.col = p.col;
  a.val = p.val;
  a.chunk_row = p.chunk_row;
  a.X = X;
  a.out = out;
  a.carry = p.carry;
  a.nnz = p.nnz;
  a.nchunks = p.nchunks;
  a.chunk = p.chunk;
  a.K = K;
  const size_t esz = t == Elem::F32 ? 4 : 2;
  const bool vec = (K % 4 == 0) && (((uintptr_t)X) % (4 * esz) == 0);
  hipError_t e = t == Elem::F32 ? launch_k<float, float>(a, vec, s)
                                : launch_k<__bf16, __bf16>(a, vec, s);
  if (e != hipSuccess) return e;
  if (p.n_fix > 0) {
    spmm_fixup<<<(unsigned)((p.n_fix + 3) / 4), 256, 0, s>>>(p.rowptr, p.fix_rows, p.n_fix, p.carry,
                                                              out, K, p.chunk);
    e = hipGetLastError();
  }
  return e;
}

// ------------------------------------------------------- CSR transpose ----
namespace {

__global__ void tr_count(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                         int64_t rows, int64_t cols, int nblk, int32_t* __restrict__ cnt) {
  const int b = blockIdx.x;
  const int64_t r0 = rows * b / nblk, r1 = rows * (b + 1) / nblk;
  const int64_t j0 = rowptr[r0], j1 = rowptr[r1];
  for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x)
    atomicAdd(&cnt[(int64_t)b * cols + col[j]], 1);
}

// per column: exclusive running offsets over blocks; column total -> tot[c]
__global__ void tr_colscan(int32_t* __restrict__ cnt, int64_t cols, int nblk,
                           int32_t* __restrict__ tot) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  int32_t run = 0;
  for (int b = 0; b < nblk; b++) {
    const int32_t t = cnt[(int64_t)b * cols + c];
    cnt[(int64_t)b * cols + c] = run;
    run += t;
  }
  tot[c] = run;
}

// single-workgroup exclusive scan of tot[0..n) into out[0..n], out[n] = total
__global__ __launch_bounds__(1024) void tr_scan(const int32_t* __restrict__ tot, int64_t n,
                                                int32_t* __restrict__ out) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t b = per * t, e = b + per < n ? b + per : n;
  int64_t s = 0;
  for (int64_t i = b; i < e; i++) s += tot[i];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int64_t run = 0;
    for (int i = 0; i < 1024; i++) {
      const int64_t v = part[i];
      part[i] = run;
      run += v;
    }
    out[n] = (int32_t)run;
  }
  __syncthreads();
  int64_t run = part[t];
  for (int64_t i = b; i < e; i++) {
    out[i] = (int32_t)run;
    run += tot[i];
  }
}

// one wave per row block, rows in order: keeps each output row sorted by the
// source row index (entries of one source row hit distinct columns)
__global__ __launch_bounds__(64) void tr_scatter(const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col,
                                                 const float* __restrict__ val, int64_t rows,
                                                 int64_t cols, int nblk, int32_t* __restrict__ cnt,
                                                 const int32_t* __restrict__ t_rowptr,
                                                 int32_t* __restrict__ t_col,
                                                 float* __restrict__ t_val) {
  const int b = blockIdx.x;
  const int64_t r0 = rows * b / nblk, r1 = rows * (b + 1) / nblk;
  int32_t* mycnt = cnt + (int64_t)b * cols;
  for (int64_t r = r0; r < r1; r++) {
    const int64_t j0 = rowptr[r], j1 = rowptr[r + 1];
    for (int64_t j = j0 + threadIdx.x; j < j1; j += 64) {
      const int32_t cc = col[j];
      const int32_t pos = t_rowptr[cc] + atomicAdd(&mycnt[cc], 1);
      t_col[pos] = (int32_t)r;
      t_val[pos] = val[j];
    }
    __threadfence_block();
  }
}

__global__ void csr_check(int64_t rows, int64_t cols, int64_t nnz, const int32_t* __restrict__ rowptr,
                          const int32_t* __restrict__ col, const float* __restrict__ val,
                          int32_t* __restrict__ flag) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > rows) return;
  if (r == rows) {
    if (rowptr[rows] != nnz || rowptr[0] != 0) atomicOr(flag, 1);
    return;
  }
  const int64_t a = rowptr[r], b = rowptr[r + 1];
  if (a > b || a < 0 || b > nnz) {
    atomicOr(flag, 1);
    return;
  }
  int32_t prev = -1;
  for (int64_t j = a; j < b; j++) {
    const int32_t c = col[j];
    if (c <= prev || c >= cols) atomicOr(flag, 2);
    prev = c;
    const float v = val[j];
    if (!(v >= 0.0f) || isinf(v)) atomicOr(flag, 4);
  }
}

}  // namespace

int csr_transpose_blocks(int64_t rows, int64_t cols, size_t scratch_ints) {
  int64_t nb = (int64_t)(scratch_ints / (size_t)(cols > 0 ? cols : 1));
  if (nb > 1024) nb = 1024;
  if (nb > rows) nb = rows;
  if (nb < 1) nb = 1;
  return (int)nb;
}

hipError_t csr_transpose(int64_t rows, int64_t cols, int64_t nnz, const int32_t* rowptr,
                         const int32_t* col, const float* val, int32_t* t_rowptr, int32_t* t_col,
                         float* t_val, int32_t* scratch, int nblk, hipStream_t s) {
  // scratch layout: cnt [nblk * cols], tot [cols]
  int32_t* cnt = scratch;
  int32_t* tot = scratch + (int64_t)nblk * cols;
  hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)nblk * (size_t)cols, s);
  if (e != hipSuccess) return e;
  if (rows > 0) tr_count<<<nblk, 256, 0, s>>>(rowptr, col, rows, cols, nblk, cnt);
  if (cols > 0) tr_colscan<<<(unsigned)((cols + 255) / 256), 256, 0, s>>>(cnt, cols, nblk, tot);
  tr_scan<<<1, 1024, 0, s>>>(tot, cols, t_rowptr);
  if (rows > 0)
    tr_scatter<<<nblk, 64, 0, s>>>(rowptr, col, val, rows, cols, nblk, cnt, t_rowptr, t_col, t_val);
  (void)nnz;
  return hipGetLastError();
}

hipError_t csr_validate(int64_t rows, int64_t cols, int64_t nnz, const int32_t* rowptr,
                        const int32_t* col, const float* val, int32_t* flag, hipStream_t s) {
  csr_check<<<(unsigned)((rows + 1 + 255) / 256), 256, 0, s>>>(rows, cols, nnz, rowptr, col, val,
                                                                flag);
  return hipGetLastError();
}

}  // namespace plnmf
