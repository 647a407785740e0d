// Elementwise and reduction kernels around the sweep: the column normalisation
// of W before the first sweep, BF16 operand casts, input checks, and the
// fixed-order FP64 reductions of the objective (Eq. 2 and the relative
// objective of Sec. 6.2).
#include "internal.hpp"

namespace plnmf {
namespace {

__device__ __forceinline__ double block_sum_d(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); i++) t += sh[i];
  __syncthreads();
  return t;
}

// partial[b][k] = sum over rows r = b, b + nblk, ... of X[r,k]^2 (FP64)
__global__ void colsq_kernel(const float* __restrict__ X, int64_t rows, int K,
                              double* __restrict__ part) {
  const int b = blockIdx.x, nblk = gridDim.x;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    double s = 0.0;
    for (int64_t r = b; r < rows; r += nblk) {
      const double x = X[r * K + k];
      s += x * x;
    }
    part[(int64_t)b * K + k] = s;
  }
}

// A column whose norm is zero (or overflows FP32) cannot be normalised: it is
// left unchanged and bit `bit` of *flag is set (every block sees the same
// norms; block 0 reports).
__global__ void colscale(float* __restrict__ X, int64_t rows, int K, const double* __restrict__ part,
                         int nblk, int32_t* flag, int bit) {
  __shared__ float norm[kMaxK];
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblk; b++) s += part[(int64_t)b * K + k];
    const float nk = (float)sqrt(s);
    const bool ok = nk > 0.0f && !isinf(nk);
    norm[k] = ok ? nk : 1.0f;
    if (!ok && blockIdx.x == 0) atomicOr(flag, bit);
  }
  __syncthreads();
  const int64_t n = rows * K;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(i % K);
    X[i] = X[i] / norm[k];
  }
}

__global__ void cast_kernel(const float* __restrict__ x, __bf16* __restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (__bf16)x[i];
}

__global__ void cast_t_kernel(const float* __restrict__ x, __bf16* __restrict__ y, int64_t rows,
                              int64_t cols) {
  __shared__ float tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows per pass
  for (int i = ty; i < 32; i += 8) {
    const int64_t r = r0 + i, c = c0 + tx;
    tile[i][tx] = (r < rows && c < cols) ? x[r * cols + c] : 0.0f;
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < cols && r < rows) y[c * rows + r] = (__bf16)tile[tx][i];
  }
}

__global__ void finite_nonneg(const float* __restrict__ x, int64_t n, int32_t* flag, int bit) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v = x[i];
    if (!(v >= 0.0f) || isinf(v)) bad = true;
  }
  if (bad) atomicOr(flag, bit);
}

__global__ void sumsq_kernel(const float* __restrict__ x, int64_t n, double* __restrict__ part) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = x[i];
    s += v * v;
  }
  const double t = block_sum_d(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// sum of x*y over FP32 inputs, products and sums in FP64
__global__ void dot_kernel(const float* __restrict__ x, const float* __restrict__ y, int64_t n,
                           double* __restrict__ part) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s += (double)x[i] * (double)y[i];
  const double t = block_sum_d(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void finish_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sh[16];
  double s = 0.0;
  // fixed assignment of partials to threads, then a fixed tree
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  const double t = block_sum_d(s, sh);
  if (threadIdx.x == 0) out[0] = t;
}

// out_half = e2 / 2, out_rel = sqrt(e2 / a2) with e2 = a2 - 2 wp + sq (identity)
// or e2 = sq when wp is null (explicit residual)
__global__ void combine_kernel(const double* a2, const double* wp, const double* sq,
                               double* out_half, double* out_rel) {
  double e2 = wp ? a2[0] - 2.0 * wp[0] + sq[0] : sq[0];
  if (e2 < 0.0) e2 = 0.0;
  out_half[0] = 0.5 * e2;
  out_rel[0] = sqrt(e2 / a2[0]);
}

}  // namespace

int reduce_blocks(int64_t n) {
  int64_t b = (n + 4095) / 4096;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t normalize_columns(float* X, int64_t rows, int K, double* part, int nblk_max,
                             int32_t* flag, int bit, hipStream_t s) {
  int nblk = (int)((rows + 63) / 64);
  if (nblk > nblk_max) nblk = nblk_max;
  if (nblk < 1) nblk = 1;
  colsq_kernel<<<nblk, 256, 0, s>>>(X, rows, K, part);
  int gb = (int)((rows * K + 255) / 256);
  if (gb > 2048) gb = 2048;
  if (gb < 1) gb = 1;
  colscale<<<gb, 256, 0, s>>>(X, rows, K, part, nblk, flag, bit);
  return hipGetLastError();
}

static int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t cast_bf16(const float* x, __bf16* y, int64_t n, hipStream_t s) {
  cast_kernel<<<grid_for(n), 256, 0, s>>>(x, y, n);
  return hipGetLastError();
}

hipError_t cast_bf16_transpose(const float* x, __bf16* y, int64_t rows, int64_t cols,
                               hipStream_t s) {
  dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  cast_t_kernel<<<grid, 256, 0, s>>>(x, y, rows, cols);
  return hipGetLastError();
}

__global__ void or_bits_kernel(int32_t* word, int32_t bits) { atomicOr(word, bits); }

hipError_t or_bits(int32_t* word, int32_t bits, hipStream_t s) {
  or_bits_kernel<<<1, 1, 0, s>>>(word, bits);
  return hipGetLastError();
}

hipError_t check_finite_nonneg(const float* x, int64_t n, int32_t* flag, int bit, hipStream_t s) {
  finite_nonneg<<<grid_for(n), 256, 0, s>>>(x, n, flag, bit);
  return hipGetLastError();
}

hipError_t sumsq_f64(const float* x, int64_t n, double* partial, int nblk, hipStream_t s) {
  sumsq_kernel<<<nblk, 256, 0, s>>>(x, n, partial);
  return hipGetLastError();
}

hipError_t dot_f64(const float* x, const float* y, int64_t n, double* partial, int nblk,
                   hipStream_t s) {
  dot_kernel<<<nblk, 256, 0, s>>>(x, y, n, partial);
  return hipGetLastError();
}

hipError_t finish_f64(const double* partial, int n, double* out, hipStream_t s) {
  finish_kernel<<<1, 256, 0, s>>>(partial, n, out);
  return hipGetLastError();
}

hipError_t combine_objective(const double* a2, const double* wp, const double* sq,
                             double* out_half, double* out_rel, hipStream_t s) {
  combine_kernel<<<1, 1, 0, s>>>(a2, wp, sq, out_half, out_rel);
  return hipGetLastError();
}


namespace {
__global__ void dense_rows_kernel(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                  const float* __restrict__ val, const int32_t* __restrict__ rows,
                                  int64_t cols, float* __restrict__ out) {
  const int i = blockIdx.x;
  const int64_t r = rows[i];
  float* o = out + (int64_t)i * cols;
  for (int64_t j = rowptr[r] + threadIdx.x; j < rowptr[r + 1]; j += blockDim.x) o[col[j]] = val[j];
}

__global__ void scatter_rows_kernel(const float* __restrict__ src, const int32_t* __restrict__ rows,
                                    int K, float* __restrict__ dst) {
  const int i = blockIdx.x;
  const int64_t r = rows[i];
  for (int c = threadIdx.x; c < K; c += blockDim.x) dst[r * K + c] = src[(int64_t)i * K + c];
}
}  // namespace

hipError_t csr_dense_rows(const int32_t* rowptr, const int32_t* col, const float* val,
                          const int32_t* rows, int n, int64_t cols, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipError_t e = hipMemsetAsync(out, 0, (size_t)n * cols * sizeof(float), s);
  if (e != hipSuccess) return e;
  dense_rows_kernel<<<(unsigned)n, 256, 0, s>>>(rowptr, col, val, rows, cols, out);
  return hipGetLastError();
}

hipError_t scatter_rows(const float* src, const int32_t* rows, int n, int K, float* dst,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  scatter_rows_kernel<<<(unsigned)n, 128, 0, s>>>(src, rows, K, dst);
  return hipGetLastError();
}

}  // namespace plnmf
