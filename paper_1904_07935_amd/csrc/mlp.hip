// Kernels of the fold-in warm-start network around its matrix-core products
// (the products themselves run through the shared GEMM with fused bias/GELU,
// bias/softplus and GELU-gradient epilogues): seeded init, the output-layer
// gradient of the mean-squared error, bias-gradient column sums, Adam, and the
// row normalisation / rescaling that wraps the network in fold-in.
#include "internal.hpp"

namespace plnmf {
namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// masters: W1 [H,K], b1 [H], W2 [K,H], b2 [K]; fan-in of layer 1 is K, of layer 2 is H
__global__ void init_kernel(float* __restrict__ p, int64_t n, int K, int H, uint64_t seed) {
  const int64_t n1 = (int64_t)H * K + H;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t z = splitmix64(seed ^ splitmix64((uint64_t)i));
    const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);  // [0,1)
    const double bound = i < n1 ? 1.0 / sqrt((double)K) : 1.0 / sqrt((double)H);
    p[i] = (float)((2.0 * u - 1.0) * bound);
  }
}

// Adam with bias corrections for step t = *step + 1 (the count is bumped by a
// separate one-thread launch afterwards)
__global__ void adam_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int64_t n, float lr,
                            const int64_t* __restrict__ step) {
  const double t = (double)(*step + 1);
  const float b1t = (float)(1.0 - pow(0.9, t));
  const float b2t = (float)(1.0 - pow(0.999, t));
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / b1t) / (sqrtf(vi / b2t) + 1e-8f);
  }
}

__global__ void bump_kernel(int64_t* step) { *step += 1; }

__global__ void acc_kernel(double* acc, const double* v, double scale) { acc[0] += v[0] * scale; }

// d = yhat - y; loss partial sum d^2 (FP64); dz2 = scale * d * softplus'(z2)
__global__ void out_grad_kernel(const float* __restrict__ z2, const float* __restrict__ yhat,
                                const float* __restrict__ y, int64_t n, float scale,
                                __bf16* __restrict__ dz2b, float* __restrict__ dz2f,
                                double* __restrict__ part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float d = yhat[i] - y[i];
    s += (double)d * (double)d;
    const float z = z2[i];
    const float sg = z > 20.0f ? 1.0f : 1.0f / (1.0f + expf(-z));
    const float gz = scale * d * sg;
    dz2b[i] = (__bf16)gz;
    dz2f[i] = gz;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// out[c] = sum_r x[r, c], rows in order per column (FP64 accumulation)
__global__ void colsum_kernel(const float* __restrict__ x, int64_t rows, int64_t cols,
                              float* __restrict__ out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int64_t r = 0; r < rows; r++) s += x[r * cols + c];
  out[c] = (float)s;
}

__global__ void gather_kernel(const float* __restrict__ x, const int32_t* __restrict__ idx,
                              int64_t n, int64_t cols, float* __restrict__ out) {
  const int64_t total = n * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols, c = i - r * cols;
    out[i] = x[(int64_t)idx[r] * cols + c];
  }
}

// one wave per row
__global__ void rownorm_kernel(const float* __restrict__ x, int64_t rows, int64_t cols,
                               float* __restrict__ xn, float* __restrict__ norms) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  const int lane = threadIdx.x & 63;
  float s = 0.0f;
  for (int64_t c = lane; c < cols; c += 64) {
    const float v = x[r * cols + c];
    s += v * v;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  const float nrm = sqrtf(s);
  if (lane == 0) norms[r] = nrm;
  for (int64_t c = lane; c < cols; c += 64) xn[r * cols + c] = nrm > 0.0f ? x[r * cols + c] / nrm : 0.0f;
}

__global__ void rescale_kernel(const float* __restrict__ y, const float* __restrict__ norms,
                               int64_t rows, int64_t cols, float eps, float* __restrict__ out) {
  const int64_t total = rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v = norms[i / cols] * y[i];
    out[i] = fmaxf(eps, v);
  }
}

__global__ void clip_kernel(const float* __restrict__ x, int64_t n, float eps, float* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = fmaxf(eps, x[i]);
}

int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

hipError_t mlp_init_params(float* master, int64_t n, int K, int hidden, uint64_t seed,
                           hipStream_t s) {
  init_kernel<<<grid_for(n), 256, 0, s>>>(master, n, K, hidden, seed);
  return hipGetLastError();
}

hipError_t mlp_adam(float* master, float* m, float* v, const float* g, int64_t n, float lr,
                    int64_t* step, hipStream_t s) {
  adam_kernel<<<grid_for(n), 256, 0, s>>>(master, m, v, g, n, lr, step);
  bump_kernel<<<1, 1, 0, s>>>(step);
  return hipGetLastError();
}

hipError_t acc_scaled(double* acc, const double* v, double scale, hipStream_t s) {
  acc_kernel<<<1, 1, 0, s>>>(acc, v, scale);
  return hipGetLastError();
}

hipError_t mlp_out_grad(const float* z2, const float* yhat, const float* y, int64_t n,
                        float scale, __bf16* dz2_bf16, float* dz2_f32, double* loss_partial,
                        int nblk, hipStream_t s) {
  out_grad_kernel<<<nblk, 256, 0, s>>>(z2, yhat, y, n, scale, dz2_bf16, dz2_f32, loss_partial);
  return hipGetLastError();
}

hipError_t col_sum(const float* x, int64_t rows, int64_t cols, float* out, hipStream_t s) {
  colsum_kernel<<<(unsigned)((cols + 255) / 256), 256, 0, s>>>(x, rows, cols, out);
  return hipGetLastError();
}

hipError_t gather_rows(const float* x, const int32_t* idx, int64_t n, int64_t cols, float* out,
                       hipStream_t s) {
  gather_kernel<<<grid_for(n * cols), 256, 0, s>>>(x, idx, n, cols, out);
  return hipGetLastError();
}

hipError_t row_normalize(const float* x, int64_t rows, int64_t cols, float* xn, float* norms,
                         hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  rownorm_kernel<<<(unsigned)((rows + 3) / 4), 256, 0, s>>>(x, rows, cols, xn, norms);
  return hipGetLastError();
}

hipError_t rescale_clip_rows(const float* y, const float* norms, int64_t rows, int64_t cols,
                             float eps, float* out, hipStream_t s) {
  rescale_kernel<<<grid_for(rows * cols), 256, 0, s>>>(y, norms, rows, cols, eps, out);
  return hipGetLastError();
}

hipError_t clip_min(const float* x, int64_t n, float eps, float* out, hipStream_t s) {
  clip_kernel<<<grid_for(n), 256, 0, s>>>(x, n, eps, out);
  return hipGetLastError();
}

}  // namespace plnmf
