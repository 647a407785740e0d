// Kernels of the fold-in warm-start network around its matrix-core products
// (the products themselves run through the shared GEMM with fused bias/GELU,
// bias/softplus and GELU-gradient epilogues): seeded init, the output-layer
// gradient of the mean-squared error, bias-gradient column sums, Adam, and the
// row normalisation / rescaling that wraps the network in fold-in.
#include <algorithm>

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

// out[c] = sum_r x[r, c] in two fixed-order passes: slice s of the rows sums
// its rows in order per column (FP64) into part[s][c], then the slices are
// added in slice order.  Thread per column and workgroup per (column block,
// row slice), so a batch of 1024 rows and 512 columns spreads over the chip.
__global__ void colsum_part_kernel(const float* __restrict__ x, int64_t rows, int64_t cols,
                                   int slices, double* __restrict__ part) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int sl = blockIdx.y;
  if (c >= cols) return;
  const int64_t r0 = rows * sl / slices, r1 = rows * (sl + 1) / slices;
  double s = 0.0;
  for (int64_t r = r0; r < r1; r++) s += x[r * cols + c];
  part[(int64_t)sl * cols + c] = s;
}

__global__ void colsum_fin_kernel(const double* __restrict__ part, int64_t cols, int slices,
                                  float* __restrict__ out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int sl = 0; sl < slices; sl++) s += part[(int64_t)sl * cols + c];
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


// Fused inference of the network for fold-in: for each row r of R = A_new^T W
//   x = r / ||r|| (BF16),  g = GELU(W1 x + b1) (BF16),
//   h0 = max(eps, ||r|| softplus(W2 g + b2)),
// the arithmetic of the two-GEMM path (BF16 operands, FP32 accumulation) in
// one pass over R and one write of h0, with nothing of the hidden layer
// leaving the CU.  A workgroup is eight waves of 32 rows.  A wave holds its
// rows' x in registers in the A-operand layout of the 32x32x16 BF16 matrix-core
// product (lane (m, h) holds row m's elements 16 s + 8 h .. + 7 in xf[s]) and
// walks the hidden units in chunks of 32: the chunk's 32-wide block of W1 x
// on the matrix cores, bias + GELU in its output layout, a transpose of the
// 32 x 32 activations through the wave's own LDS rows, then their product
// with the chunk's columns of W2 into the output accumulators.  The chunk's
// weights are staged in LDS for all eight waves, the next chunk's already in
// flight in registers.  Needs K % 8 == 0, K <= 208 and hidden % 32 == 0.
constexpr int kInfWaves = 8, kInfRows = 32 * kInfWaves, kHC = 32;

struct MlpInferArgs {
  const float* R;
  int64_t N;
  int K, H;
  const __bf16* W1b;  // [H, K]
  const float* b1;    // [H]
  const __bf16* W2b;  // [K, H]
  const float* b2;    // [K]
  float eps;
  float* out;         // [N, K]
};

__host__ __device__ constexpr int inf_kp1(int NKB) { return 16 * NKB + 8; }  // W1 row pitch
constexpr int kInfHP = kHC + 8;                                              // W2 / G row pitch
__host__ __device__ constexpr size_t inf_smem_bytes(int NKB) {
  return 2 * ((size_t)kHC * inf_kp1(NKB) + (size_t)32 * ((NKB + 1) / 2) * kInfHP +
              (size_t)kInfWaves * 32 * kInfHP) +
         4 * (size_t)kInfWaves * 32;
}

__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NKB>
__global__ __launch_bounds__(512) void mlp_infer_kernel(MlpInferArgs a) {
  constexpr int NB2 = (NKB + 1) / 2;  // 32-column output blocks: 32 NB2 >= 16 NKB >= K
  constexpr int KP1 = inf_kp1(NKB), HP = kInfHP;
  constexpr int P1 = kHC * 2 * NKB, P2 = 32 * NB2 * (kHC / 8);  // 16-byte pieces per chunk
  constexpr int L1 = (P1 + 511) / 512, L2 = (P2 + 511) / 512;
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16* w1s = (__bf16*)smem;                       // [kHC][KP1]
  __bf16* w2s = w1s + kHC * KP1;                     // [32 NB2][HP]
  __bf16* gs = w2s + 32 * NB2 * HP;                  // [waves][32][HP]
  float* nrs = (float*)(gs + kInfWaves * 32 * HP);   // [waves][32]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m = lane & 31, h = lane >> 5;
  const int K = a.K, H = a.H;
  const int64_t r0 = (int64_t)blockIdx.x * kInfRows + 32 * w;
  const int64_t row = r0 + m;
  const bf16x8 zero8 = {};

  // this lane's pieces of its row, the row's norm, and x in BF16 (the row is
  // read twice, the second time from the L2, so that the FP32 values and x
  // are never held together)
  bf16x8 xf[NKB];
  {
    auto piece = [&](int s, int q) -> floatx4 {
      const int k = 16 * s + 8 * h + 4 * q;
      return (row < a.N && k < K) ? *(const floatx4*)(a.R + row * K + k) : floatx4{0, 0, 0, 0};
    };
    float ss = 0.0f;
#pragma unroll
    for (int s = 0; s < NKB; s++)
#pragma unroll
      for (int q = 0; q < 2; q++) {
        const floatx4 v = piece(s, q);
#pragma unroll
        for (int e = 0; e < 4; e++) ss += v[e] * v[e];
      }
    ss += __shfl_xor(ss, 32);
    const float nrm = sqrtf(ss);
    const float inv = nrm > 0.0f ? 1.0f / nrm : 0.0f;
#pragma unroll
    for (int s = 0; s < NKB; s++)
#pragma unroll
      for (int q = 0; q < 2; q++) {
        const floatx4 v = piece(s, q);
#pragma unroll
        for (int e = 0; e < 4; e++) xf[s][4 * q + e] = (__bf16)(v[e] * inv);
      }
    if (h == 0) nrs[32 * w + m] = nrm;
  }

  bf16x8 pre1[L1], pre2[L2];
  auto fetch = [&](int c) {
#pragma unroll
    for (int u = 0; u < L1; u++) {
      const int i = tid + 512 * u;
      const int jl = i / (2 * NKB), k = 8 * (i % (2 * NKB));
      pre1[u] = (i < P1 && k < K) ? *(const bf16x8*)(a.W1b + (int64_t)(c * kHC + jl) * K + k)
                                  : zero8;
    }
#pragma unroll
    for (int u = 0; u < L2; u++) {
      const int i = tid + 512 * u;
      const int kr = i / (kHC / 8), hq = i % (kHC / 8);
      pre2[u] = (i < P2 && kr < K) ? *(const bf16x8*)(a.W2b + (int64_t)kr * H + c * kHC + 8 * hq)
                                   : zero8;
    }
  };
  auto put = [&]() {
#pragma unroll
    for (int u = 0; u < L1; u++) {
      const int i = tid + 512 * u;
      if (i < P1) *(bf16x8*)(w1s + (i / (2 * NKB)) * KP1 + 8 * (i % (2 * NKB))) = pre1[u];
    }
#pragma unroll
    for (int u = 0; u < L2; u++) {
      const int i = tid + 512 * u;
      if (i < P2) *(bf16x8*)(w2s + (i / (kHC / 8)) * HP + 8 * (i % (kHC / 8))) = pre2[u];
    }
  };

  floatx16 acc2[NB2];
#pragma unroll
  for (int o = 0; o < NB2; o++)
#pragma unroll
    for (int e = 0; e < 16; e++) acc2[o][e] = 0.0f;
  __bf16* gw = gs + 32 * w * HP;  // this wave's activation rows
  const int nch = H / kHC;
  fetch(0);
#pragma unroll 1
  for (int c = 0; c < nch; c++) {
    put();
    __syncthreads();
    if (c + 1 < nch) fetch(c + 1);
    // W1 x for the chunk's 32 hidden units: even and odd steps in two
    // accumulator chains (one chain would wait out every product's latency)
    floatx16 acc1, acc1b;
#pragma unroll
    for (int e = 0; e < 16; e++) acc1[e] = acc1b[e] = 0.0f;
#pragma unroll
    for (int s = 0; s < NKB; s++) {
      const bf16x8 wb = *(const bf16x8*)(w1s + m * KP1 + 16 * s + 8 * h);
      if (s & 1)
        acc1b = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xf[s], wb, acc1b, 0, 0, 0);
      else
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xf[s], wb, acc1, 0, 0, 0);
    }
    acc1 += acc1b;
    // bias + GELU; lane holds rows 8 jj + 4 h + i of hidden unit m
    {
      const float bb = a.b1[c * kHC + m];
#pragma unroll
      for (int jj = 0; jj < 4; jj++)
#pragma unroll
        for (int i = 0; i < 4; i++)
          gw[(8 * jj + 4 * h + i) * HP + m] = (__bf16)gelu_f(acc1[4 * jj + i] + bb);
    }
    wave_lds_order();
    // activations (A operand: row m, hidden 16 t + 8 h ..) times the chunk's W2 columns
#pragma unroll
    for (int t = 0; t < kHC / 16; t++) {
      const bf16x8 gf = *(const bf16x8*)(gw + m * HP + 16 * t + 8 * h);
#pragma unroll
      for (int o = 0; o < NB2; o++) {
        const bf16x8 wf = *(const bf16x8*)(w2s + (32 * o + m) * HP + 16 * t + 8 * h);
        acc2[o] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(gf, wf, acc2[o], 0, 0, 0);
      }
    }
    __syncthreads();  // the chunk's weights are no longer read
  }
  // bias + softplus, rescaled by the row's norm and clipped at eps
#pragma unroll
  for (int o = 0; o < NB2; o++) {
    const int kc = 32 * o + m;
    if (kc >= K) continue;
    const float bb = a.b2[kc];
#pragma unroll
    for (int jj = 0; jj < 4; jj++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int rr = 8 * jj + 4 * h + i;
        if (r0 + rr >= a.N) continue;
        const float y = softplus_f(acc2[o][4 * jj + i] + bb);
        a.out[(r0 + rr) * K + kc] = fmaxf(a.eps, nrs[32 * w + rr] * y);
      }
  }
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

hipError_t col_sum(const float* x, int64_t rows, int64_t cols, float* out, double* part,
                   hipStream_t s) {
  if (cols <= 0) return hipSuccess;
  const int slices = (int)std::max<int64_t>(1, std::min<int64_t>(kColSlices, rows));
  const unsigned cb = (unsigned)((cols + 255) / 256);
  colsum_part_kernel<<<dim3(cb, (unsigned)slices), 256, 0, s>>>(x, rows, cols, slices, part);
  colsum_fin_kernel<<<cb, 256, 0, s>>>(part, cols, slices, out);
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


// K <= 208: at most 13 steps of x in registers (at 14 the kernel would spill)
bool mlp_infer_fused_ok(int K, int H) {
  return K >= 1 && K <= 208 && K % 8 == 0 && H >= kHC && H % kHC == 0;
}

hipError_t mlp_infer_fused(const float* R, int64_t N, int K, int H, const __bf16* W1b,
                           const float* b1, const __bf16* W2b, const float* b2, float eps,
                           float* out, hipStream_t s) {
  if (!mlp_infer_fused_ok(K, H)) return hipErrorInvalidValue;
  if (N <= 0) return hipSuccess;
  MlpInferArgs a{R, N, K, H, W1b, b1, W2b, b2, eps, out};
  const unsigned blocks = (unsigned)((N + kInfRows - 1) / kInfRows);
  const int nkb = (K + 15) / 16;  // 16-wide steps over the rank
#define PLNMF_INF(NKB)                                                                        \
  case NKB: {                                                                                 \
    const size_t bytes = inf_smem_bytes(NKB);                                                 \
    hipError_t e = hipFuncSetAttribute((const void*)mlp_infer_kernel<NKB>,                    \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes); \
    if (e != hipSuccess) return e;                                                            \
    mlp_infer_kernel<NKB><<<blocks, 512, bytes, s>>>(a);                                      \
    break;                                                                                    \
  }
  switch (nkb) {
    PLNMF_INF(1) PLNMF_INF(2) PLNMF_INF(3) PLNMF_INF(4) PLNMF_INF(5) PLNMF_INF(6)
    PLNMF_INF(7) PLNMF_INF(8) PLNMF_INF(9) PLNMF_INF(10) PLNMF_INF(11) PLNMF_INF(12)
    PLNMF_INF(13)
    default: return hipErrorInvalidValue;
  }
#undef PLNMF_INF
  return hipGetLastError();
}

hipError_t clip_min(const float* x, int64_t n, float eps, float* out, hipStream_t s) {
  clip_kernel<<<grid_for(n), 256, 0, s>>>(x, n, eps, out);
  return hipGetLastError();
}

}  // namespace plnmf
