// Gram matrices of the sweep, S = W^T W and Q = H H^T = Ht^T Ht (Alg. 1, the
// S and Q statements): C = X^T X for X [rows, K] row-major, K <= 512.
//
// The contraction (rows) is long and the output small, so the work is split
// by rows: one 512-thread workgroup per chunk of rows stages its chunk through
// LDS (X is read from HBM exactly once) and accumulates the chunk's partial
// Gram on the matrix cores, 32 x 32 output blocks of the upper triangle only
// (C is symmetric), a fixed set of blocks per wave.  A second kernel adds the
// chunks' partials in chunk order and writes both triangles: the result is
// bitwise reproducible and independent of scheduling.
#include "internal.hpp"

namespace plnmf {
namespace {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kRS = 32;             // rows per LDS stage
constexpr int kMaxBlocksPerWave = 4;
constexpr int kBlocksPerPass = kWaves * kMaxBlocksPerWave;

__host__ __device__ inline int nblk(int K) { return (K + 31) / 32; }
__host__ __device__ inline int upper_blocks(int K) { return nblk(K) * (nblk(K) + 1) / 2; }

// block index u -> (bi, bj), bi <= bj, in row-major order of the upper triangle
__device__ __forceinline__ void block_of(int u, int nb, int& bi, int& bj) {
  int i = 0, rowlen = nb;
  while (u >= rowlen) {
    u -= rowlen;
    i++;
    rowlen--;
  }
  bi = i;
  bj = i + u;
}

// partial[chunk][u][32][32] for the blocks u of pass blockIdx.y
template <bool VEC>
__global__ __launch_bounds__(kThreads) void gram_partial(const float* __restrict__ X, int64_t rows,
                                                         int K, int64_t rows_per_chunk,
                                                         float* __restrict__ partial) {
  extern __shared__ float stage[];  // [kRS][P], P = 32 * nblk(K)
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nb = nblk(K), P = 32 * nb, nu = upper_blocks(K);
  const int64_t chunk = blockIdx.x;
  const int64_t r0 = chunk * rows_per_chunk;
  int64_t r1 = r0 + rows_per_chunk;
  if (r1 > rows) r1 = rows;
  const int ubase = blockIdx.y * kBlocksPerPass;
  int bi[kMaxBlocksPerWave], bj[kMaxBlocksPerWave];
  bool has[kMaxBlocksPerWave];
#pragma unroll
  for (int k = 0; k < kMaxBlocksPerWave; k++) {
    const int u = ubase + k * kWaves + w;
    has[k] = u < nu && u < ubase + kBlocksPerPass;
    if (has[k]) block_of(u, nb, bi[k], bj[k]);
    else bi[k] = bj[k] = 0;  // computed like block (0, 0), never stored: no branch in the loop
  }
  floatx16 acc[kMaxBlocksPerWave];
#pragma unroll
  for (int k = 0; k < kMaxBlocksPerWave; k++)
#pragma unroll
    for (int e = 0; e < 16; e++) acc[k][e] = 0.0f;

  const int nq = P / 4;  // float4 per staged row
  // thread's share of a stage: float4 i = tid + kThreads * u of kRS * nq
  constexpr int kPer = (kRS * 32 * kMaxK / 32 / 4 + kThreads - 1) / kThreads;  // <= 8
  auto fetch = [&](int64_t s0, floatx4 (&buf)[kPer]) {
#pragma unroll
    for (int u = 0; u < kPer; u++) {
      const int i = tid + kThreads * u;
      const int rl = i / nq, c = 4 * (i % nq);
      const int64_t r = s0 + rl;
      floatx4 v = floatx4{0, 0, 0, 0};
      if (i < kRS * nq && r < r1) {
        const float* src = X + r * K + c;
        if constexpr (VEC) {
          if (c < K) v = *(const floatx4*)src;
        } else {
#pragma unroll
          for (int e = 0; e < 4; e++)
            if (c + e < K) v[e] = src[e];
        }
      }
      buf[u] = v;
    }
  };
  auto put = [&](const floatx4 (&buf)[kPer]) {
#pragma unroll
    for (int u = 0; u < kPer; u++) {
      const int i = tid + kThreads * u;
      if (i < kRS * nq) *(floatx4*)(stage + (i / nq) * P + 4 * (i % nq)) = buf[u];
    }
  };
  floatx4 nxt[kPer];
  fetch(r0, nxt);
  const int h = lane >> 5, m = lane & 31;
  for (int64_t s0 = r0; s0 < r1; s0 += kRS) {
    __syncthreads();  // the previous stage is no longer read
    put(nxt);
    __syncthreads();
    if (s0 + kRS < r1) fetch(s0 + kRS, nxt);  // in flight during this stage's products
    auto ksteps = [&](int kk) {
      const float* row = stage + (kk + h) * P;
      float av[kMaxBlocksPerWave], bv[kMaxBlocksPerWave];
#pragma unroll
      for (int k = 0; k < kMaxBlocksPerWave; k++) {
        av[k] = row[32 * bi[k] + m];
        bv[k] = row[32 * bj[k] + m];
      }
#pragma unroll
      for (int k = 0; k < kMaxBlocksPerWave; k++)
        acc[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[k], bv[k], acc[k], 0, 0, 0);
    };
    if (s0 + kRS <= r1) {
#pragma unroll
      for (int kk = 0; kk < kRS; kk += 2) ksteps(kk);
    } else {  // the chunk's ragged last stage: only its rows (the rest is zero)
      const int nk = (int)(r1 - s0);
      for (int kk = 0; kk < nk; kk += 2) ksteps(kk);
    }
  }
  // lane holds C block row 8 j + 4 h + i, column lane % 32, in acc[4 j + i]
  const int n = lane & 31;
#pragma unroll
  for (int k = 0; k < kMaxBlocksPerWave; k++) {
    if (!has[k]) continue;
    const int u = ubase + k * kWaves + w;
    float* dst = partial + ((int64_t)chunk * nu + u) * 1024;
#pragma unroll
    for (int j = 0; j < 4; j++)
#pragma unroll
      for (int i = 0; i < 4; i++) dst[(8 * j + 4 * h + i) * 32 + n] = acc[k][4 * j + i];
  }
}

// C[K][K] from the partials: workgroup (u, part) handles 32 float4 of block u;
// thread (f, sl) sums chunks sl, sl + 16, ... of float4 f, then slice 0 adds
// the 16 slice sums in slice order.
constexpr int kRedSlices = 16;
constexpr int kRedThreads = 32 * kRedSlices;

// Panel entry of C[l][col] for the tile products of the column updates (the B
// operand of the tile of col, contraction row l): 1 - C or 0 on the diagonal,
// 0 for l inside the tile and left of col, -C elsewhere.  Same layout as the
// update kernels read: panel[j][l][c] (l < kpad(K), c < 32), then gblk[j][t][c].
// The same entries in the H rows kernel's staging order, one block of
// NB * NT * 1024 + tile^2 floats per tile (NT = ceil(K / 32), NB = max(1,
// tile / 32)): entry (l, c) of the tile's panel at
// ((((c / 32) NT + l / 32) 4 + s / 4) 2 + l % 2) 32 + c % 32) 4 + s % 4 with
// s = (l % 32) / 2 -- lane (m, h) then reads rows 32 t + 2 (4 sq + i) + h of
// column m as one float4 -- then the G block split by column parity,
// [h][t][k] = G[t][2 k + h] where 2 k + h > t (zero elsewhere).
__device__ __forceinline__ void put_panel_rows(float* panel, int K, int diag_one, int tile, int l, int col,
                                               float v) {
  const int nt = (K + 31) / 32, nb = tile >= 32 ? tile / 32 : 1;
  const int64_t per_tile = (int64_t)nb * nt * 1024 + tile * tile;
  const int j = col / tile, c = col % tile, a0 = tile * j;
  float pv;
  if (l == col) pv = diag_one ? 1.0f - v : 0.0f;
  else if (l >= a0 && l < col) pv = 0.0f;
  else pv = -v;
  const int r = l & 31, s2 = r >> 1;
  float* pt = panel + j * per_tile;
  pt[(((((c >> 5) * nt + (l >> 5)) * 4 + (s2 >> 2)) * 2 + (r & 1)) * 32 + (c & 31)) * 4 + (s2 & 3)] = pv;
  const int t = l - a0;
  if (l / tile == j && c > t)
    pt[(int64_t)nb * nt * 1024 + (c & 1) * (tile * tile / 2) + t * (tile / 2) + (c >> 1)] = v;
}

__device__ __forceinline__ void put_panel(float* panel, int K, int diag_one, int tile, int l, int col,
                                          float v) {
  const int kp = (K + 7) / 8 * 8, ntiles = (K + tile - 1) / tile;
  const int j = col / tile, c = col % tile, a0 = tile * j;
  float pv;
  if (l == col) pv = diag_one ? 1.0f - v : 0.0f;
  else if (l >= a0 && l < col) pv = 0.0f;
  else pv = -v;
  panel[((int64_t)j * kp + l) * tile + c] = pv;
  if (l / tile == j)
    panel[(int64_t)ntiles * kp * tile + ((int64_t)j * tile + (l - a0)) * tile + c] = v;
}

__global__ __launch_bounds__(kRedThreads) void gram_reduce(const float* __restrict__ partial, int nchunks,
                                                    int K, float* __restrict__ C, int64_t ldc,
                                                    float* __restrict__ panel, int diag_one, int tile,
                                                    int rows_layout) {
  __shared__ floatx4 part[kRedThreads];
  const int nb = nblk(K), nu = upper_blocks(K);
  const int u = blockIdx.x / 8, piece = blockIdx.x % 8;
  const int t = threadIdx.x, f = piece * 32 + (t & 31), sl = t >> 5;
  floatx4 acc = floatx4{0, 0, 0, 0};
  int c = sl;
  for (; c + 3 * kRedSlices < nchunks; c += 4 * kRedSlices) {
    const floatx4 a0 = *(const floatx4*)(partial + ((int64_t)c * nu + u) * 1024 + 4 * f);
    const floatx4 a1 = *(const floatx4*)(partial + ((int64_t)(c + kRedSlices) * nu + u) * 1024 + 4 * f);
    const floatx4 a2 = *(const floatx4*)(partial + ((int64_t)(c + 2 * kRedSlices) * nu + u) * 1024 + 4 * f);
    const floatx4 a3 = *(const floatx4*)(partial + ((int64_t)(c + 3 * kRedSlices) * nu + u) * 1024 + 4 * f);
    acc += a0;
    acc += a1;
    acc += a2;
    acc += a3;
  }
  for (; c < nchunks; c += kRedSlices)
    acc += *(const floatx4*)(partial + ((int64_t)c * nu + u) * 1024 + 4 * f);
  part[t] = acc;
  __syncthreads();
  if (sl == 0) {
    floatx4 tot = part[t];
    for (int k = 1; k < kRedSlices; k++) tot += part[k * 32 + (t & 31)];
    int bi, bj;
    {
      int uu = u, i = 0, rowlen = nb;
      while (uu >= rowlen) {
        uu -= rowlen;
        i++;
        rowlen--;
      }
      bi = i;
      bj = i + uu;
    }
    const int rr = (4 * f) / 32, cc = (4 * f) % 32;  // element (rr, cc..cc+3) of the block
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int gi = 32 * bi + rr, gj = 32 * bj + cc + e;
      if (gi < K && gj < K) {
        C[(int64_t)gi * ldc + gj] = tot[e];
        if (bi != bj) C[(int64_t)gj * ldc + gi] = tot[e];
        if (panel && rows_layout) {
          put_panel_rows(panel, K, diag_one, tile, gi, gj, tot[e]);
          if (bi != bj) put_panel_rows(panel, K, diag_one, tile, gj, gi, tot[e]);
        } else if (panel) {
          put_panel(panel, K, diag_one, tile, gi, gj, tot[e]);
          if (bi != bj) put_panel(panel, K, diag_one, tile, gj, gi, tot[e]);
        }
      }
    }
  }
}

}  // namespace

constexpr int kMaxChunks = 256;

int gram_max_chunks() { return kMaxChunks; }

int gram_chunks(int64_t rows, int device_cus) {
  int64_t n = (rows + 63) / 64;
  if (n > device_cus) n = device_cus;
  if (n > kMaxChunks) n = kMaxChunks;
  return n < 1 ? 1 : (int)n;
}

size_t gram_partial_floats(int K, int chunks) { return (size_t)chunks * upper_blocks(K) * 1024; }

hipError_t gram_xtx(const float* X, int64_t rows, int K, float* C, int64_t ldc, float* partial,
                    int chunks, hipStream_t s, float* panel, int diag_one, int tile, bool rows_layout) {
  if (K <= 0) return hipSuccess;
  if (K > kMaxK || chunks < 1) return hipErrorInvalidValue;
  const int64_t rpc = (rows + chunks - 1) / chunks;
  const int passes = (upper_blocks(K) + kBlocksPerPass - 1) / kBlocksPerPass;
  const size_t bytes = (size_t)kRS * 32 * nblk(K) * 4;
  const bool vec = (K % 4 == 0) && (((uintptr_t)X & 15) == 0);
  const void* fn = vec ? (const void*)gram_partial<true> : (const void*)gram_partial<false>;
  if (bytes > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  const dim3 grid((unsigned)chunks, (unsigned)passes);
  if (vec) gram_partial<true><<<grid, kThreads, bytes, s>>>(X, rows, K, rpc, partial);
  else gram_partial<false><<<grid, kThreads, bytes, s>>>(X, rows, K, rpc, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  gram_reduce<<<(unsigned)(upper_blocks(K) * 8), kRedThreads, 0, s>>>(partial, chunks, K, C, ldc, panel,
                                                                diag_one, tile, rows_layout ? 1 : 0);
  return hipGetLastError();
}

}  // namespace plnmf
