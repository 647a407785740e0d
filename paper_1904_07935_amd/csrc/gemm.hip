// Matrix-core GEMM for gfx950: C = op(A) op(B) with FP32 accumulation.
//
// Used for every dense product of the sweep (A H^T and A^T W on dense A, Alg. 1
// statements forming R and P), the Gram matrices W^T W and H H^T (the S and Q
// statements of Alg. 1), the dense residual of the objective (Eq. 2), and the
// warm-start network's forward and backward products.
//
// Tiles of 128 x 128 per workgroup, four wave64s in a 2 x 2 arrangement, each
// owning 64 x 64 = 2 x 2 blocks of the 32 x 32 MFMA output.  Operands are staged
// through double-buffered LDS in the layout each MFMA variant reads with
// conflict-light unit-stride lane access:
//   FP32  v_mfma_f32_32x32x2_f32   lane l supplies A[l%32][l/32], B[l/32][l%32]
//         -> LDS k-major: As[k][m], Bs[k][n]; BK = 16
//   BF16  v_mfma_f32_32x32x16_bf16 lane l supplies A[l%32][8(l/32)..+7] and
//         B[8(l/32)..+7][l%32] -> LDS k-contiguous: As[m][k], Bs[n][k]; BK = 32
// Output block layout (both): lane l holds C[8j + 4(l/32) + i][l%32], j,i < 4.
// Split-K writes FP32 partials that a fixed-order pass sums (deterministic).
#include <cmath>
#include <type_traits>

#include "internal.hpp"

namespace plnmf {
namespace {

constexpr int BM = 128, BN = 128;

// Operand tiles are read through buffer descriptors whose base is the step's
// tile origin.  A lane whose element lies outside the matrix (a row past M or
// N, a term past the end of its split) uses an offset past the descriptor's
// range, and the hardware returns zeros for it without touching memory: no
// branches, so the loads of a step issue back to back and the wait before the
// LDS store counts them exactly.  Valid offsets stay below 2^31 bytes (the
// host routes leading dimensions of 2^22 or more to the scalar path).
constexpr uint32_t kOutside = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_view(const void* base, int64_t bytes) {
  const int64_t n = bytes < 0 ? 0 : (bytes > 0x7fffffff ? 0x7fffffff : bytes);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)n, 0x00020000);
}
__device__ __forceinline__ floatx4 ld4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ bf16x8 ld8h(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

__device__ __forceinline__ float gelu_grad_f(float z) {
  float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  float pdf = expf(-0.5f * z * z) * 0.39894228040143268f;
  return cdf + z * pdf;
}

// Epilogue over one wave's 2 x 2 blocks.  `acc[i][j]` is the 32x32 block at
// rows r0 + 32 i, cols c0 + 32 j.  Every field is passed by value so nothing
// here takes the address of the kernel argument block.  The epilogue kind and
// whether the wave's 64 x 64 block lies wholly inside C are template
// parameters: each instantiation is one straight run of 64 element updates,
// with no per-element dispatch on the kind and, inside C, no bounds checks.
template <int EPI, bool FULL>
__device__ __forceinline__ void epi_block(int64_t M, int64_t N, float* __restrict__ out,
                                          int64_t ldo, bool split, const float* __restrict__ bias,
                                          const float* Dm, int64_t ldd, void* __restrict__ C2,
                                          float* C, int64_t ldc, floatx16 (&acc)[2][2],
                                          int64_t r0, int64_t c0, bool mirror, float mu_delta,
                                          double& ss) {
  const int lane = threadIdx.x & 63;
  const float* bs = (EPI != EPI_STORE || !split) ? bias : nullptr;
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
      for (int jj = 0; jj < 4; jj++)
#pragma unroll
        for (int ii = 0; ii < 4; ii++) {
          const int64_t m = r0 + 32 * i + 8 * jj + 4 * (lane >> 5) + ii;
          const int64_t n = c0 + 32 * j + (lane & 31);
          if (!FULL && (m >= M || n >= N)) continue;
          float v = acc[i][j][jj * 4 + ii];
          if constexpr (EPI == EPI_STORE) {
            if (bs) v += bs[n];
            out[m * ldo + n] = v;
            if (mirror) out[n * ldo + m] = v;  // symmetric product, tile above the diagonal
          } else if constexpr (EPI == EPI_RESID_SQ) {
            const float e = Dm[m * ldd + n] - v;
            ss += (double)e * (double)e;
          } else if constexpr (EPI == EPI_BIAS_GELU) {
            const float z = v + bs[n];
            if (C) C[m * ldc + n] = z;
            ((__bf16*)C2)[m * ldc + n] = (__bf16)gelu_f(z);
          } else if constexpr (EPI == EPI_BIAS_SOFTPLUS) {
            const float z = v + bs[n];
            if (C) C[m * ldc + n] = z;
            ((float*)C2)[m * ldc + n] = softplus_f(z);
          } else if constexpr (EPI == EPI_GELU_GRAD) {
            const float d = v * gelu_grad_f(Dm[m * ldd + n]);
            if (C) C[m * ldc + n] = d;
            ((__bf16*)C2)[m * ldc + n] = (__bf16)d;
          } else if constexpr (EPI == EPI_MU) {
            const float num = Dm[m * ldd + n], x = ((const float*)C2)[m * ldc + n];
            C[m * ldc + n] = x * num / (v + mu_delta);
          }
        }
}

template <int EPI>
__device__ __forceinline__ void epi_kind(int64_t M, int64_t N, float* __restrict__ out,
                                         int64_t ldo, bool split, const float* __restrict__ bias,
                                         const float* Dm, int64_t ldd, void* __restrict__ C2,
                                         float* C, int64_t ldc, floatx16 (&acc)[2][2], int64_t r0,
                                         int64_t c0, bool mirror, float mu_delta, double& ss) {
  if (r0 + 64 <= M && c0 + 64 <= N)
    epi_block<EPI, true>(M, N, out, ldo, split, bias, Dm, ldd, C2, C, ldc, acc, r0, c0, mirror,
                         mu_delta, ss);
  else
    epi_block<EPI, false>(M, N, out, ldo, split, bias, Dm, ldd, C2, C, ldc, acc, r0, c0, mirror,
                          mu_delta, ss);
}

__device__ __forceinline__ void epilogue(int epi, int64_t M, int64_t N, float* __restrict__ out,
                                         int64_t ldo, bool split, const float* __restrict__ bias,
                                         const float* Dm, int64_t ldd,
                                         void* __restrict__ C2, float* C,
                                         int64_t ldc, double* __restrict__ red_out,
                                         floatx16 (&acc)[2][2], int64_t r0, int64_t c0,
                                         double* red_smem, bool mirror, float mu_delta,
                                         int64_t red_slot) {
  double ss = 0.0;
#define PLNMF_EPI(K)                                                                        \
  epi_kind<K>(M, N, out, ldo, split, bias, Dm, ldd, C2, C, ldc, acc, r0, c0, mirror, mu_delta, \
              ss)
  switch (epi) {
    case EPI_STORE: PLNMF_EPI(EPI_STORE); break;
    case EPI_RESID_SQ: PLNMF_EPI(EPI_RESID_SQ); break;
    case EPI_BIAS_GELU: PLNMF_EPI(EPI_BIAS_GELU); break;
    case EPI_BIAS_SOFTPLUS: PLNMF_EPI(EPI_BIAS_SOFTPLUS); break;
    case EPI_GELU_GRAD: PLNMF_EPI(EPI_GELU_GRAD); break;
    case EPI_MU: PLNMF_EPI(EPI_MU); break;
  }
#undef PLNMF_EPI
  if (epi == EPI_RESID_SQ) {
    const int lane = threadIdx.x & 63;
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
    const int w = threadIdx.x >> 6;
    if (lane == 0) red_smem[w] = ss;
    __syncthreads();
    if (threadIdx.x == 0) {
      const double t = red_smem[0] + red_smem[1] + red_smem[2] + red_smem[3];
      red_out[red_slot] = t;
    }
  }
}

// XCD-aware tile order.  Workgroups go to the eight XCDs round robin by
// linear id; this maps the ids that land on one XCD to a contiguous run of
// tiles, N-tile fastest, so the tiles that share an A row block (and, for a
// split, a B block) run on the same XCD and find it in that XCD's L2.  A
// bijection on [0, tiles) whatever the dispatch order.
__device__ __forceinline__ void tile_of(int& tx, int& ty, int& tz) {
  const unsigned gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const unsigned total = gx * gy * gz;
  const unsigned lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const unsigned xcd = lin & 7, q = lin >> 3, per = total >> 3, rem = total & 7;
  const unsigned t = xcd < rem ? xcd * (per + 1) + q : rem * (per + 1) + (xcd - rem) * per + q;
  ty = (int)(t % gy);
  tx = (int)((t / gy) % gx);
  tz = (int)(t / (gx * gy));
}

// Global -> register -> LDS staging of one K-step of the A and B tiles.
template <typename T, bool AT, bool BT, bool VEC, int BK>
struct Stage;

// FP32: As[k][m], Bs[k][n] (k-major), BK = 16
template <bool AT, bool BT, bool VEC>
struct Stage<float, AT, BT, VEC, 16> {
  static constexpr int LDS_A = BM + 4, LDS_B = BN + 4;
  floatx4 ra[2], rb[2];
  float sa[8], sb[8];
  __device__ __forceinline__ void load(const float* __restrict__ A, const float* __restrict__ B,
                                       int64_t lda, int64_t ldb, int64_t M, int64_t N,
                                       int64_t m0, int64_t n0, int64_t k0, int64_t ke, int64_t Kd,
                                       int tid) {
    if constexpr (VEC) {
      // this step's tile origin in each operand (wave-uniform), and the bytes
      // from there to the operand's last element
      const int64_t a0 = AT ? k0 * lda + m0 : m0 * lda + k0;
      const int64_t b0 = BT ? n0 * ldb + k0 : k0 * ldb + n0;
      const int64_t a_end = AT ? (Kd - 1) * lda + M : (M - 1) * lda + Kd;
      const int64_t b_end = BT ? (N - 1) * ldb + Kd : (Kd - 1) * ldb + N;
      const __amdgpu_buffer_rsrc_t va = tile_view(A + a0, (a_end - a0) * 4);
      const __amdgpu_buffer_rsrc_t vb = tile_view(B + b0, (b_end - b0) * 4);
#pragma unroll
      for (int p = 0; p < 2; p++) {
        const int idx = tid + 256 * p;
        if constexpr (!AT) {  // along k
          const int ml = idx >> 2, kq = idx & 3;
          const bool ok = m0 + ml < M && k0 + 4 * kq < ke;
          ra[p] = ld4(va, ok ? (uint32_t)(ml * lda + 4 * kq) * 4u : kOutside);
        } else {  // along m
          const int kl = idx >> 5, mq = idx & 31;
          const bool ok = m0 + 4 * mq < M && k0 + kl < ke;
          ra[p] = ld4(va, ok ? (uint32_t)(kl * lda + 4 * mq) * 4u : kOutside);
        }
        if constexpr (!BT) {  // along n
          const int kl = idx >> 5, nq = idx & 31;
          const bool ok = n0 + 4 * nq < N && k0 + kl < ke;
          rb[p] = ld4(vb, ok ? (uint32_t)(kl * ldb + 4 * nq) * 4u : kOutside);
        } else {  // along k
          const int nl = idx >> 2, kq = idx & 3;
          const bool ok = n0 + nl < N && k0 + 4 * kq < ke;
          rb[p] = ld4(vb, ok ? (uint32_t)(nl * ldb + 4 * kq) * 4u : kOutside);
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; e++) {
        const int idx = tid + 256 * e;           // element of the 128 x 16 tile
        const int kl = idx & 15, ml = idx >> 4;  // k fastest
        const int64_t k = k0 + kl;
        const int64_t m = m0 + ml, n = n0 + ml;
        sa[e] = (m < M && k < ke) ? (AT ? A[k * lda + m] : A[m * lda + k]) : 0.0f;
        sb[e] = (n < N && k < ke) ? (BT ? B[n * ldb + k] : B[k * ldb + n]) : 0.0f;
      }
    }
  }
  __device__ __forceinline__ void store(float (*As)[LDS_A], float (*Bs)[LDS_B], int tid) {
    if constexpr (VEC) {
#pragma unroll
      for (int p = 0; p < 2; p++) {
        const int idx = tid + 256 * p;
        if constexpr (!AT) {
          const int ml = idx >> 2, kq = idx & 3;
#pragma unroll
          for (int e = 0; e < 4; e++) As[4 * kq + e][ml] = ra[p][e];
        } else {
          const int kl = idx >> 5, mq = idx & 31;
          *(floatx4*)&As[kl][4 * mq] = ra[p];
        }
        if constexpr (!BT) {
          const int kl = idx >> 5, nq = idx & 31;
          *(floatx4*)&Bs[kl][4 * nq] = rb[p];
        } else {
          const int nl = idx >> 2, kq = idx & 3;
#pragma unroll
          for (int e = 0; e < 4; e++) Bs[4 * kq + e][nl] = rb[p][e];
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; e++) {
        const int idx = tid + 256 * e;
        const int kl = idx & 15, ml = idx >> 4;
        As[kl][ml] = sa[e];
        Bs[kl][ml] = sb[e];
      }
    }
  }
};

// BF16: As[m][k], Bs[n][k] (k-contiguous), BK = 32
template <bool AT, bool BT, bool VEC>
struct Stage<__bf16, AT, BT, VEC, 32> {
  static constexpr int LDS_K = 32 + 8;  // 80-byte rows keep 16-byte alignment
  bf16x8 ra[2], rb[2];
  __bf16 sa[16], sb[16];
  __device__ __forceinline__ void load(const __bf16* __restrict__ A, const __bf16* __restrict__ B,
                                       int64_t lda, int64_t ldb, int64_t M, int64_t N,
                                       int64_t m0, int64_t n0, int64_t k0, int64_t ke, int64_t Kd,
                                       int tid) {
    if constexpr (VEC) {
      const int64_t a0 = AT ? k0 * lda + m0 : m0 * lda + k0;
      const int64_t b0 = BT ? n0 * ldb + k0 : k0 * ldb + n0;
      const int64_t a_end = AT ? (Kd - 1) * lda + M : (M - 1) * lda + Kd;
      const int64_t b_end = BT ? (N - 1) * ldb + Kd : (Kd - 1) * ldb + N;
      const __amdgpu_buffer_rsrc_t va = tile_view(A + a0, (a_end - a0) * 2);
      const __amdgpu_buffer_rsrc_t vb = tile_view(B + b0, (b_end - b0) * 2);
#pragma unroll
      for (int p = 0; p < 2; p++) {
        const int idx = tid + 256 * p;
        if constexpr (!AT) {
          const int ml = idx >> 2, kq = idx & 3;
          const bool ok = m0 + ml < M && k0 + 8 * kq < ke;
          ra[p] = ld8h(va, ok ? (uint32_t)(ml * lda + 8 * kq) * 2u : kOutside);
        } else {
          const int kl = idx >> 4, mq = idx & 15;
          const bool ok = m0 + 8 * mq < M && k0 + kl < ke;
          ra[p] = ld8h(va, ok ? (uint32_t)(kl * lda + 8 * mq) * 2u : kOutside);
        }
        if constexpr (!BT) {
          const int kl = idx >> 4, nq = idx & 15;
          const bool ok = n0 + 8 * nq < N && k0 + kl < ke;
          rb[p] = ld8h(vb, ok ? (uint32_t)(kl * ldb + 8 * nq) * 2u : kOutside);
        } else {
          const int nl = idx >> 2, kq = idx & 3;
          const bool ok = n0 + nl < N && k0 + 8 * kq < ke;
          rb[p] = ld8h(vb, ok ? (uint32_t)(nl * ldb + 8 * kq) * 2u : kOutside);
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; e++) {
        const int idx = tid + 256 * e;           // element of the 128 x 32 tile
        const int kl = idx & 31, ml = idx >> 5;  // k fastest
        const int64_t k = k0 + kl;
        const int64_t m = m0 + ml, n = n0 + ml;
        sa[e] = (m < M && k < ke) ? (AT ? A[k * lda + m] : A[m * lda + k]) : (__bf16)0.0f;
        sb[e] = (n < N && k < ke) ? (BT ? B[n * ldb + k] : B[k * ldb + n]) : (__bf16)0.0f;
      }
    }
  }
  __device__ __forceinline__ void store(__bf16 (*As)[LDS_K], __bf16 (*Bs)[LDS_K], int tid) {
    if constexpr (VEC) {
#pragma unroll
      for (int p = 0; p < 2; p++) {
        const int idx = tid + 256 * p;
        if constexpr (!AT) {
          const int ml = idx >> 2, kq = idx & 3;
          *(bf16x8*)&As[ml][8 * kq] = ra[p];
        } else {
          const int kl = idx >> 4, mq = idx & 15;
#pragma unroll
          for (int e = 0; e < 8; e++) As[8 * mq + e][kl] = ra[p][e];
        }
        if constexpr (!BT) {
          const int kl = idx >> 4, nq = idx & 15;
#pragma unroll
          for (int e = 0; e < 8; e++) Bs[8 * nq + e][kl] = rb[p][e];
        } else {
          const int nl = idx >> 2, kq = idx & 3;
          *(bf16x8*)&Bs[nl][8 * kq] = rb[p];
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; e++) {
        const int idx = tid + 256 * e;
        const int kl = idx & 31, ml = idx >> 5;
        As[ml][kl] = sa[e];
        Bs[ml][kl] = sb[e];
      }
    }
  }
};

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  static constexpr int BK = 16;
  // one K-step of 2 on the four 32x32 blocks of this wave
  template <typename AS, typename BS>
  __device__ __forceinline__ static void step(AS As, BS Bs, floatx16 (&acc)[2][2], int wm, int wn,
                                              int lane) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const int kr = kk + (lane >> 5);
      const float a0 = As[kr][wm * 64 + (lane & 31)];
      const float a1 = As[kr][wm * 64 + 32 + (lane & 31)];
      const float b0 = Bs[kr][wn * 64 + (lane & 31)];
      const float b1 = Bs[kr][wn * 64 + 32 + (lane & 31)];
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
};
template <>
struct Mfma<__bf16> {
  static constexpr int BK = 32;
  template <typename AS, typename BS>
  __device__ __forceinline__ static void step(AS As, BS Bs, floatx16 (&acc)[2][2], int wm, int wn,
                                              int lane) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const int kc = kk + 8 * (lane >> 5);
      const bf16x8 a0 = *(const bf16x8*)&As[wm * 64 + (lane & 31)][kc];
      const bf16x8 a1 = *(const bf16x8*)&As[wm * 64 + 32 + (lane & 31)][kc];
      const bf16x8 b0 = *(const bf16x8*)&Bs[wn * 64 + (lane & 31)][kc];
      const bf16x8 b1 = *(const bf16x8*)&Bs[wn * 64 + 32 + (lane & 31)][kc];
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
};

// Main loop: two register stages and two LDS buffers.  The global load of
// K-step k + 2 is issued before computing step k and stored to LDS after
// computing step k + 1, so each load has two compute steps to arrive.  The
// loop body is a pair of steps (an odd count gets one step of zeros).
//
// FP32: two-level accumulation.  The matrix cores accumulate each pair of
// K-steps (32 terms) into a fresh accumulator, which is then added to the
// running total.  A single accumulator chain over a contraction of n terms
// carries a rounding error that grows like sqrt(n) units of FP32 rounding;
// with chunks of c terms the chain is n / c long, which cuts the error of the
// 800 - 10^4 term products several times.  A chunk per loop iteration keeps
// the fresh accumulator local to the body, so it stays in the matrix-core
// registers instead of moving through the VALU every step.
// BF16: one chain.  The inputs' rounding (2^-9 relative) dwarfs the FP32
// chain's, and at BF16 rates the chunk additions would cost as much VALU time
// as the products take on the matrix cores.
template <typename T, typename St, typename TA, typename TB>
__device__ __forceinline__ void pipeline(TA As, TB Bs, const T* __restrict__ A,
                                         const T* __restrict__ B, int64_t lda, int64_t ldb,
                                         int64_t M, int64_t N, int64_t Kd, int64_t m0, int64_t n0,
                                         int64_t kb, int64_t ke, int nk, int tid,
                                         floatx16 (&tot)[2][2], int wm, int wn, int lane) {
  constexpr int BK = Mfma<T>::BK;
  constexpr bool kChunked = std::is_same<T, float>::value;
  if (nk <= 0) return;
  St s0, s1;
  s0.load(A, B, lda, ldb, M, N, m0, n0, kb, ke, Kd, tid);
  s1.load(A, B, lda, ldb, M, N, m0, n0, kb + BK, ke, Kd, tid);
  s0.store(As[0], Bs[0], tid);
  __syncthreads();
  auto pair = [&](int kt, floatx16(&acc)[2][2]) {
    s0.load(A, B, lda, ldb, M, N, m0, n0, kb + (int64_t)(kt + 2) * BK, ke, Kd, tid);
    Mfma<T>::step(As[0], Bs[0], acc, wm, wn, lane);
    s1.store(As[1], Bs[1], tid);
    __syncthreads();
    s1.load(A, B, lda, ldb, M, N, m0, n0, kb + (int64_t)(kt + 3) * BK, ke, Kd, tid);
    Mfma<T>::step(As[1], Bs[1], acc, wm, wn, lane);
    s0.store(As[0], Bs[0], tid);
    __syncthreads();
  };
  if constexpr (kChunked) {
#pragma unroll 1
    for (int kt = 0; kt < nk; kt += 2) {
      floatx16 acc[2][2];
#pragma unroll
      for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
          for (int e = 0; e < 16; e++) acc[i][j][e] = 0.0f;
      pair(kt, acc);
#pragma unroll
      for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) tot[i][j] += acc[i][j];
    }
  } else {
#pragma unroll 1
    for (int kt = 0; kt < nk; kt += 2) pair(kt, tot);
  }
}

template <typename T, bool AT, bool BT, bool VEC>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  constexpr int BK = Mfma<T>::BK;
  using St = Stage<T, AT, BT, VEC, BK>;
  // scalar copies of the argument block (keeps its address untaken)
  const T* __restrict__ A = (const T*)g.A;
  const T* __restrict__ B = (const T*)g.B;
  const int64_t M = g.M, N = g.N, Kd = g.Kd, lda = g.lda, ldb = g.ldb;
  const int splits = g.splits;
  const int64_t kps = g.k_per_split;
  const int sym = g.sym;
  int tx, ty, tz;
  tile_of(tx, ty, tz);
  if (sym && ty < tx) return;  // symmetric product: upper tiles only
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int64_t m0 = (int64_t)tx * BM, n0 = (int64_t)ty * BN;
  int64_t kb = 0, ke = Kd;
  if (splits > 1) {
    kb = (int64_t)tz * kps;
    ke = kb + kps < Kd ? kb + kps : Kd;
  }
  const int nk = (int)((ke - kb + BK - 1) / BK);
  __shared__ double red[4];
  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
      for (int e = 0; e < 16; e++) acc[i][j][e] = 0.0f;

  if constexpr (std::is_same<T, float>::value) {
    __shared__ float As[2][BK][St::LDS_A];
    __shared__ float Bs[2][BK][St::LDS_B];
    pipeline<T, St>(As, Bs, A, B, lda, ldb, M, N, Kd, m0, n0, kb, ke, nk, tid, acc, wm, wn, lane);
  } else {
    __shared__ __bf16 As[2][BM][St::LDS_K];
    __shared__ __bf16 Bs[2][BN][St::LDS_K];
    pipeline<T, St>(As, Bs, A, B, lda, ldb, M, N, Kd, m0, n0, kb, ke, nk, tid, acc, wm, wn, lane);
  }
  const bool split = splits > 1;
  float* out = split ? g.partial + (int64_t)tz * M * N : g.C;
  epilogue(g.epi, M, N, out, split ? N : g.ldc, split, g.bias, g.D, g.ldd, g.C2, g.C, g.ldc,
           g.red_out, acc, m0 + wm * 64, n0 + wn * 64, red,
           sym && !split && ty != tx, g.mu_delta, (int64_t)ty * gridDim.x + tx);
}

__global__ void splitk_reduce_kernel(const float* __restrict__ partial, int splits, int64_t M,
                                     int64_t N, float* __restrict__ C, int64_t ldc,
                                     const float* __restrict__ bias, int sym) {
  const int64_t total = M * N;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = i / N, n = i - m * N;
    // symmetric products computed only tiles at or above the diagonal
    const int64_t src = (sym && m / BM > n / BN) ? n * N + m : i;
    float s = 0.0f;
    for (int z = 0; z < splits; z++) s += partial[(int64_t)z * total + src];
    if (bias) s += bias[n];
    C[m * ldc + n] = s;
  }
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

// Split-K choice: the estimated time of `s` splits is the number of rounds of
// workgroups over the chip's slots (256 CUs, two workgroups each) times the
// matrix-core time of one split's share of the contraction, plus the HBM time
// of writing and summing the s partial products.  Every split keeps at least
// 256 terms of the contraction.
int gemm_pick_splits(int64_t M, int64_t N, int64_t Kd, int64_t* k_per_split) {
  const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  constexpr double kSlots = 512.0;
  constexpr double kTermSec = 2.0 * BM * BN / 307.2e9;  // one term of a tile, FP32 rate per slot
  constexpr double kBytesPerSec = 4.0e12;
  int best = 1;
  double best_t = 0.0;
  for (int s = 1; s <= 256; s++) {
    if (s > 1 && Kd / s < 256) break;
    int64_t kps = (Kd + s - 1) / s;
    kps = (kps + 31) / 32 * 32;
    const int real = (int)((Kd + kps - 1) / kps);
    if (real != s) continue;
    const double rounds = std::ceil((double)(tiles * s) / kSlots);
    double t = rounds * (double)kps * kTermSec;
    if (s > 1) t += (2.0 * s + 1.0) * (double)M * (double)N * 4.0 / kBytesPerSec;
    if (s == 1 || t < best_t * 0.97) {  // a split must pay for itself
      best = s;
      best_t = t;
    }
  }
  int64_t kps = (Kd + best - 1) / best;
  kps = (kps + 31) / 32 * 32;  // a multiple of both BK values
  const int splits = (int)((Kd + kps - 1) / kps);
  if (k_per_split) *k_per_split = kps;
  return splits;
}

hipError_t splitk_reduce(const float* partial, int splits, int64_t M, int64_t N, float* C,
                         int64_t ldc, const float* bias, int sym, hipStream_t s) {
  const int64_t total = M * N;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  splitk_reduce_kernel<<<blocks, 256, 0, s>>>(partial, splits, M, N, C, ldc, bias, sym);
  return hipGetLastError();
}

hipError_t gemm(Elem t, bool a_trans, bool b_trans, const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int vw = t == Elem::F32 ? 4 : 8;
  // vector path: the contiguous extent of each operand and its leading dim
  // are multiples of the vector width, and the base is 16-byte aligned
  const int64_t a_cont = a_trans ? g.M : g.Kd, b_cont = b_trans ? g.Kd : g.N;
  const bool vec = aligned16(g.A) && aligned16(g.B) && g.lda % vw == 0 && g.ldb % vw == 0 &&
                   g.lda < (int64_t(1) << 22) && g.ldb < (int64_t(1) << 22) &&
                   a_cont % vw == 0 && b_cont % vw == 0 &&
                   (g.splits <= 1 || g.k_per_split % vw == 0);
  dim3 grid((unsigned)((g.M + BM - 1) / BM), (unsigned)((g.N + BN - 1) / BN),
            (unsigned)(g.splits > 1 ? g.splits : 1));
  const int code = (a_trans ? 4 : 0) | (b_trans ? 2 : 0) | (vec ? 1 : 0);
#define PLNMF_GEMM_CASES(T)                                                             \
  switch (code) {                                                                       \
    case 0: gemm_kernel<T, false, false, false><<<grid, 256, 0, s>>>(g); break;         \
    case 1: gemm_kernel<T, false, false, true><<<grid, 256, 0, s>>>(g); break;          \
    case 2: gemm_kernel<T, false, true, false><<<grid, 256, 0, s>>>(g); break;          \
    case 3: gemm_kernel<T, false, true, true><<<grid, 256, 0, s>>>(g); break;           \
    case 4: gemm_kernel<T, true, false, false><<<grid, 256, 0, s>>>(g); break;          \
    case 5: gemm_kernel<T, true, false, true><<<grid, 256, 0, s>>>(g); break;           \
    case 6: gemm_kernel<T, true, true, false><<<grid, 256, 0, s>>>(g); break;           \
    case 7: gemm_kernel<T, true, true, true><<<grid, 256, 0, s>>>(g); break;            \
  }
  if (t == Elem::F32) {
    PLNMF_GEMM_CASES(float)
  } else {
    PLNMF_GEMM_CASES(__bf16)
  }
#undef PLNMF_GEMM_CASES
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (g.splits > 1 && g.epi == EPI_STORE)
    return splitk_reduce(g.partial, g.splits, g.M, g.N, g.C, g.ldc, g.bias, g.sym, s);
  return hipSuccess;
}

}  // namespace plnmf
