// Tiled FAST-HALS updates (Alg. 1 H and W loops, reordered as in Sec. 3.3,
// Alg. 2 and Eq. 4-6) for gfx950.
//
// Both halves are the same recurrence over the rows of a factor X [rows, K]
// (X = H^T for the H half, X = W for the W half), column t in order:
//
//   y[r,t] = Bterm[r,t] + cdiag(t) X[r,t] - sum_{l != t} X[r,l] G[l,t]
//   X[r,t] = max(eps, y[r,t])                      (W half: then / ||X[:,t]||)
//
// with columns l < t already new.  H half: Bterm = R = A^T W, G = S = W^T W,
// cdiag = 1 - S_tt (the H_k + R_k - H^T S_k of Alg. 1).  W half: Bterm = P =
// A H^T, G = Q = H H^T, cdiag = 0 (W_k Q_kk cancels the l = k term of W Q_k).
//
// Tiles of T = 32 columns.  For tile [a, b) one matrix-core product over the
// whole contraction forms every contribution that does not depend on the
// tile's own new values: columns l < a are already new in X (the new-to-right
// work of phase 3, Eq. 6), columns l >= b are still old (the old-to-left work
// of phase 1, Eq. 4), and inside the tile the old values of l > t plus the
// diagonal.  Done in place, one product per tile replaces both GEMM phases.
// Its B operand (G's tile columns with the in-tile mask and diagonal folded
// in) is staged once per tile in LDS; the A operand (this group's rows of X)
// streams from global memory in double-buffered register chunks.  What remains
// is phase 2 (Eq. 5 with +P, as in Alg. 2): within the tile, column by column,
// clip, normalise (W), and apply the new value to the tile's later columns.
//
// The W half needs the L2 norm of each finished column over all rows before
// the next column can be clipped (Alg. 1 normalises inside the k loop), so the
// W kernel is persistent: its workgroups are co-resident (cooperative launch)
// and exchange one FP32 partial per column through tagged 64-bit slots.  Every
// workgroup sums all partials in the same fixed order, so every workgroup (and
// every run) gets the bitwise-identical norm; the paper's atomicAdd of partial
// sums (Alg. 4) would be order-dependent.  Only the update of the next column
// sits between two exchanges; the rest of the in-tile work runs while the
// exchange is in flight.  Waits are bounded: on a timeout a status bit is set,
// every group stops waiting, and the kernel still runs to completion.
#include "internal.hpp"

namespace plnmf {
namespace {

constexpr int T = kTile;
constexpr int TP = T + 1;  // LDS row pitch (bank spread)
constexpr int kMaxRowsW = 512;
constexpr int kRowsH = 32;

// dynamic LDS layout (floats): xt [rows][TP] | gt [T][TP] | part [4][32][TP] |
// bp [Kp][TP] | red [8], with Kp = K rounded up to a multiple of 8 (the product
// reads the contraction in groups of 8; rows >= K of bp hold zeros)
struct Smem {
  float* xt;
  float* gt;
  float* part;
  float* bp;
  float* red;
};

__host__ __device__ inline int kpad(int K) { return (K + 7) / 8 * 8; }

__host__ __device__ inline size_t smem_floats(int rows, int K) {
  return (size_t)rows * TP + (size_t)T * TP + 4 * 32 * TP + (size_t)kpad(K) * TP + 8;
}

__device__ __forceinline__ Smem carve(float* base, int rows, int K) {
  Smem s;
  s.xt = base;
  s.gt = s.xt + rows * TP;
  s.part = s.gt + T * TP;
  s.bp = s.part + 4 * 32 * TP;
  s.red = s.bp + kpad(K) * TP;
  return s;
}

__device__ __forceinline__ unsigned long long pack_slot(unsigned tag, float v) {
  return ((unsigned long long)tag << 32) | (unsigned long long)__float_as_uint(v);
}

// The slot array is replicated kSlotReplicas times (kSlotStride apart): every
// group writes its partial into all replicas and polls only replica g %
// kSlotReplicas, so the polling traffic of all groups does not converge on the
// same few cache lines.  Called by lanes 0..kSlotReplicas-1 of one wave.
__device__ __forceinline__ void publish(unsigned long long* slots, int groups, int g, unsigned tag,
                                        int par, float mine, int replica) {
  __hip_atomic_store(slots + (int64_t)replica * kSlotStride + (int64_t)par * groups + g,
                     pack_slot(tag, mine), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Chip-wide fixed-order sum of the published partials (wave 0, all lanes).
__device__ float collect_sum(const unsigned long long* slots, int groups, int g, unsigned tag,
                             int par, int32_t* status) {
  const int lane = threadIdx.x & 63;
  const unsigned long long* base =
      slots + (int64_t)(g % kSlotReplicas) * kSlotStride + (int64_t)par * groups;
  constexpr int MAXS = 16;  // groups <= 1024
  unsigned long long v[MAXS];
  int spins = 0;
  bool done;
  do {
    done = true;
#pragma unroll
    for (int s = 0; s < MAXS; s++) {
      const int i = lane + 64 * s;
      if (i < groups) {
        v[s] = __hip_atomic_load(base + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        done = done && ((unsigned)(v[s] >> 32) == tag);
      }
    }
    // give up at once if any workgroup already timed out (bounded total wait)
    if (!done && (++spins & 255) == 0 &&
        (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 256))
      break;
  } while (!done && spins < kSpinLimit);
  if (!done) atomicOr(status, 256);
  float t = 0.0f;
#pragma unroll
  for (int s = 0; s < MAXS; s++)
    if (lane + 64 * s < groups) t += __uint_as_float((unsigned)v[s]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
  return t;
}

// B operand of the tile product: contraction row l, output column c of the tile [a0, b0).
__device__ __forceinline__ float bm_value(const float* __restrict__ G, int K, int l, int c, int a0,
                                          int b0, int diag_one) {
  if (l >= K || c >= b0) return 0.0f;
  const float gv = G[(int64_t)l * K + c];
  if (l == c) return diag_one ? 1.0f - gv : 0.0f;
  if (l >= a0 && l < b0 && l < c) return 0.0f;  // new in-tile value: phase 2
  return -gv;
}

constexpr int CH = 8;  // float4 groups (of 8 contraction indices) per register chunk

template <bool VEC>
__device__ __forceinline__ void load_chunk(floatx4 (&buf)[CH], const float* __restrict__ xr, bool rok,
                                           int l0, int le, int K, int h) {
#pragma unroll
  for (int gi = 0; gi < CH; gi++) {
    const int lc = l0 + 8 * gi + 4 * h;
    if constexpr (VEC) {
      buf[gi] = (rok && lc < le) ? *(const floatx4*)(xr + lc) : floatx4{0, 0, 0, 0};
    } else {
#pragma unroll
      for (int s = 0; s < 4; s++) buf[gi][s] = (rok && lc + s < le) ? xr[lc + s] : 0.0f;
    }
  }
}

__device__ __forceinline__ void mfma_chunk(const floatx4 (&buf)[CH], const float* __restrict__ bp,
                                           int l0, int le, int lane, floatx16& acc) {
  const int h = lane >> 5, c = lane & 31;
#pragma unroll
  for (int gi = 0; gi < CH; gi++) {
    const int lc = l0 + 8 * gi + 4 * h;
    if (l0 + 8 * gi < le) {
#pragma unroll
      for (int s = 0; s < 4; s++) {
        const float b = bp[(lc + s) * TP + c];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(buf[gi][s], b, acc, 0, 0, 0);
      }
    }
  }
}

// The tile product for every row of this group into xt (Bterm added).
template <bool VEC>
__device__ void tile_product(const HalsArgs& a, const Smem& sm, int64_t row0, int64_t row1, int nr,
                             int a0, int tw) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int K = a.K;
  const int nrb = (nr + 31) / 32;
  const int parts = nrb >= 4 ? 1 : (nrb == 2 ? 2 : (nrb == 1 ? 4 : 1));
  const int chunk = ((K + parts - 1) / parts + 63) / 64 * 64;
  const int h = lane >> 5;
  const float* __restrict__ X = a.X;
  for (int job = w; job < nrb * parts; job += 4) {
    const int rb = job / parts, p = job % parts;
    const int lb = p * chunk;
    const int le = lb + chunk < K ? lb + chunk : K;
    const int64_t r = row0 + rb * 32 + (lane & 31);
    const bool rok = r < row1;
    const float* xr = X + (rok ? r : row0) * K;
    floatx16 acc;
#pragma unroll
    for (int e = 0; e < 16; e++) acc[e] = 0.0f;
    floatx4 b0[CH], b1[CH];
    if (lb < le) load_chunk<VEC>(b0, xr, rok, lb, le, K, h);
    for (int l0 = lb; l0 < le; l0 += 2 * 8 * CH) {
      const int l1 = l0 + 8 * CH;
      if (l1 < le) load_chunk<VEC>(b1, xr, rok, l1, le, K, h);
      mfma_chunk(b0, sm.bp, l0, le, lane, acc);
      const int l2 = l1 + 8 * CH;
      if (l2 < le) load_chunk<VEC>(b0, xr, rok, l2, le, K, h);
      if (l1 < le) mfma_chunk(b1, sm.bp, l1, le, lane, acc);
    }
    // lane holds y[rb*32 + 8 j + 4 h + i][lane%32]
    if (parts == 1) {
#pragma unroll
      for (int j = 0; j < 4; j++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int rl = rb * 32 + 8 * j + 4 * h + i;
          const int cl = lane & 31;
          if (rl < nr && cl < tw) sm.xt[rl * TP + cl] = acc[4 * j + i] + a.Bterm[(row0 + rl) * K + a0 + cl];
        }
    } else {
#pragma unroll
      for (int j = 0; j < 4; j++)
#pragma unroll
        for (int i = 0; i < 4; i++) sm.part[(w * 32 + 8 * j + 4 * h + i) * TP + (lane & 31)] = acc[4 * j + i];
    }
  }
  if (parts > 1) {
    __syncthreads();
    for (int i = tid; i < nr * tw; i += 256) {
      const int rl = i / tw, cl = i % tw;
      const int rb = rl / 32;
      float v = a.Bterm[(row0 + rl) * K + a0 + cl];
      for (int p = 0; p < parts; p++) v += sm.part[((rb * parts + p) * 32 + rl % 32) * TP + cl];
      sm.xt[rl * TP + cl] = v;
    }
  }
}

template <bool NORM, bool VEC>
__global__ __launch_bounds__(256) void hals_kernel(HalsArgs a) {
  extern __shared__ float smem_raw[];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int K = a.K;
  const int g = blockIdx.x, groups = gridDim.x;
  const int64_t row0 = (int64_t)g * a.rows_per_group;
  int64_t row1 = row0 + a.rows_per_group;
  if (row1 > a.rows) row1 = a.rows;
  const int nr = row0 < row1 ? (int)(row1 - row0) : 0;
  const Smem sm = carve(smem_raw, a.rows_per_group, K);
  float* __restrict__ X = a.X;
  const float eps = a.eps;

  for (int a0 = 0; a0 < K; a0 += T) {
    const int b0 = a0 + T < K ? a0 + T : K;
    const int tw = b0 - a0;
    for (int i = tid; i < T * T; i += 256) {
      const int r = i / T, c = i % T;
      sm.gt[r * TP + c] = (r < tw && c < tw) ? a.G[(int64_t)(a0 + r) * K + a0 + c] : 0.0f;
    }
    for (int i = tid; i < kpad(K) * T; i += 256) {
      const int l = i / T, c = i % T;
      sm.bp[l * TP + c] = bm_value(a.G, K, l, a0 + c, a0, b0, a.diag_one);
    }
    __syncthreads();
    tile_product<VEC>(a, sm, row0, row1, nr, a0, tw);
    __syncthreads();

    if constexpr (!NORM) {
      // eight threads per row, each owning four of the tile's columns
      const int rl = tid >> 3, j = tid & 7;
      const bool rok = rl < nr;
      float y[4];
#pragma unroll
      for (int e = 0; e < 4; e++) y[e] = rok ? sm.xt[rl * TP + 4 * j + e] : 0.0f;
#pragma unroll
      for (int t = 0; t < T; t++) {
        if (t < tw) {
          const int jt = t >> 2, et = t & 3;
          float x = 0.0f;
          if (j == jt) {
            x = fmaxf(eps, y[et]);
            y[et] = x;
          }
          x = __shfl(x, (lane & ~7) | jt);
#pragma unroll
          for (int e = 0; e < 4; e++)
            if (4 * j + e > t) y[e] -= x * sm.gt[t * TP + 4 * j + e];
        }
      }
      if (rok) {
#pragma unroll
        for (int e = 0; e < 4; e++) sm.xt[rl * TP + 4 * j + e] = y[e];
      }
    } else {
      constexpr int RPT = (kMaxRowsW + 255) / 256;  // rows per thread
      // invariant at step t: xt[r][t] = u_t (clipped, not normalised), ss = my
      // partial of sum u_t^2; columns > t lack only the pending x_{t-1} term
      float ss = 0.0f;
#pragma unroll
      for (int q = 0; q < RPT; q++) {
        const int rl = tid + 256 * q;
        if (rl < nr) {
          const float u = fmaxf(eps, sm.xt[rl * TP]);
          sm.xt[rl * TP] = u;
          ss += u * u;
        }
      }
      float xprev[RPT];
#pragma unroll
      for (int q = 0; q < RPT; q++) xprev[q] = 0.0f;
      for (int t = 0; t < tw; t++) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
        if (lane == 0) sm.red[w] = ss;
        __syncthreads();
        const unsigned tag = (a.epoch << 10) | (unsigned)(a0 + t);
        const int par = (a0 + t) & 1;
        if (tid < kSlotReplicas)
          publish(a.slots, groups, g, tag, par, sm.red[0] + sm.red[1] + sm.red[2] + sm.red[3], tid);
        // off the critical path: the previous column's contribution to columns > t
        if (t > 0) {
#pragma unroll
          for (int q = 0; q < RPT; q++) {
            const int rl = tid + 256 * q;
            if (rl < nr)
              for (int c = t + 1; c < tw; c++) sm.xt[rl * TP + c] -= xprev[q] * sm.gt[(t - 1) * TP + c];
          }
        }
        if (w == 0) {
          const float tot = collect_sum(a.slots, groups, g, tag, par, a.status);
          if (lane == 0) sm.red[4] = tot;
        }
        __syncthreads();
        const float nrm = sqrtf(sm.red[4]);
        ss = 0.0f;
#pragma unroll
        for (int q = 0; q < RPT; q++) {
          const int rl = tid + 256 * q;
          if (rl < nr) {
            const float x = sm.xt[rl * TP + t] / nrm;
            sm.xt[rl * TP + t] = x;
            xprev[q] = x;
            if (t + 1 < tw) {
              const float u = fmaxf(eps, sm.xt[rl * TP + t + 1] - x * sm.gt[t * TP + t + 1]);
              sm.xt[rl * TP + t + 1] = u;
              ss += u * u;
            }
          }
        }
      }
    }
    __syncthreads();
    // write the finished tile back (rows are K-contiguous)
    for (int i = tid; i < nr * tw; i += 256) {
      const int rl = i / tw, cl = i % tw;
      X[(row0 + rl) * K + a0 + cl] = sm.xt[rl * TP + cl];
    }
    __syncthreads();
  }
}

template <bool NORM, bool VEC>
const void* kernel_ptr() {
  return (const void*)hals_kernel<NORM, VEC>;
}

hipError_t allow_smem(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

int hals_rows_per_group_h() { return kRowsH; }

size_t hals_smem_bytes(int rows_per_group, int K) { return smem_floats(rows_per_group, K) * 4; }

int hals_w_groups(int64_t rows, int K, int device_cus) {
  (void)K;
  int g = device_cus;  // one persistent group per compute unit
  const int64_t min_groups = (rows + kMaxRowsW - 1) / kMaxRowsW;
  const int64_t max_useful = (rows + 31) / 32;
  if (g > max_useful) g = (int)max_useful;
  if (g < min_groups) g = (int)min_groups;  // caller checks co-residency
  if (g < 1) g = 1;
  return g;
}

int hals_w_max_rows() { return kMaxRowsW; }

// Largest cooperative grid of the W kernel for this slab height and K.
int hals_w_max_coresident(int device_cus, int rows_per_group, int K) {
  const size_t bytes = hals_smem_bytes(rows_per_group, K);
  const void* fn = kernel_ptr<true, true>();
  if (allow_smem(fn, bytes) != hipSuccess) return 0;
  if (allow_smem(kernel_ptr<true, false>(), bytes) != hipSuccess) return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, hals_kernel<true, true>, 256, bytes) !=
      hipSuccess)
    return 0;
  return nb * device_cus;
}

hipError_t hals_update(const HalsArgs& a, bool norm, int groups, hipStream_t s) {
  const bool vec = (a.K % 4 == 0) && (((uintptr_t)a.X & 15) == 0);
  if (!norm) {
    HalsArgs b = a;
    b.rows_per_group = kRowsH;
    const unsigned grid = (unsigned)((a.rows + kRowsH - 1) / kRowsH);
    if (grid == 0) return hipSuccess;
    const size_t bytes = hals_smem_bytes(kRowsH, a.K);
    const void* fn = vec ? kernel_ptr<false, true>() : kernel_ptr<false, false>();
    hipError_t e = allow_smem(fn, bytes);
    if (e != hipSuccess) return e;
    if (vec) hals_kernel<false, true><<<grid, 256, bytes, s>>>(b);
    else hals_kernel<false, false><<<grid, 256, bytes, s>>>(b);
    return hipGetLastError();
  }
  HalsArgs b = a;
  void* args[] = {&b};
  const size_t bytes = hals_smem_bytes(a.rows_per_group, a.K);
  const void* fn = vec ? kernel_ptr<true, true>() : kernel_ptr<true, false>();
  hipError_t e = allow_smem(fn, bytes);
  if (e != hipSuccess) return e;
  return hipLaunchCooperativeKernel(fn, dim3(groups), dim3(256), args, (unsigned)bytes, s);
}

}  // namespace plnmf
