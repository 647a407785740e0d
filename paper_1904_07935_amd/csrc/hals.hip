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
// diagonal.  This is done in place, so one product per tile replaces both
// GEMM phases.  What remains is phase 2 (Eq. 5 with +P, as in Alg. 2): within
// the tile, column by column, clip, normalise (W), and apply the new value to
// the tile's later columns, on the tile held in LDS.
//
// The W half needs the L2 norm of each finished column over all rows before
// the next column can be clipped (Alg. 1 normalises inside the k loop), so the
// W kernel is persistent: its workgroups are co-resident (cooperative launch)
// and exchange one FP32 partial per column through tagged 64-bit slots.  Every
// workgroup sums all partials in the same fixed order, so every workgroup (and
// every run) gets the bitwise-identical norm; the paper's atomicAdd of partial
// sums (Alg. 4) would be order-dependent.  Waits are bounded: on a timeout a
// status bit is set and the kernel still runs to completion.
#include "internal.hpp"

namespace plnmf {
namespace {

constexpr int T = kTile;
constexpr int TP = T + 1;  // LDS row pitch (bank spread)

template <int MAXR>
struct HalsSmem {
  float xt[MAXR][TP];       // the tile's columns for this group's rows
  float gt[T][TP];          // G restricted to the tile
  float part[4][32][TP];    // contraction-split partial products
  float red[8];
};

__device__ __forceinline__ unsigned long long pack_slot(unsigned tag, float v) {
  return ((unsigned long long)tag << 32) | (unsigned long long)__float_as_uint(v);
}

// Chip-wide fixed-order sum of one float per workgroup (wave 0 only).
__device__ float exchange_sum(unsigned long long* slots, int groups, int g, unsigned tag,
                              int par, float mine, int32_t* status) {
  const int lane = threadIdx.x & 63;
  unsigned long long* base = slots + (int64_t)par * groups;
  if (lane == 0)
    __hip_atomic_store(base + g, pack_slot(tag, mine), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// B operand of the tile product: row lrow of the contraction, column c.
__device__ __forceinline__ float bm_value(const float* __restrict__ G, int K, int lrow, int c,
                                          int a0, int b0, int diag_one) {
  if (lrow >= K || c >= b0) return 0.0f;
  const float gv = G[(int64_t)lrow * K + c];
  if (lrow == c) return diag_one ? 1.0f - gv : 0.0f;
  if (lrow >= a0 && lrow < b0 && lrow < c) return 0.0f;  // new in-tile value: phase 2
  return -gv;
}

template <bool NORM, bool VEC, int MAXR>
__global__ __launch_bounds__(256) void hals_kernel(HalsArgs a) {
  __shared__ HalsSmem<MAXR> sm;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int K = a.K;
  const int g = blockIdx.x, groups = gridDim.x;
  const int64_t row0 = (int64_t)g * a.rows_per_group;
  int64_t row1 = row0 + a.rows_per_group;
  if (row1 > a.rows) row1 = a.rows;
  const int nr = row0 < row1 ? (int)(row1 - row0) : 0;
  const int nrb = (nr + 31) / 32;
  const int parts = nrb >= 4 ? 1 : (nrb == 2 ? 2 : (nrb == 1 ? 4 : 1));
  float* __restrict__ X = a.X;

  for (int a0 = 0; a0 < K; a0 += T) {
    const int b0 = a0 + T < K ? a0 + T : K;
    const int tw = b0 - a0;
    for (int i = tid; i < T * T; i += 256) {
      const int r = i / T, c = i % T;
      sm.gt[r][c] = (r < tw && c < tw) ? a.G[(int64_t)(a0 + r) * K + a0 + c] : 0.0f;
    }
    // ---- tile product: every contribution not involving the tile's new values
    {
      const int c = a0 + (lane & 31);
      const int h = lane >> 5;
      const int chunk = ((K + parts - 1) / parts + 7) / 8 * 8;
      for (int job = w; job < nrb * parts; job += 4) {
        const int rb = job / parts, p = job % parts;
        const int lb = p * chunk;
        const int le = lb + chunk < K ? lb + chunk : K;
        const int64_t r = row0 + rb * 32 + (lane & 31);
        const bool rok = r < row1;
        const float* xr = X + r * K;
        floatx16 acc;
#pragma unroll
        for (int e = 0; e < 16; e++) acc[e] = 0.0f;
        for (int l0 = lb; l0 < le; l0 += 8) {
          const int lc = l0 + 4 * h;
          floatx4 av;
          if constexpr (VEC) {
            av = (rok && lc < K) ? *(const floatx4*)(xr + lc) : floatx4{0, 0, 0, 0};
          } else {
#pragma unroll
            for (int s = 0; s < 4; s++) av[s] = (rok && lc + s < K) ? xr[lc + s] : 0.0f;
          }
          float bv[4];
#pragma unroll
          for (int s = 0; s < 4; s++) bv[s] = bm_value(a.G, K, lc + s, c, a0, b0, a.diag_one);
#pragma unroll
          for (int s = 0; s < 4; s++)
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s], bv[s], acc, 0, 0, 0);
        }
        // lane holds y[rb*32 + 8 j + 4 h + i][lane%32]
        if (parts == 1) {
#pragma unroll
          for (int j = 0; j < 4; j++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
              const int rl = rb * 32 + 8 * j + 4 * h + i;
              const int cl = lane & 31;
              if (rl < nr && cl < tw)
                sm.xt[rl][cl] = acc[4 * j + i] + a.Bterm[(row0 + rl) * K + a0 + cl];
            }
        } else {
#pragma unroll
          for (int j = 0; j < 4; j++)
#pragma unroll
            for (int i = 0; i < 4; i++) sm.part[w][8 * j + 4 * h + i][lane & 31] = acc[4 * j + i];
        }
      }
      if (parts > 1) {
        __syncthreads();
        for (int i = tid; i < nr * tw; i += 256) {
          const int rl = i / tw, cl = i % tw;
          const int rb = rl / 32;
          float v = a.Bterm[(row0 + rl) * K + a0 + cl];
          for (int p = 0; p < parts; p++) v += sm.part[rb * parts + p][rl % 32][cl];
          sm.xt[rl][cl] = v;
        }
      }
      __syncthreads();
    }
    // ---- phase 2: in-tile recurrence
    if constexpr (!NORM) {
      for (int rl = tid; rl < nr; rl += 256) {
        float y[T];
#pragma unroll
        for (int t = 0; t < T; t++) y[t] = sm.xt[rl][t];
#pragma unroll
        for (int t = 0; t < T; t++) {
          if (t < tw) {
            const float x = fmaxf(a.eps, y[t]);
            y[t] = x;
#pragma unroll
            for (int cc = t + 1; cc < T; cc++) y[cc] -= x * sm.gt[t][cc];
          }
        }
#pragma unroll
        for (int t = 0; t < T; t++) sm.xt[rl][t] = y[t];
      }
    } else {
      constexpr int RPT = (MAXR + 255) / 256;  // rows per thread
      float y[RPT][T];
#pragma unroll
      for (int q = 0; q < RPT; q++) {
        const int rl = tid + 256 * q;
#pragma unroll
        for (int t = 0; t < T; t++) y[q][t] = rl < nr ? sm.xt[rl][t] : 0.0f;
      }
#pragma unroll
      for (int t = 0; t < T; t++) {
        if (t < tw) {
          float ss = 0.0f;
#pragma unroll
          for (int q = 0; q < RPT; q++) {
            const int rl = tid + 256 * q;
            if (rl < nr) {
              const float u = fmaxf(a.eps, y[q][t]);
              y[q][t] = u;
              ss += u * u;
            }
          }
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
          if (lane == 0) sm.red[w] = ss;
          __syncthreads();
          if (w == 0) {
            const float mine = sm.red[0] + sm.red[1] + sm.red[2] + sm.red[3];
            const unsigned tag = (a.epoch << 10) | (unsigned)(a0 + t);
            const float tot = exchange_sum(a.slots, groups, g, tag, (a0 + t) & 1, mine, a.status);
            if (lane == 0) sm.red[4] = tot;
          }
          __syncthreads();
          const float nrm = sqrtf(sm.red[4]);
#pragma unroll
          for (int q = 0; q < RPT; q++) {
            const float x = y[q][t] / nrm;
            y[q][t] = x;
#pragma unroll
            for (int cc = t + 1; cc < T; cc++) y[q][cc] -= x * sm.gt[t][cc];
          }
        }
      }
#pragma unroll
      for (int q = 0; q < RPT; q++) {
        const int rl = tid + 256 * q;
        if (rl < nr) {
#pragma unroll
          for (int t = 0; t < T; t++) sm.xt[rl][t] = y[q][t];
        }
      }
    }
    __syncthreads();
    // ---- write the finished tile back (rows are K-contiguous)
    for (int i = tid; i < nr * tw; i += 256) {
      const int rl = i / tw, cl = i % tw;
      X[(row0 + rl) * K + a0 + cl] = sm.xt[rl][cl];
    }
    __syncthreads();
  }
}

constexpr int kMaxRowsW = 512;
constexpr int kRowsH = 32;

}  // namespace

int hals_rows_per_group_h() { return kRowsH; }

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

hipError_t hals_update(const HalsArgs& a, bool norm, int groups, hipStream_t s) {
  const bool vec = (a.K % 4 == 0) && (((uintptr_t)a.X & 15) == 0);
  if (!norm) {
    HalsArgs b = a;
    b.rows_per_group = kRowsH;
    const unsigned grid = (unsigned)((a.rows + kRowsH - 1) / kRowsH);
    if (grid == 0) return hipSuccess;
    if (vec) hals_kernel<false, true, kRowsH><<<grid, 256, 0, s>>>(b);
    else hals_kernel<false, false, kRowsH><<<grid, 256, 0, s>>>(b);
    return hipGetLastError();
  }
  HalsArgs b = a;
  void* args[] = {&b};
  const void* fn = vec ? (const void*)hals_kernel<true, true, kMaxRowsW>
                       : (const void*)hals_kernel<true, false, kMaxRowsW>;
  return hipLaunchCooperativeKernel(fn, dim3(groups), dim3(256), args, 0, s);
}

// Largest cooperative grid of the W kernel on this device.
int hals_w_max_coresident(int device_cus) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, hals_kernel<true, true, kMaxRowsW>, 256, 0) !=
      hipSuccess)
    return 0;
  return nb * device_cus;
}

}  // namespace plnmf
