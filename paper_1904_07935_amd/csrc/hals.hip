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
// in) is staged once per tile in LDS; the A operand (rows of X) streams from
// global memory in double-buffered register chunks.  What remains is phase 2
// (Eq. 5 with +P, as in Alg. 2): within the tile, column by column, clip,
// normalise (W), and apply the new value to the tile's later columns.
//
// H half: rows are independent, so each workgroup runs the whole sweep over a
// slab of 32 rows (product and phase 2 per tile, in LDS).
//
// W half: each column needs the L2 norm of the finished column over all rows
// before the next column can be clipped (Alg. 1 normalises inside the k
// loop), so phase 2 is a chain of K chip-level reductions and their latency,
// not arithmetic, bounds the kernel.  One launch of one 512-thread workgroup
// per CU (all resident at once) splits the work by role:
//   * column groups (as many as one XCD holds, at most 1792 rows each) hold
//     the tile's 32 columns of their rows in registers and run phase 2,
//     exchanging one FP32 partial per group and column through tagged 64-bit
//     slots.  They are the workgroups whose index is a multiple of 8 (then
//     8i+1, ...): the dispatcher places workgroup b on XCD b % 8, so up to 32
//     column groups share one XCD and its L2, where the exchange round trip is
//     shortest.  Placement only affects speed.
//   * product groups (all others) compute the tile product of every row into
//     a [rows, 32] hand-off buffer once the column groups have published the
//     previous tile (the product reads those new columns).
// Every column group sums all partials in the same fixed order, so all of them
// (and every run) get the bitwise-identical norm; the paper's atomicAdd of
// partial sums (Alg. 4) would be order-dependent.  Hand-offs between roles are
// tagged flags over device-scope (XCD-coherent) loads and stores.  All waits are
// bounded: on a timeout a status bit is set, every group stops waiting, and
// the kernel still runs to completion.
#include <cstdlib>

#include "internal.hpp"

namespace plnmf {
namespace {

constexpr int T = kTile;
constexpr int TP = T + 1;  // LDS row pitch (bank spread)
constexpr int kRowsH = 32;

// --------------------------------------------------------- shared pieces ----

__host__ __device__ inline int kpad(int K) { return (K + 7) / 8 * 8; }

__device__ __forceinline__ unsigned long long pack_slot(unsigned tag, float v) {
  return ((unsigned long long)tag << 32) | (unsigned long long)__float_as_uint(v);
}

// Device-scope exchange (column groups on several XCDs).  The slot array can
// be replicated kSlotReplicas times (kSlotStride apart; one copy at present):
// every group writes its partial into all replicas and polls only replica
// g % kSlotReplicas.  Called by lanes 0..kSlotReplicas-1 of one wave.
__device__ __forceinline__ void publish(unsigned long long* slots, int groups, int g, unsigned tag,
                                        int par, float mine, int replica) {
  __hip_atomic_store(slots + (int64_t)replica * kSlotStride + (int64_t)par * groups + g,
                     pack_slot(tag, mine), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool timed_out(const int32_t* status) {
  return (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 256) != 0;
}


// Sum over all 64 lanes, the same in every lane, in a fixed order: DPP steps
// within each row of 16 lanes (lane pairs, quads, halves), then the four row
// sums in row order.  VALU data movement only (no LDS round trips).
__device__ __forceinline__ float wave_sum(float v) {
  v += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x140, 0xF, 0xF, false));
  const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
  const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
  const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
  const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
  return ((r0 + r1) + r2) + r3;
}

// The same as collect_sum for at most 128 groups (slots lane and lane + 64
// per lane), with each lane's pair added in slot order and the lanes summed by
// wave_sum: a fixed order, the same in every group.
__device__ __forceinline__ float collect_sum64(const unsigned long long* slots, int groups, int g,
                                               unsigned tag, int par, int32_t* status) {
  const int lane = threadIdx.x & 63;
  const unsigned long long* p =
      slots + (int64_t)(g % kSlotReplicas) * kSlotStride + (int64_t)par * groups + lane;
  const bool act0 = lane < groups, act1 = lane + 64 < groups;
  unsigned long long v0 = (unsigned long long)tag << 32;  // inactive slots: ready, zero
  unsigned long long v1 = v0;
  int spins = 0;
  bool done;
  do {
    if (act0) v0 = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (act1) v1 = __hip_atomic_load(p + 64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    done = __all((unsigned)(v0 >> 32) == tag && (unsigned)(v1 >> 32) == tag);
    if (!done && (++spins & 255) == 0 && timed_out(status)) break;
  } while (!done && spins < kSpinLimit);
  if (!done && lane == 0) atomicOr(status, 256);
  return wave_sum(__uint_as_float((unsigned)v0) + __uint_as_float((unsigned)v1));
}

// Bounded wait of one wave until flags[i * stride], i < n, all hold `tag`.
__device__ void wait_flags(const unsigned* flags, int n, int stride, unsigned tag, int32_t* status) {
  const int lane = threadIdx.x & 63;
  int spins = 0;
  bool done;
  do {
    done = true;
    for (int i = lane; i < n; i += 64)
      done = done && (__hip_atomic_load(flags + (int64_t)i * stride, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT) == tag);
    if (!done && (++spins & 255) == 0 && timed_out(status)) break;
  } while (!done && spins < kSpinLimit);
  if (!done) atomicOr(status, 256);
}

// Hand-off data between workgroups of the W kernel: every tile has its own
// region of the hand-off buffers, so each of their cache lines is written once
// per launch, by device-scope stores (the sc1 cache policy, written through
// past the XCD's own L2), and read only after the producer's flag.  No XCD can
// hold a stale copy of such a line (caches are invalidated at kernel start and
// nobody reads the line earlier), so the readers use plain cached loads and no
// L2 write-back or invalidation is needed.  The producer waits until its
// stores are complete before it raises the flag.
constexpr int kThrough = 16;  // buffer cache-policy bit sc1 (device scope)

typedef unsigned uintx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t store_view(void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ void st_through4(__amdgpu_buffer_rsrc_t r, uint32_t byte_off, floatx4 v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uintx4, v), r, byte_off, 0, kThrough);
}
__device__ __forceinline__ void st_through(__amdgpu_buffer_rsrc_t r, uint32_t byte_off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, byte_off, 0, kThrough);
}

// Every thread: wait for its stores to complete; then one thread raises the flag.
__device__ __forceinline__ void signal_flag(unsigned* flag, unsigned tag) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave 0 waits for the flags; the barrier keeps every later load after it.
__device__ __forceinline__ void await_flags(const unsigned* flags, int n, int stride, unsigned tag,
                                            int32_t* status) {
  if ((threadIdx.x >> 6) == 0) wait_flags(flags, n, stride, tag, status);
  __syncthreads();
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
                                           int l0, int le, int h) {
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

// One wave: the 32 x 32 product of rows xr (this lane's row, lane % 32) over
// contraction [lb, le) with the LDS panel bp.  Lane holds result row
// 8 j + 4 (lane / 32) + i, column lane % 32, in acc[4 j + i].
template <bool VEC>
__device__ __forceinline__ floatx16 block_product(const float* __restrict__ xr, bool rok, int lb,
                                                  int le, const float* __restrict__ bp, int lane) {
  const int h = lane >> 5;
  floatx16 acc;
#pragma unroll
  for (int e = 0; e < 16; e++) acc[e] = 0.0f;
  floatx4 b0[CH], b1[CH];
  if (lb < le) load_chunk<VEC>(b0, xr, rok, lb, le, h);
  for (int l0 = lb; l0 < le; l0 += 2 * 8 * CH) {
    const int l1 = l0 + 8 * CH;
    if (l1 < le) load_chunk<VEC>(b1, xr, rok, l1, le, h);
    mfma_chunk(b0, bp, l0, le, lane, acc);
    const int l2 = l1 + 8 * CH;
    if (l2 < le) load_chunk<VEC>(b0, xr, rok, l2, le, h);
    if (l1 < le) mfma_chunk(b1, bp, l1, le, lane, acc);
  }
  return acc;
}

// ---------------------------------------------------------------- H half ----

// One workgroup per 32 rows, the whole sweep of Alg. 1's H loop for them.  The
// rows live in LDS from start to end (updated in place); per tile: the tile
// product on the matrix cores with the contraction split over the four waves,
// Bterm added, then phase 2 by wave 0 (one lane per row, the tile's columns in
// registers) while waves 1..3 stage the next tile's panel.
// LDS (floats): xs [32][XP] | bp [kpad(K)][TP] | gt [2][T][GP] | part [3][32][TP],
// XP = 32 * ntiles + 1 (odd: conflict-free row and column access); GP = T + 4
// keeps every G row 16-byte aligned (phase 2 reads G rows, the same address in
// every lane, as 16-byte vectors).
__host__ __device__ inline int h_xp(int K) { return 32 * ((K + T - 1) / T) + 1; }
constexpr int GP = T + 4;
__host__ __device__ inline size_t h_smem_floats(int K) {
  return (size_t)kRowsH * h_xp(K) + (size_t)kpad(K) * TP + 2 * T * GP + 3 * 32 * TP;
}

__device__ __forceinline__ void copy_panel(const float* __restrict__ panel, const float* __restrict__ gblk,
                                           int K, int j, float* bp, float* gt, int t0, int nt) {
  const int kp = kpad(K);
  const floatx4* src = (const floatx4*)(panel + (int64_t)j * kp * T);
  for (int i = t0; i < kp * T / 4; i += nt) {
    const floatx4 v = src[i];
    float* d = bp + (4 * i / T) * TP + (4 * i) % T;
    d[0] = v[0];
    d[1] = v[1];
    d[2] = v[2];
    d[3] = v[3];
  }
  const floatx4* gs = (const floatx4*)(gblk + (int64_t)j * T * T);
  for (int i = t0; i < T * T / 4; i += nt) *(floatx4*)(gt + (4 * i / T) * GP + (4 * i) % T) = gs[i];
}

template <bool VEC>
__global__ __launch_bounds__(256) void hals_h_kernel(HalsArgs a) {
  extern __shared__ float smem_raw[];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, h = lane >> 5, m = lane & 31;
  const int K = a.K, kp = kpad(K), XP = h_xp(K), ntiles = (K + T - 1) / T;
  const int64_t row0 = (int64_t)blockIdx.x * kRowsH;
  const int nr = a.rows - row0 < kRowsH ? (int)(a.rows - row0) : kRowsH;
  float* xs = smem_raw;
  float* bp = xs + kRowsH * XP;
  float* gtb = bp + kp * TP;
  float* part = gtb + 2 * T * GP;
  const float eps = a.eps;

  // the group's rows, zero-padded to 32 * ntiles columns
  const int nq = 8 * ntiles;
  for (int i = tid; i < kRowsH * nq; i += 256) {
    const int rl = i / nq, c = 4 * (i % nq);
    floatx4 v = floatx4{0, 0, 0, 0};
    if (rl < nr) {
      const float* src = a.X + (row0 + rl) * K + c;
      if constexpr (VEC) {
        if (c < K) v = *(const floatx4*)src;
      } else {
#pragma unroll
        for (int e = 0; e < 4; e++)
          if (c + e < K) v[e] = src[e];
      }
    }
    float* d = xs + rl * XP + c;
    d[0] = v[0];
    d[1] = v[1];
    d[2] = v[2];
    d[3] = v[3];
  }
  copy_panel(a.panel, a.gblk, K, 0, bp, gtb, tid, 256);
  __syncthreads();

  const int chunk = ((kp + 3) / 4 + 7) / 8 * 8;  // contraction per wave, a multiple of 8
  const int lb = w * chunk, le = lb + chunk < kp ? lb + chunk : kp;
  // wave 0: a tile's Bterm in the product's lane layout, loaded one tile ahead
  auto load_bt = [&](int jt, float (&b)[16]) {
    const int at = jt * T, twt = at + T < K ? T : K - at;
#pragma unroll
    for (int jj = 0; jj < 4; jj++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int rl = 8 * jj + 4 * h + i;
        b[4 * jj + i] = (rl < nr && m < twt) ? a.Bterm[(row0 + rl) * K + at + m] : 0.0f;
      }
  };
  float btn[16];
  if (w == 0) load_bt(0, btn);
  for (int j = 0; j < ntiles; j++) {
    const int a0 = j * T, tw = a0 + T < K ? T : K - a0;
    const float* gt = gtb + (j & 1) * T * GP;
    float bt[16];
#pragma unroll
    for (int e = 0; e < 16; e++) bt[e] = btn[e];
    if (w == 0 && j + 1 < ntiles) load_bt(j + 1, btn);
    // the tile product, contraction [lb, le) of this wave
    floatx16 acc;
#pragma unroll
    for (int e = 0; e < 16; e++) acc[e] = 0.0f;
    for (int l = lb; l < le; l += 8) {
#pragma unroll
      for (int s = 0; s < 4; s++) {
        const int ll = l + 2 * s + h;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[m * XP + ll], bp[ll * TP + m], acc, 0, 0, 0);
      }
    }
    if (w > 0) {
      float* pw = part + (w - 1) * 32 * TP;
#pragma unroll
      for (int jj = 0; jj < 4; jj++)
#pragma unroll
        for (int i = 0; i < 4; i++) pw[(8 * jj + 4 * h + i) * TP + m] = acc[4 * jj + i];
    }
    __syncthreads();
    if (w == 0) {
      // y = Bterm + product, into part[0] (each element read, then written, by one lane)
#pragma unroll
      for (int jj = 0; jj < 4; jj++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int e = (8 * jj + 4 * h + i) * TP + m;
          part[e] = bt[4 * jj + i] + ((acc[4 * jj + i] + part[e]) + part[32 * TP + e]) + part[64 * TP + e];
        }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      // phase 2: one lane per row, the tile's columns in registers
      if (lane < kRowsH) {
        float y[T];
#pragma unroll
        for (int c = 0; c < T; c++) y[c] = part[lane * TP + c];
        if (tw == T) {
          // a full tile: no branch per step (a branch around a step makes the
          // compiler copy all of y on both sides of it), and step t + 1's G row
          // loaded during step t; the compiler barrier keeps later rows' loads
          // from being hoisted further, which would exhaust the registers
          float gr[T];
#pragma unroll
          for (int q = 0; q < T / 4; q++) {
            const floatx4 v = *(const floatx4*)(gt + 4 * q);
#pragma unroll
            for (int e = 0; e < 4; e++) gr[4 * q + e] = v[e];
          }
#pragma unroll
          for (int t = 0; t < T; t++) {
            float gn[T];
#pragma unroll
            for (int q = (t + 2) / 4; q < T / 4; q++) {
              const floatx4 v = *(const floatx4*)(gt + (t + 1) * GP + 4 * q);
#pragma unroll
              for (int e = 0; e < 4; e++) gn[4 * q + e] = v[e];
            }
            asm volatile("" ::: "memory");
            const float x = fmaxf(eps, y[t]);
            y[t] = x;
#pragma unroll
            for (int c = t + 1; c < T; c++) y[c] -= x * gr[c];
#pragma unroll
            for (int c = t + 2; c < T; c++) gr[c] = gn[c];
          }
        } else {
#pragma unroll
          for (int t = 0; t < T; t++) {
            if (t < tw) {
              const float x = fmaxf(eps, y[t]);
              y[t] = x;
#pragma unroll
              for (int c = t + 1; c < T; c++) y[c] -= x * gt[t * GP + c];
            }
          }
        }
#pragma unroll
        for (int c = 0; c < T; c++)
          if (c < tw) xs[lane * XP + a0 + c] = y[c];
      }
    } else if (j + 1 < ntiles) {
      // waves 1..3: the next tile's panel (bp is free once every wave has its product)
      copy_panel(a.panel, a.gblk, K, j + 1, bp, gtb + ((j + 1) & 1) * T * GP, tid - 64, 192);
    }
    __syncthreads();
  }
  // the finished rows back to X
  for (int i = tid; i < kRowsH * nq; i += 256) {
    const int rl = i / nq, c = 4 * (i % nq);
    if (rl >= nr || c >= K) continue;
    const float* sp = xs + rl * XP + c;
    float* dst = a.X + (row0 + rl) * K + c;
    if constexpr (VEC) {
      *(floatx4*)dst = floatx4{sp[0], sp[1], sp[2], sp[3]};
    } else {
#pragma unroll
      for (int e = 0; e < 4; e++)
        if (c + e < K) dst[e] = sp[e];
    }
  }
}

hipError_t allow_smem(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Rows-in-registers variant for many rows (large D).  A workgroup is four
// waves, each owning 32 rows that stay in VGPRs for the whole sweep, laid out
// as the A operand of the 32x32x2 FP32 matrix-core product: lane (m, h) holds
// X[row m][32 t + 2 s + h] in xa[16 t + s].  Per tile every wave forms its
// rows' whole-contraction product itself, with the B operand (the tile's
// panel) read from LDS, where the workgroup stages it one tile ahead in the
// order the lanes read it (16-byte reads, no bank conflicts).  Phase 2 runs on
// all 64 lanes in the same layout: lane (m, h) keeps row m's tile columns of
// parity h, and at each column step the lane pair exchanges the clipped value
// with one cross-half lane swap (v_permlane32_swap), so every lane does half
// of the row's updates and the finished values already sit where xa wants
// them.  Compared with the LDS-resident kernel, which holds 32 rows and a
// panel per workgroup, four times as many rows share one panel and every
// SIMD runs its own wave's product and phase 2.
//
// The tile width TT (the paper's T) is a template parameter: 32 is the
// product's output width; 64 takes two 32-column products per tile; 16 uses
// half of each 32-column product (the other half multiplies zeros).
// LDS (floats): panel [2][NB][32 NT][32] | gh [2][TT][TT] | part [4][32][TT + 1],
// NB = max(1, TT / 32).
constexpr int kRowsRR = 32;    // rows per wave
constexpr int kWavesRR = 4;    // waves per workgroup
__host__ __device__ constexpr int rr_nb(int TT) { return TT >= 32 ? TT / 32 : 1; }
__host__ __device__ constexpr int rr_pp(int TT) { return TT + 1 > TP ? TT + 1 : TP; }  // part pitch
__host__ __device__ inline size_t rr_smem_floats(int NT, int TT) {
  return 2 * (size_t)rr_nb(TT) * NT * 1024 + 2 * (size_t)TT * TT + kWavesRR * 32 * rr_pp(TT);
}
constexpr size_t kRrLdsMax = 160 * 1024;

// Tile j's staging block, as the Gram writes it for this kernel: the panel in
// lane-read order -- float4 (((q NT + t) 4 + sq) 2 + h) 32 + m holds rows
// 32 t + 2 (4 sq + i) + h of column 32 q + m (zeros past K) -- then the G
// block split by column parity, gh[h][t][k] = G[t][2 k + h] for 2 k + h > t,
// else 0 (the columns a phase-2 step updates).  A contiguous copy into the
// LDS: loads are issued by rr_load (early), stores by rr_store.
__host__ __device__ inline size_t rr_stage_floats(int NT, int TT) {
  return (size_t)rr_nb(TT) * NT * 1024 + (size_t)TT * TT;
}
template <int NT, int TT>
struct RrStage {
  static constexpr int NP = rr_nb(TT) * NT;             // float4 of the panel per thread
  static constexpr int NG = (TT * TT / 4 + 255) / 256;  // float4 of the G block per thread
  floatx4 v[NP];
  floatx4 g[NG];
};

template <int NT, int TT>
__device__ __forceinline__ void rr_load(const float* __restrict__ panel, int j, int tid,
                                        RrStage<NT, TT>& st) {
  const floatx4* src = (const floatx4*)(panel + (int64_t)j * rr_stage_floats(NT, TT));
#pragma unroll
  for (int k = 0; k < RrStage<NT, TT>::NP; k++) st.v[k] = src[tid + 256 * k];
  const floatx4* gs = src + rr_nb(TT) * NT * 256;
#pragma unroll
  for (int k = 0; k < RrStage<NT, TT>::NG; k++) {
    const int idx = tid + 256 * k;
    st.g[k] = idx < TT * TT / 4 ? gs[idx] : floatx4{0, 0, 0, 0};
  }
}

template <int NT, int TT>
__device__ __forceinline__ void rr_store(const RrStage<NT, TT>& st, float* lp, float* gt, int tid) {
#pragma unroll
  for (int k = 0; k < RrStage<NT, TT>::NP; k++) ((floatx4*)lp)[tid + 256 * k] = st.v[k];
#pragma unroll
  for (int k = 0; k < RrStage<NT, TT>::NG; k++) {
    const int idx = tid + 256 * k;
    if (idx < TT * TT / 4) ((floatx4*)gt)[idx] = st.g[k];
  }
}

template <int NT, int TT, bool VEC>
__global__ __launch_bounds__(256) void hals_h_rows_kernel(HalsArgs a) {
  constexpr int NB = rr_nb(TT), HP = TT / 2, PP = rr_pp(TT);
  extern __shared__ float smem_raw[];
  // w is the same in every lane of a wave: taken as such, the wave's row
  // offsets and buffer views below stay scalar
  const int tid = threadIdx.x, lane = tid & 63, m = lane & 31, h = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int K = a.K, ntiles = (K + TT - 1) / TT;
  float* lpb = smem_raw;                           // [2][NB * NT * 1024]
  float* gtb = lpb + 2 * NB * NT * 1024;           // [2][TT * TT]
  float* part = gtb + 2 * TT * TT + w * 32 * PP;   // this wave's [32][TT + 1]
  const int64_t row0 = ((int64_t)blockIdx.x * kWavesRR + w) * kRowsRR;
  const int nr = a.rows - row0 < kRowsRR ? (int)(a.rows - row0) : kRowsRR;  // may be <= 0
  const float eps = a.eps;
  float* __restrict__ X = a.X;

  {
    RrStage<NT, TT> st;
    rr_load<NT, TT>(a.panel, 0, tid, st);
    rr_store<NT, TT>(st, lpb, gtb, tid);
  }
  // Buffer views of the wave's rows of X and of Bterm (nr rows of K floats):
  // a load past the view returns zero, so rows beyond the matrix need no test,
  // and the constant column offsets stay in the instructions.
  const int64_t wave_bytes = nr > 0 ? (int64_t)nr * K * 4 : 0;
  const __amdgpu_buffer_rsrc_t xv =
      __builtin_amdgcn_make_buffer_rsrc(X + (nr > 0 ? row0 * K : 0), 0, (int)wave_bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t bv = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(a.Bterm + (nr > 0 ? row0 * K : 0)), 0, (int)wave_bytes, 0x00020000);
  // the wave's rows straight into the A-operand layout, all loads in flight
  // at once: lane (m, h) reads X[row m][32 t + 2 s + h].  Columns past K
  // (only in the last 32) hold the next row's values or zero and are cleared
  // once every load is issued.
  float xa[16 * NT];
  {
    const uint32_t xo = (uint32_t)((m * K + h) * 4);
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
      for (int s2 = 0; s2 < 16; s2++)
        xa[16 * t + s2] = __uint_as_float(
            __builtin_amdgcn_raw_buffer_load_b32(xv, xo + (uint32_t)((32 * t + 2 * s2) * 4), 0, 0));
#pragma unroll
    for (int s2 = 0; s2 < 16; s2++)
      if (32 * (NT - 1) + 2 * s2 + h >= K) xa[16 * (NT - 1) + s2] = 0.0f;
  }
  // Bterm of a tile in the product's lane layout: lane (m, h) takes column
  // a0 + 32 q + m of rows 8 jj + 4 h + i; loaded one tile ahead, into the
  // registers the previous tile has just consumed, and not used until after
  // that tile's product.  Columns past the tile's width are masked where
  // the values are used.
  float bt[NB][16];
  auto load_bt = [&](int a0) {
#pragma unroll
    for (int q = 0; q < NB; q++)
#pragma unroll
      for (int jj = 0; jj < 4; jj++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int rl = 8 * jj + 4 * h + i, c = 32 * q + m;
          bt[q][4 * jj + i] = __uint_as_float(
              __builtin_amdgcn_raw_buffer_load_b32(bv, (uint32_t)((rl * K + a0 + c) * 4), 0, 0));
        }
  };
  load_bt(0);
  __syncthreads();  // tile 0's panel, staged above, is seen by every wave

#pragma unroll 1
  for (int j = 0; j < ntiles; j++) {
    const int a0 = j * TT, tw = a0 + TT < K ? TT : K - a0;
    const float* lp = lpb + (j & 1) * NB * NT * 1024;
    const float* gt = gtb + (j & 1) * TT * TT;
    // the next tile's staging: global loads now, LDS stores after the product
    RrStage<NT, TT> st;
    if (j + 1 < ntiles) rr_load<NT, TT>(a.panel, j + 1, tid, st);
    // the tile product over the whole contraction, B operand from LDS
    floatx16 acc[NB];
#pragma unroll
    for (int q = 0; q < NB; q++)
#pragma unroll
      for (int e = 0; e < 16; e++) acc[q][e] = 0.0f;
#pragma unroll
    for (int t = 0; t < NT; t++) {
#pragma unroll
      for (int sq = 0; sq < 4; sq++) {
#pragma unroll
        for (int q = 0; q < NB; q++) {
          const floatx4 b = *(const floatx4*)(lp + ((((q * NT + t) * 4 + sq) * 2 + h) * 32 + m) * 4);
#pragma unroll
          for (int i = 0; i < 4; i++)
            acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(xa[16 * t + 4 * sq + i], b[i], acc[q], 0, 0, 0);
        }
      }
    }
    if (j + 1 < ntiles)
      rr_store<NT, TT>(st, lpb + ((j + 1) & 1) * NB * NT * 1024, gtb + ((j + 1) & 1) * TT * TT, tid);
#pragma unroll
    for (int q = 0; q < NB; q++)
#pragma unroll
      for (int jj = 0; jj < 4; jj++)
#pragma unroll
        for (int i = 0; i < 4; i++)
          if (32 * q + m < TT)
            part[(8 * jj + 4 * h + i) * PP + 32 * q + m] =
                32 * q + m < tw ? acc[q][4 * jj + i] + bt[q][4 * jj + i] : 0.0f;
    if (j + 1 < ntiles) load_bt(a0 + TT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // phase 2 on all lanes: lane (m, h) holds row m's columns 2 k + h
    float yh[HP];
#pragma unroll
    for (int k = 0; k < HP; k++) yh[k] = part[m * PP + 2 * k + h];
    {
      const float* gp = gt + h * TT * HP;
      float gc[HP], gn[HP];
#pragma unroll
      for (int q = 0; q < HP / 4; q++) {
        const floatx4 v = *(const floatx4*)(gp + 4 * q);
#pragma unroll
        for (int e = 0; e < 4; e++) gc[4 * q + e] = v[e];
      }
#pragma unroll
      for (int t = 0; t < TT; t++) {
        const int u = t >> 1;
        if (t + 1 < TT) {  // step t + 1's G row, loaded during step t
#pragma unroll
          for (int q = ((t + 1) >> 1) >> 2; q < HP / 4; q++) {
            const floatx4 v = *(const floatx4*)(gp + (t + 1) * HP + 4 * q);
#pragma unroll
            for (int e = 0; e < 4; e++) gn[4 * q + e] = v[e];
          }
        }
        asm volatile("" ::: "memory");
        // column t lives in the lanes of parity t & 1: clip there, then one
        // swap gives both halves the clipped value
        const float cand = fmaxf(eps, yh[u]);
        const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(cand), __float_as_uint(cand),
                                                         false, false);
        const float x = __uint_as_float((t & 1) ? sw[1] : sw[0]);
        yh[u] = h == (t & 1) ? x : yh[u];
#pragma unroll
        for (int k = u; k < HP; k++) yh[k] -= x * gc[k];  // gc is 0 for columns <= t
#pragma unroll
        for (int k = (t + 1) >> 1; k < HP; k++) gc[k] = gn[k];
      }
    }
    if (tw < TT) {
#pragma unroll
      for (int k = 0; k < HP; k++)
        if (2 * k + h >= tw) yh[k] = 0.0f;
    }
    // the new tile values: into xa, and through part to the rows in global memory
#pragma unroll
    for (int t = 0; t < NT; t++) {
      if constexpr (TT >= 32) {
#pragma unroll
        for (int q = 0; q < NB; q++)
          if (t == NB * j + q) {  // uniform: one branch per 32 columns, no copy of xa
#pragma unroll
            for (int s2 = 0; s2 < 16; s2++) xa[16 * t + s2] = yh[16 * q + s2];
          }
      } else {
        if (2 * t == j) {
#pragma unroll
          for (int s2 = 0; s2 < 8; s2++) xa[16 * t + s2] = yh[s2];
        } else if (2 * t + 1 == j) {
#pragma unroll
          for (int s2 = 0; s2 < 8; s2++) xa[16 * t + 8 + s2] = yh[s2];
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int k = 0; k < HP; k++) part[m * PP + 2 * k + h] = yh[k];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    {
      const int rl = lane >> 1, c0 = HP * (lane & 1);  // row rl, columns c0 .. c0 + HP - 1
      if (rl < nr) {
        float* dst = X + (row0 + rl) * K + a0 + c0;
        const float* sp = part + rl * PP + c0;
        if (VEC && tw == TT) {
#pragma unroll
          for (int q = 0; q < HP / 4; q++)
            *(floatx4*)(dst + 4 * q) = floatx4{sp[4 * q], sp[4 * q + 1], sp[4 * q + 2], sp[4 * q + 3]};
        } else {
#pragma unroll
          for (int c = 0; c < HP; c++)
            if (c0 + c < tw) dst[c] = sp[c];
        }
      }
    }
    // every wave is done with this tile's panel and part; the next panel is staged
    __syncthreads();
  }
}

template <int NT, int TT>
hipError_t launch_h_rows(const HalsArgs& b, bool vec, hipStream_t s) {
  const unsigned grid = (unsigned)((b.rows + kWavesRR * kRowsRR - 1) / (kWavesRR * kRowsRR));
  const size_t bytes = rr_smem_floats(NT, TT) * 4;
  if (bytes > kRrLdsMax) return hipErrorInvalidValue;
  if constexpr (TT == 64 && NT > 6) {
    return hipErrorInvalidValue;  // the double-buffered 64-wide panel exceeds the LDS
  } else if constexpr (TT == 32) {
    const void* fn = vec ? (const void*)hals_h_rows_kernel<NT, TT, true>
                         : (const void*)hals_h_rows_kernel<NT, TT, false>;
    hipError_t e = allow_smem(fn, bytes);
    if (e != hipSuccess) return e;
    if (vec) hals_h_rows_kernel<NT, TT, true><<<grid, 256, bytes, s>>>(b);
    else hals_h_rows_kernel<NT, TT, false><<<grid, 256, bytes, s>>>(b);
  } else {
    if (!vec) return hipErrorInvalidValue;  // other widths: K % 4 == 0 only
    const void* fn = (const void*)hals_h_rows_kernel<NT, TT, true>;
    hipError_t e = allow_smem(fn, bytes);
    if (e != hipSuccess) return e;
    hals_h_rows_kernel<NT, TT, true><<<grid, 256, bytes, s>>>(b);
  }
  return hipGetLastError();
}

template <int TT>
hipError_t h_rows_tt(const HalsArgs& b, bool vec, hipStream_t s) {
  switch ((b.K + 31) / 32) {
    case 1: return launch_h_rows<1, TT>(b, vec, s);
    case 2: return launch_h_rows<2, TT>(b, vec, s);
    case 3: return launch_h_rows<3, TT>(b, vec, s);
    case 4: return launch_h_rows<4, TT>(b, vec, s);
    case 5: return launch_h_rows<5, TT>(b, vec, s);
    case 6: return launch_h_rows<6, TT>(b, vec, s);
    case 7: return launch_h_rows<7, TT>(b, vec, s);
    case 8: return launch_h_rows<8, TT>(b, vec, s);
    case 9: return launch_h_rows<9, TT>(b, vec, s);
    case 10: return launch_h_rows<10, TT>(b, vec, s);
    case 11: return launch_h_rows<11, TT>(b, vec, s);
    case 12: return launch_h_rows<12, TT>(b, vec, s);
    case 13: return launch_h_rows<13, TT>(b, vec, s);
    case 14: return launch_h_rows<14, TT>(b, vec, s);
    case 15: return launch_h_rows<15, TT>(b, vec, s);
    case 16: return launch_h_rows<16, TT>(b, vec, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t h_rows_dispatch(const HalsArgs& b, bool vec, hipStream_t s) {
  if (b.tile == 16) return h_rows_tt<16>(b, vec, s);
  if (b.tile == 64) return h_rows_tt<64>(b, vec, s);
  return h_rows_tt<32>(b, vec, s);
}

// ---------------------------------------------------------------- W half ----

constexpr int kWThreads = 512;
constexpr int kWWaves = kWThreads / 64;
constexpr int kWRowThreads = kWThreads - 64;        // wave 0 of a column group runs the exchange
constexpr int kWMaxRpt = 4;                         // rows per row thread of a column group
constexpr int kWMaxRows = kWRowThreads * kWMaxRpt;  // rows per column group
constexpr size_t kWSmemMin = 82 * 1024;             // > half the LDS: one group per CU
constexpr int kWMaxColGroups = 128;

// LDS (floats).  Column role: gt [T][TP] | wave sums [2][kWWaves] (in 2 kWWaves u64) |
// column totals [2] (in 2 u64) | protocol flag [2] (u64) | lane partials
// [2][kWWaves - 1][64].  Product role:
// bp [kpad(K)][TP] | per-wave stash [kWWaves][jobs per wave][32][TP] (partial
// products, then the transpose).
constexpr size_t kLdsMax = 160 * 1024;

__host__ __device__ inline size_t w_smem_bytes(int K, int jpw) {
  size_t b = ((size_t)kpad(K) * TP + (size_t)kWWaves * jpw * 32 * TP) * 4;
  const size_t col = (size_t)T * TP * 4 + (2 * kWWaves + 4) * 8 + 2 * (kWWaves - 1) * 64 * 4;
  if (b < col) b = col;
  return b < kWSmemMin ? kWSmemMin : b;
}

__device__ __forceinline__ unsigned tile_tag(unsigned epoch, int j) { return (epoch << 10) | (unsigned)j; }

// Rank of workgroup b when the grid is ordered XCD-major: b % 8 first, then b / 8.
__device__ __forceinline__ int xcd_major_rank(int b, int grid) {
  int key = b >> 3;
  for (int m = 0; m < (b & 7); m++) key += (grid - m + 7) >> 3;
  return key;
}

// Hand-off layout: tile j of Y (the product) and of Wn (the finished columns)
// is stored column-quad-major, float4 (j, v, r) = columns 4v..4v+3 of row r at
// float4 index (j * 8 + v) * rows + r, so that a wave's rows are contiguous.
__device__ __forceinline__ int64_t quad_index(int64_t rows, int j, int v, int64_t r) {
  return ((int64_t)j * (T / 4) + v) * rows + r;
}


// Column groups.  Waves 1..7 hold rows (RPT per thread) and run phase 2: per
// column, each posts its partial sum of u_t^2, applies the previous column to
// the rest of the tile while the exchange is in flight, and then needs the sum
// of all partials.  Within the group, workgroup barriers order the steps (the
// hardware barrier is cheaper than waves spinning on LDS flags).  Three
// exchange protocols, all summing in a fixed order (so every wave of every
// group gets the bitwise-identical norm):
//  * LOCAL (one column group): each row wave writes its wave sum to LDS; after
//    one barrier every row wave adds the seven in order.
//  * XCD and DEVICE: the row waves write their lane partials to LDS; after a
//    barrier wave 0 adds them (per lane in wave order, then across lanes),
//    exchanges one partial per group with the other groups and writes the
//    total to LDS, while the row waves apply the deferred update; a second
//    barrier hands the total to the row waves.  XCD, when all column groups run
//    on one XCD (checked at kernel start): non-temporal stores and loads,
//    served by that XCD's L2, which all its CUs share (about half the latency
//    of device-scope accesses, which go past the L2; measured), one partial per
//    group in two replica slots.  DEVICE (any placement): device-scope atomics.
// Slots hold tag and value in one 64-bit word, so a slot is either this
// column's value or not yet ready.
enum : int { kProtoLocal = 0, kProtoXcd = 1, kProtoDevice = 2 };
constexpr int kSlotDev = 0;      // [2][n_col] group partials (device scope)
constexpr int kSlotPlace = 256;  // [n_col] XCD of each column group (device scope)
constexpr int kSlotXcd = 512;    // [2 parities][2 replicas][64] group partials (XCD-local)
static_assert(kSlotXcd + 2 * 128 <= kSlotWords, "slot regions");
static_assert(kWMaxColGroups <= 128, "two slots per lane");
static_assert(kWMaxColGroups <= 256 - kSlotDev / 2, "slot regions");


// Sum of the n (<= 64) group partials of one column.  Each group publishes its
// partial in two replica slots (base + rank, base + 64 + rank); the poller
// keeps a non-temporal load of each replica in flight and checks them in turn,
// reissuing each as soon as it has been checked, which finds a late partial
// sooner than one load per L2 round trip (measured: W update 274 -> 246 us at
// 26000 x 200).  Lanes >= n re-read slot n - 1.  Summed across lanes in a
// fixed order.
__device__ __forceinline__ float collect_xcd(const unsigned long long* base, int n, unsigned tag,
                                             int32_t* status) {
  const int lane = threadIdx.x & 63;
  const int i = lane < n ? lane : n - 1;
  const unsigned long long* pa = base + i;
  const unsigned long long* pb = base + 64 + i;
  unsigned long long va = __builtin_nontemporal_load(pa);
  unsigned long long vb = __builtin_nontemporal_load(pb);
  unsigned long long v = 0;
  int spins = 0;
  bool done = false;
  while (true) {
    // the register constraint orders each check after the reload issued before it
    asm volatile("" : "+v"(va)::"memory");
    if (__all(lane >= n || (unsigned)(va >> 32) == tag)) {
      v = va;
      done = true;
      break;
    }
    va = __builtin_nontemporal_load(pa);
    asm volatile("" : "+v"(vb)::"memory");
    if (__all(lane >= n || (unsigned)(vb >> 32) == tag)) {
      v = vb;
      done = true;
      break;
    }
    vb = __builtin_nontemporal_load(pb);
    if ((++spins & 127) == 0 && timed_out(status)) break;
    if (spins >= kSpinLimit) break;
  }
  if (!done && lane == 0) atomicOr(status, 256);
  return wave_sum(lane < n ? __uint_as_float((unsigned)v) : 0.0f);
}

template <int RPT, bool VEC, int PROTO>
__device__ __forceinline__ void column_tiles(const HalsWArgs& a, int rank, int n_prod, float* lds) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const bool xwave = w == 0;
  const int K = a.K;
  const int64_t rows = a.rows;
  float* gt = lds;  // [T][TP] G of the tile
  unsigned long long* lpart = (unsigned long long*)(lds + T * TP);  // exchange words
  float* lsum = (float*)lpart;                                      // [2][kWWaves] (LOCAL)
  float* ltot = (float*)(lpart + 2 * kWWaves);                      // [2] (two-level)
  float* lvals = (float*)(lpart + 2 * kWWaves + 4);                 // [2][kWWaves - 1][64]
  const int64_t row0 = (int64_t)rank * a.rows_per_group;
  int64_t row1 = row0 + a.rows_per_group;
  if (row1 > rows) row1 = rows;
  const float eps = a.eps;
  const floatx4* __restrict__ Y4 = (const floatx4*)a.Y;
  const __amdgpu_buffer_rsrc_t wnview = store_view(a.Wn, (int64_t)((K + T - 1) / T) * rows * T * 4);
  bool valid[RPT];
  int64_t rr[RPT];
#pragma unroll
  for (int q = 0; q < RPT; q++) {
    rr[q] = row0 + (tid - 64) + kWRowThreads * q;
    valid[q] = !xwave && rr[q] < row1;
  }
  float y[RPT][T];

  for (int j = 0, a0 = 0; a0 < K; j++, a0 += T) {
    const int tw = a0 + T < K ? T : K - a0;
    __syncthreads();  // gt of the previous tile is no longer read
    {
      const floatx4* src =
          (const floatx4*)(a.panel + (int64_t)((K + T - 1) / T) * kpad(K) * T + (int64_t)j * T * T);
      for (int i = tid; i < T * T / 4; i += kWThreads) {
        const floatx4 v = src[i];
        float* d = gt + (4 * i / T) * TP + (4 * i) % T;
        d[0] = v[0];
        d[1] = v[1];
        d[2] = v[2];
        d[3] = v[3];
      }
    }
    // the product groups serving this column group: rank, rank + n_col, ...
    await_flags(a.flags + rank, (n_prod - rank + a.n_col - 1) / a.n_col, a.n_col,
                tile_tag(a.epoch, j), a.status);
    if (!xwave) {
      // this group's rows of the tile's product (one contiguous run of rows per wave)
#pragma unroll
      for (int q = 0; q < RPT; q++) {
#pragma unroll
        for (int v = 0; v < T / 4; v++) {
          const floatx4 f = valid[q] ? Y4[quad_index(rows, j, v, rr[q])] : floatx4{0, 0, 0, 0};
#pragma unroll
          for (int e = 0; e < 4; e++) y[q][4 * v + e] = f[e];
        }
      }
    }
    // invariant at step t: y[q][t] = u_t (clipped, not normalised) and ss = this
    // thread's part of sum u_t^2; columns > t lack only the pending x_{t-1} term
    float ss = 0.0f;
#pragma unroll
    for (int q = 0; q < RPT; q++) {
      const float u = fmaxf(eps, y[q][0]);
      y[q][0] = u;
      ss += valid[q] ? u * u : 0.0f;
    }
    float xprev[RPT];
#pragma unroll
    for (int q = 0; q < RPT; q++) xprev[q] = 0.0f;
#pragma unroll
    for (int t = 0; t < T; t++) {
      if (t < tw) {
        const unsigned ctag = (a.epoch << 10) | (unsigned)(a0 + t);
        const int par = (a0 + t) & 1;
        // off the critical path, while the exchange is in flight: the previous
        // column's contribution to columns > t
        auto deferred = [&]() {
          if (t > 0) {
#pragma unroll
            for (int c = t + 1; c < T; c++) {
              const float gv = gt[(t - 1) * TP + c];
#pragma unroll
              for (int q = 0; q < RPT; q++) y[q][c] -= xprev[q] * gv;
            }
            // finished here, before the wait: left to itself the compiler sinks
            // these products below the wait, onto the critical path
#pragma unroll
            for (int c = t + 1; c < T; c++)
#pragma unroll
              for (int q = 0; q < RPT; q++) asm volatile("" : "+v"(y[q][c]));
          }
        };
        float tot = 0.0f;
        {
          if (!xwave) {
            if constexpr (PROTO == kProtoLocal) {
              const float mine = wave_sum(ss);
              if (lane == 0) lsum[par * kWWaves + w] = mine;
            } else {
              lvals[(par * (kWWaves - 1) + (w - 1)) * 64 + lane] = ss;
            }
          }
          __syncthreads();
          if (xwave) {
            if constexpr (PROTO != kProtoLocal) {
              // the group's partial: per lane over the row waves in order, then across lanes
              float g = 0.0f;
#pragma unroll
              for (int i = 0; i < kWWaves - 1; i++) g += lvals[(par * (kWWaves - 1) + i) * 64 + lane];
              g = wave_sum(g);
              float tg;
              if constexpr (PROTO == kProtoXcd) {
                unsigned long long* sb = a.slots + kSlotXcd + par * 128;
                if (lane < 2) __builtin_nontemporal_store(pack_slot(ctag, g), sb + 64 * lane + rank);
                tg = collect_xcd(sb, a.n_col, ctag, a.status);
              } else {
                if (lane < kSlotReplicas) publish(a.slots + kSlotDev, a.n_col, rank, ctag, par, g, lane);
                tg = collect_sum64(a.slots + kSlotDev, a.n_col, rank, ctag, par, a.status);
              }
              if (lane == 0) ltot[par] = tg;
            }
          } else {
            deferred();
          }
          if constexpr (PROTO == kProtoLocal) {
            if (!xwave)
#pragma unroll
              for (int i = 1; i < kWWaves; i++) tot += lsum[par * kWWaves + i];
          } else {
            __syncthreads();
            if (!xwave) tot = ltot[par];
          }
        }
        if (!xwave) {
          const float gnext = t + 1 < T ? gt[t * TP + t + 1] : 0.0f;
          // hardware reciprocal square root (within about 1 ulp; every wave of
          // every group computes it from the identical total)
          const float rn = __builtin_amdgcn_rsqf(tot);
          ss = 0.0f;
#pragma unroll
          for (int q = 0; q < RPT; q++) {
            const float x = y[q][t] * rn;
            y[q][t] = x;
            xprev[q] = x;
            if (t + 1 < T) {
              const float u = fmaxf(eps, y[q][t + 1] - x * gnext);
              y[q][t + 1] = u;
              ss += valid[q] ? u * u : 0.0f;
            }
          }
        }
      }
    }
    if (!xwave) {
      // the finished tile to its hand-off region; product groups copy it into X
#pragma unroll
      for (int q = 0; q < RPT; q++) {
        if (!valid[q]) continue;
#pragma unroll
        for (int v = 0; v < T / 4; v++)
          if (4 * v < tw)
            st_through4(wnview, (uint32_t)(quad_index(rows, j, v, rr[q]) * 16),
                        floatx4{y[q][4 * v], y[q][4 * v + 1], y[q][4 * v + 2], y[q][4 * v + 3]});
      }
    }
    signal_flag(a.flags + kWFlagCol + rank, tile_tag(a.epoch, j));
  }
}

template <int RPT, bool VEC, bool LOCAL>
__device__ __forceinline__ void w_column_role(const HalsWArgs a, int rank, int n_prod, float* lds) {
  const int tid = threadIdx.x, lane = tid & 63;
  unsigned long long* lpart = (unsigned long long*)(lds + T * TP);
  int* lflag = (int*)(lpart + 2 * kWWaves + 2);
  if (tid < 2 * kWWaves + 2) lpart[tid] = 0;  // exchange words and the protocol flag
  if constexpr (LOCAL) {
    __syncthreads();
    column_tiles<RPT, VEC, kProtoLocal>(a, rank, n_prod, lds);
  } else {
    // are all column groups on one XCD?  (one device-scope exchange per launch;
    // every group sees the same answers, so all take the same protocol)
    if (tid < 64) {
      const unsigned xcc = __builtin_amdgcn_s_getreg((31 << 11) | (0 << 6) | 20);
      const unsigned ptag = (a.epoch << 10) | 1023u;  // no column has index 1023
      if (lane == 0)
        __hip_atomic_store(a.slots + kSlotPlace + rank, pack_slot(ptag, __uint_as_float(xcc)),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      unsigned long long v = (unsigned long long)ptag << 32, v1 = v;
      int spins = 0;
      bool done;
      do {
        if (lane < a.n_col)
          v = __hip_atomic_load(a.slots + kSlotPlace + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (lane + 64 < a.n_col)
          v1 = __hip_atomic_load(a.slots + kSlotPlace + 64 + lane, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        done = __all((unsigned)(v >> 32) == ptag && (unsigned)(v1 >> 32) == ptag);
        if (!done && (++spins & 255) == 0 && timed_out(a.status)) break;
      } while (!done && spins < kSpinLimit);
      if (!done && lane == 0) atomicOr(a.status, 256);
      const unsigned first = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 0);
      const bool same = __all((lane >= a.n_col || (unsigned)v == first) &&
                              (lane + 64 >= a.n_col || (unsigned)v1 == first));
      if (lane == 0) *lflag = same;
    }
    __syncthreads();
    if (*lflag) column_tiles<RPT, VEC, kProtoXcd>(a, rank, n_prod, lds);
    else column_tiles<RPT, VEC, kProtoDevice>(a, rank, n_prod, lds);
  }
}

// A operand of the product for tile j, contraction columns [32 s, 32 s + 32):
// finished tiles (s < j) from their hand-off region, the rest still old in X.
template <bool VEC>
__device__ __forceinline__ void load_segment(floatx4 (&buf)[4], const HalsWArgs& a, int64_t r,
                                             bool rok, int j, int s, int h) {
  const int K = a.K;
  if (s < j) {
    const floatx4* __restrict__ Wn4 = (const floatx4*)a.Wn;
#pragma unroll
    for (int gi = 0; gi < 4; gi++)
      buf[gi] = rok ? Wn4[quad_index(a.rows, s, 2 * gi + h, r)] : floatx4{0, 0, 0, 0};
  } else {
    const float* p = a.X + r * K;
#pragma unroll
    for (int gi = 0; gi < 4; gi++) {
      const int lc = T * s + 8 * gi + 4 * h;
      if constexpr (VEC) {
        buf[gi] = (rok && lc < K) ? *(const floatx4*)(p + lc) : floatx4{0, 0, 0, 0};
      } else {
#pragma unroll
        for (int e = 0; e < 4; e++) buf[gi][e] = (rok && lc + e < K) ? p[lc + e] : 0.0f;
      }
    }
  }
}

__device__ __forceinline__ void mfma_segment(const floatx4 (&buf)[4], const float* __restrict__ bp,
                                             int s, int K, int lane, floatx16& acc) {
  const int h = lane >> 5, c = lane & 31;
#pragma unroll
  for (int gi = 0; gi < 4; gi++) {
    const int l = T * s + 8 * gi;
    if (l < K) {
#pragma unroll
      for (int e = 0; e < 4; e++)
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(buf[gi][e], bp[(l + 4 * h + e) * TP + c], acc, 0, 0, 0);
    }
  }
}

// acc += the product of row block r over every contraction segment but `skip`
// (off the critical path: one segment in flight at a time keeps registers low).
template <bool VEC>
__device__ __forceinline__ void block_segments(floatx16& acc, const HalsWArgs& a, int64_t r, bool rok,
                                               int j, int nseg, int skip, const float* __restrict__ bp,
                                               int lane) {
  const int h = lane >> 5;
  for (int sg = 0; sg < nseg; sg++) {
    if (sg == skip) continue;
    floatx4 buf[4];
    load_segment<VEC>(buf, a, r, rok, j, sg, h);
    mfma_segment(buf, bp, sg, a.K, lane, acc);
  }
}

// Copy finished tile s (width tws) of rows [rb, re) from its hand-off region
// into X; part i of np.
template <bool VEC>
__device__ __forceinline__ void copy_tile(const HalsWArgs& a, int s, int tws, int64_t rb, int64_t re,
                                          int i, int np) {
  const int64_t rows = a.rows;
  const int K = a.K;
  const int nv = (tws + 3) / 4;
  const int64_t nr = re - rb;
  const floatx4* __restrict__ Wn4 = (const floatx4*)a.Wn;
  const int64_t n = nr * nv;
  for (int64_t e = (int64_t)i * kWThreads + threadIdx.x; e < n; e += (int64_t)np * kWThreads) {
    const int v = (int)(e / nr);
    const int64_t r = rb + e % nr;
    const floatx4 f = Wn4[quad_index(rows, s, v, r)];
    float* dst = a.X + r * K + T * s + 4 * v;
    if (VEC && 4 * v + 4 <= tws) {
      *(floatx4*)dst = f;
    } else {
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (4 * v + q < tws) dst[q] = f[q];
    }
  }
}

// Product groups.  Only the previous tile's columns of the product for tile j
// depend on the column groups' latest output: everything else (Bterm, the old
// columns in X, the earlier finished tiles) is accumulated before waiting for
// the previous tile's flags and parked in LDS, so that after them only one
// 32-column segment of the contraction remains per row block.  Product group p
// serves column group g = p % n_col (the row blocks of its rows, which are a
// multiple of 32): it waits for that group's flags only, and that group waits
// only for its own product groups.
template <bool VEC>
__device__ __forceinline__ void w_product_role(const HalsWArgs a, int prank, int n_prod, float* lds) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, h = lane >> 5, c = lane & 31;
  const int K = a.K;
  const int jpw = a.jobs_per_wave, jpk = a.jobs_parked;      // jpk <= jpw
  float* bp = lds;                                            // [kpad(K)][TP]
  float* stash = lds + kpad(K) * TP + w * jpk * 32 * TP;      // this wave's [jpk][32][TP]
  const int64_t rows = a.rows;
  const int g = prank % a.n_col, gi = prank / a.n_col;
  const int npg = (n_prod - g + a.n_col - 1) / a.n_col;       // product groups serving g
  const int64_t grow0 = (int64_t)g * a.rows_per_group;
  const int64_t grow1 = grow0 + a.rows_per_group < rows ? grow0 + a.rows_per_group : rows;
  const int64_t blk0 = grow0 / 32;
  const int64_t nblk = (grow1 - grow0 + 31) / 32;             // row blocks of g
  const int nseg = (K + T - 1) / T;
  const __amdgpu_buffer_rsrc_t yview = store_view(a.Y, (int64_t)nseg * rows * T * 4);
  int j = 0;
  for (int a0 = 0; a0 < K; j++, a0 += T) {
    const int b0 = a0 + T < K ? a0 + T : K;
    const int tw = b0 - a0;
    __syncthreads();  // the previous tile's products no longer read bp
    {
      const floatx4* src = (const floatx4*)(a.panel + (int64_t)j * kpad(K) * T);
      for (int i = tid; i < kpad(K) * T / 4; i += kWThreads) {
        const floatx4 v = src[i];
        float* d = bp + (4 * i / T) * TP + (4 * i) % T;
        d[0] = v[0];
        d[1] = v[1];
        d[2] = v[2];
        d[3] = v[3];
      }
    }
    __syncthreads();
    // before the wait: Bterm plus every segment but the previous tile's, for
    // the jobs the LDS can park (all of them unless the rows per product
    // group are many and K large)
    for (int k = 0; k < jpk; k++) {
      const int64_t lb = ((int64_t)k * kWWaves + w) * npg + gi;
      if (lb >= nblk) break;
      const int64_t job = blk0 + lb;
      floatx16 acc;
#pragma unroll
      for (int jj = 0; jj < 4; jj++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int64_t rg = job * 32 + 8 * jj + 4 * h + i;
          acc[4 * jj + i] = (c < tw && rg < rows) ? a.Bterm[rg * K + a0 + c] : 0.0f;
        }
      const int64_t r = job * 32 + c;
      const bool rok = r < rows;
      block_segments<VEC>(acc, a, rok ? r : 0, rok, j, nseg, j - 1, bp, lane);
      float* st = stash + k * 32 * TP;
#pragma unroll
      for (int jj = 0; jj < 4; jj++)
#pragma unroll
        for (int i = 0; i < 4; i++) st[(8 * jj + 4 * h + i) * TP + c] = c < tw ? acc[4 * jj + i] : 0.0f;
    }
    if (j > 0) await_flags(a.flags + kWFlagCol + g, 1, 1, tile_tag(a.epoch, j - 1), a.status);
    for (int k = 0; k < jpw; k++) {
      const int64_t lb = ((int64_t)k * kWWaves + w) * npg + gi;
      if (lb >= nblk) break;
      const int64_t job = blk0 + lb;
      float* st = stash + (k % jpk) * 32 * TP;  // a later job reuses a stored job's slot
      if (k >= jpk) {
        // not parked: the whole product now, the previous tile's columns included
        floatx16 acc;
#pragma unroll
        for (int jj = 0; jj < 4; jj++)
#pragma unroll
          for (int i = 0; i < 4; i++) {
            const int64_t rg = job * 32 + 8 * jj + 4 * h + i;
            acc[4 * jj + i] = (c < tw && rg < rows) ? a.Bterm[rg * K + a0 + c] : 0.0f;
          }
        const int64_t r = job * 32 + c;
        const bool rok = r < rows;
        block_segments<VEC>(acc, a, rok ? r : 0, rok, j, nseg, -1, bp, lane);
#pragma unroll
        for (int jj = 0; jj < 4; jj++)
#pragma unroll
          for (int i = 0; i < 4; i++) st[(8 * jj + 4 * h + i) * TP + c] = c < tw ? acc[4 * jj + i] : 0.0f;
      } else if (j > 0) {
        const int64_t r = job * 32 + c;
        floatx4 last[4];
        load_segment<VEC>(last, a, r < rows ? r : 0, r < rows, j, j - 1, h);
        floatx16 acc;
#pragma unroll
        for (int e = 0; e < 16; e++) acc[e] = 0.0f;
        mfma_segment(last, bp, j - 1, K, lane, acc);
#pragma unroll
        for (int jj = 0; jj < 4; jj++)
#pragma unroll
          for (int i = 0; i < 4; i++)
            if (c < tw) st[(8 * jj + 4 * h + i) * TP + c] += acc[4 * jj + i];
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      // the block in the column-quad layout of Y
      const int64_t rg = job * 32 + c;
      if (rg < rows) {
#pragma unroll
        for (int kk = 0; kk < 4; kk++) {
          const int v = 4 * h + kk;
          const float* sp = st + c * TP + 4 * v;
          st_through4(yview, (uint32_t)(quad_index(rows, j, v, rg) * 16),
                      floatx4{sp[0], sp[1], sp[2], sp[3]});
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    signal_flag(a.flags + prank, tile_tag(a.epoch, j));
    // while the column groups run this tile: the previous finished tile into X
    if (j > 0) copy_tile<VEC>(a, j - 1, T, grow0, grow1, gi, npg);
  }
  // the last tile
  await_flags(a.flags + kWFlagCol + g, 1, 1, tile_tag(a.epoch, j - 1), a.status);
  copy_tile<VEC>(a, j - 1, K - (j - 1) * T, grow0, grow1, gi, npg);
}

template <int RPT, bool VEC, bool LOCAL>
__global__ __launch_bounds__(kWThreads) void hals_w_kernel(HalsWArgs a) {
  extern __shared__ float lds[];
  const int key = xcd_major_rank(blockIdx.x, gridDim.x);
  const int n_prod = (int)gridDim.x - a.n_col;
  if (key < a.n_col) w_column_role<RPT, VEC, LOCAL>(a, key, n_prod, lds);
  else w_product_role<VEC>(a, key - a.n_col, n_prod, lds);
}

template <int RPT, bool VEC, bool LOCAL>
const void* w_kernel_ptr() {
  return (const void*)hals_w_kernel<RPT, VEC, LOCAL>;
}

template <bool LOCAL>
const void* w_kernel_for_t(int rpt, bool vec) {
  if (rpt <= 1) return vec ? w_kernel_ptr<1, true, LOCAL>() : w_kernel_ptr<1, false, LOCAL>();
  if (rpt == 2) return vec ? w_kernel_ptr<2, true, LOCAL>() : w_kernel_ptr<2, false, LOCAL>();
  return vec ? w_kernel_ptr<4, true, LOCAL>() : w_kernel_ptr<4, false, LOCAL>();
}

const void* w_kernel_for(int rpt, bool vec, bool local) {
  return local ? w_kernel_for_t<true>(rpt, vec) : w_kernel_for_t<false>(rpt, vec);
}


}  // namespace

int hals_rows_per_group_h() { return kRowsH; }

// Which H-update kernel.  The rows-in-registers kernel takes 128 rows per
// workgroup and fills the chip from about 256 x 128 rows on.  Below that the
// LDS-resident kernel (32 rows per workgroup) keeps more CUs busy, as long as
// all its workgroups are resident at once; once they need a second round (its
// LDS holds two workgroups per CU up to K = 224, one above), the rows kernel's
// single round is shorter.  Measured on 11,000 rows: K = 200 LDS 48 us, rows
// 64 us; K = 240 LDS 96 us, rows 76 us; K = 400 LDS 220 us, rows 161 us; on
// 10,000 rows at K = 240: LDS 111 us, rows 79 us.
// NMF_H_KERNEL=rows|lds forces one (read when the half starts: measurement,
// tests).
static bool h_rows_kernel_for(int64_t rows, int K, int cus) {
  if (const char* e = getenv("NMF_H_KERNEL")) {
    if (e[0] == 'r') return true;
    if (e[0] == 'l') return false;
  }
  if (rows >= 32768) return true;
  const int64_t per_cu = (int64_t)(kRrLdsMax / (h_smem_floats(K) * 4));
  const int64_t groups = (rows + kRowsH - 1) / kRowsH;
  return groups > (int64_t)(cus > 0 ? cus : 256) * per_cu;
}

size_t hals_panel_floats(int K, int tile) {
  // the larger of the two orders: [tile][row][column] + the G blocks, or the
  // rows kernel's staging blocks (rows padded to 32 NT)
  const int ntiles = (K + tile - 1) / tile;
  const size_t plain = (size_t)ntiles * kpad(K) * tile + (size_t)ntiles * tile * tile;
  const size_t rows = (size_t)ntiles * rr_stage_floats((K + 31) / 32, tile);
  return plain > rows ? plain : rows;
}

bool hals_h_rows_layout(int64_t rows, int K, int cus, int tile) {
  return (tile != 0 && tile != T) || h_rows_kernel_for(rows, K, cus);
}

bool hals_tile_supported(int K, int tile) {
  if (tile == 32) return true;
  if (tile != 16 && tile != 64) return false;
  const int nt = (K + 31) / 32;
  return K % 4 == 0 && rr_smem_floats(nt, tile) * 4 <= kRrLdsMax && (tile != 64 || nt <= 6);
}

hipError_t hals_update(const HalsArgs& a, hipStream_t s) {
  const unsigned grid = (unsigned)((a.rows + kRowsH - 1) / kRowsH);
  if (grid == 0 || a.K <= 0) return hipSuccess;
  if (a.K > kMaxK || !a.panel) return hipErrorInvalidValue;
  HalsArgs b = a;
  const int tile = a.tile ? a.tile : T;
  if (!hals_tile_supported(a.K, tile)) return hipErrorInvalidValue;
  b.tile = tile;
  b.gblk = a.panel + (int64_t)((a.K + tile - 1) / tile) * kpad(a.K) * tile;
  const bool vec = (a.K % 4 == 0) && (((uintptr_t)a.X & 15) == 0);
  if (tile != T && !vec) return hipErrorInvalidValue;
  // widths other than 32: the rows-in-registers kernel only
  if (a.rows_layout) return h_rows_dispatch(b, vec, s);
  if (tile != T) return hipErrorInvalidValue;  // other widths: the rows kernel only
  const size_t bytes = h_smem_floats(a.K) * 4;
  const void* fn = vec ? (const void*)hals_h_kernel<true> : (const void*)hals_h_kernel<false>;
  hipError_t e = allow_smem(fn, bytes);
  if (e != hipSuccess) return e;
  if (vec) hals_h_kernel<true><<<grid, 256, bytes, s>>>(b);
  else hals_h_kernel<false><<<grid, 256, bytes, s>>>(b);
  return hipGetLastError();
}

int hals_w_max_rows_per_group() { return kWMaxRows; }

int hals_w_column_groups(int64_t rows, int device_cus) {
  const int64_t need = (rows + kWMaxRows - 1) / kWMaxRows;
  if (need <= 1) return 1;  // one group: the exchange stays in LDS
  // otherwise as many groups as one XCD holds (down to one row per row thread):
  // fewer rows per group shorten the per-column arithmetic and the per-tile
  // hand-offs, and the exchange among the groups of one XCD costs about the same
  int64_t n = (rows + kWRowThreads - 1) / kWRowThreads;
  const int64_t xcd = device_cus / 8;
  if (n > xcd) n = xcd;
  if (n < need) n = need;
  return (int)n;
}

int hals_w_max_column_groups() { return kWMaxColGroups; }

namespace {
// Row blocks per product wave: column group g's blocks over its product groups.
int jobs_per_wave(int rows_per_group, int grid, int n_col) {
  const int min_npg = (grid - n_col) / n_col;
  if (min_npg < 1) return 0;
  const int nb = (rows_per_group + 31) / 32;
  return (nb + kWWaves * min_npg - 1) / (kWWaves * min_npg);
}
}  // namespace

int hals_w_rows_per_group(int64_t rows, int n_col) {
  const int64_t r = (rows + n_col - 1) / n_col;
  return (int)((r + 31) / 32 * 32);
}

// Jobs per wave the product role parks in LDS before its wait (the rest are
// computed whole after it): as many as fit beside the tile's panel.
int jobs_parked(int K, int jpw) {
  int p = jpw;
  while (p > 1 && w_smem_bytes(K, p) > kLdsMax) p--;
  return p;
}

int hals_w_grid(int device_cus, int64_t rows, int K, int n_col) {
  const int grid = device_cus;  // one group per CU (the LDS request admits no second one)
  if (n_col < 1 || 2 * n_col > grid || grid > kWFlagCol) return 0;
  const int jpw = jobs_per_wave(hals_w_rows_per_group(rows, n_col), grid, n_col);
  if (jpw < 1) return 0;
  const size_t bytes = w_smem_bytes(K, jobs_parked(K, jpw));
  if (bytes > kLdsMax) return 0;
  for (int rpt : {1, 2, 4})
    for (bool vec : {false, true})
      for (bool local : {false, true}) {
        const void* fn = w_kernel_for(rpt, vec, local);
        if (allow_smem(fn, bytes) != hipSuccess) return 0;
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kWThreads, bytes) != hipSuccess ||
            nb < 1)
          return 0;
      }
  return grid;
}

hipError_t hals_w_update(const HalsWArgs& a, int grid, hipStream_t s) {
  if (a.rows <= 0 || a.K <= 0) return hipSuccess;
  if (a.n_col < 1 || 2 * a.n_col > grid || a.n_col > kWMaxColGroups || a.rows_per_group > kWMaxRows ||
      a.rows_per_group % 32 != 0 || (int64_t)a.n_col * a.rows_per_group < a.rows ||
      grid > kWFlagCol)
    return hipErrorInvalidValue;
  if (!a.panel) return hipErrorInvalidValue;
  HalsWArgs b = a;
  b.jobs_per_wave = jobs_per_wave(a.rows_per_group, grid, a.n_col);
  if (b.jobs_per_wave < 1) return hipErrorInvalidValue;
  b.jobs_parked = jobs_parked(a.K, b.jobs_per_wave);
  const size_t bytes = w_smem_bytes(a.K, b.jobs_parked);
  if (bytes > kLdsMax) return hipErrorInvalidValue;
  const int rpt = (a.rows_per_group + kWRowThreads - 1) / kWRowThreads;
  const bool vec = (a.K % 4 == 0) && (((uintptr_t)a.X & 15) == 0);
  const void* fn = w_kernel_for(rpt, vec, a.n_col == 1);
  hipError_t e = allow_smem(fn, bytes);
  if (e != hipSuccess) return e;
  void* args[] = {&b};
  // One group per CU, checked resident at plan creation (hals_w_grid), on a
  // stream whose earlier kernels have finished: a plain launch makes every
  // group resident.  The cooperative API guarantees it even on a shared device
  // but costs ~25 us per launch here; NMF_W_COOPERATIVE=1 selects it.  Without
  // it, a group that cannot become resident ends the sweep with a timeout
  // error (bounded waits), never a hang.
  static const bool coop = [] {
    const char* e = getenv("NMF_W_COOPERATIVE");
    return e && atoi(e) > 0;
  }();
  if (coop)
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kWThreads), args, (unsigned)bytes, s);
  return hipLaunchKernel(fn, dim3(grid), dim3(kWThreads), args, bytes, s);
}

}  // namespace plnmf
