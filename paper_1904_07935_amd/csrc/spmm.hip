// Sparse products of the sweep on CSR inputs: R = A^T W (over the CSR of A^T,
// gathering rows of W) and P = A H^T (over the CSR of A, gathering rows of
// Ht); the sparse-matrix/dense-matrix products of Alg. 1 (R and P statements)
// and of the GPU implementation in Sec. 4.2.
//
// Design: one wave per work item.  Items are planned once on the host from the
// row pointers: consecutive short rows are grouped until an item holds about
// L nonzeros (empty rows included, written as zeros), and a row longer than L
// -- the Zipf-skewed head of a term-by-document matrix -- is cut into segments
// of L.  So the grid stays balanced whatever the row-length skew.  Each nonzero
// gathers one K-contiguous factor row with 16-byte (FP32) or 8-byte (BF16)
// lane loads, several nonzeros in flight per wave.  Segments of long rows
// leave partial rows that a second pass adds up in segment order; nothing
// else needs a second pass, and no atomics are used: results are
// bitwise-reproducible.
//
// Wide rows (K > 128: one nonzero per wave step) take a flat variant.  A wave
// walking an item row by row waits, per step, for a column index and then for
// the factor row it names, a dependent chain of global loads of which the
// machine holds too few in flight (the gathers themselves mostly hit the L2).
// The flat variant loads the item's row pointers, column indices and values
// into registers at once (the item bounds are known), then walks the item's
// nonzeros as one list, 16 gathers in flight per step, and writes out each row
// as its end is passed.  BF16 rows stay packed in registers until use, so a
// batch holds 16 nonzeros at K up to 512 (FP32 at K > 256: 8); measured on
// the 10^5 x 3*10^5 corpus at K = 400, the BF16 product of A^T W runs at half
// the FP32 time that way, while deeper FP32 batches (16, at 3 waves/SIMD)
// gain nothing -- the FP32 gathers are bound by the memory system there.
// Summation order within a row is the nonzero order, as in the row-by-row
// kernel.
#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace plnmf {
namespace {

struct SpmmKArgs {
  const int32_t* rowptr;
  const int32_t* col;
  const void* val;
  const int4* items;
  const int32_t* slot;
  const void* X;
  float* out;
  float* carry;
  int64_t n_items;
  int K;             // columns computed (a slice of the factor's columns, or all)
  int64_t ldx, ldo;  // row strides of the factor and of the output
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
__global__ __launch_bounds__(256) void spmm_items(SpmmKArgs a) {
  constexpr int NPAR = 64 / LPN;  // nonzeros processed side by side per wave
  constexpr int UNR = 4;
  const int lane = threadIdx.x & 63;
  const int64_t it = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (it >= a.n_items) return;
  const int grp = lane / LPN, q = lane % LPN;
  const int K = a.K;
  const TX* X = (const TX*)a.X;
  const int4 item = a.items[it];
  const int slot = a.slot[it];
  for (int r = item.x; r < item.y; r++) {
    const int64_t rs = max(a.rowptr[r], item.z), re = min(a.rowptr[r + 1], item.w);
    floatx4 acc[VPL];
#pragma unroll
    for (int v = 0; v < VPL; v++) acc[v] = floatx4{0, 0, 0, 0};
    int64_t jj = rs + grp;
    for (; jj + (UNR - 1) * NPAR < re; jj += UNR * NPAR) {
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
        for (int v = 0; v < VPL; v++) x[u][v] = ld_x4<TX, VEC>(X + (int64_t)cc[u] * a.ldx, 4 * (q + LPN * v), K);
#pragma unroll
      for (int u = 0; u < UNR; u++)
#pragma unroll
        for (int v = 0; v < VPL; v++) acc[v] += vv[u] * x[u][v];
    }
    for (; jj < re; jj += NPAR) {
      const int32_t cc = a.col[jj];
      const float vv = ld_val<TV>(a.val, jj);
#pragma unroll
      for (int v = 0; v < VPL; v++) acc[v] += vv * ld_x4<TX, VEC>(X + (int64_t)cc * a.ldx, 4 * (q + LPN * v), K);
    }
    // combine the NPAR lane groups (fixed butterfly order)
#pragma unroll
    for (int off = LPN; off < 64; off <<= 1)
#pragma unroll
      for (int v = 0; v < VPL; v++)
#pragma unroll
        for (int e = 0; e < 4; e++) acc[v][e] += __shfl_xor(acc[v][e], off);
    float* dst = slot >= 0 ? a.carry + (int64_t)slot * K : a.out + (int64_t)r * a.ldo;
    if (grp == 0) {
#pragma unroll
      for (int v = 0; v < VPL; v++) {
        const int cb = 4 * (q + LPN * v);
#pragma unroll
        for (int e = 0; e < 4; e++)
          if (cb + e < K) dst[cb + e] = acc[v][e];
      }
    }
  }
}

constexpr int kMaxRowsPerItem = 256;
constexpr int kFlatMaxNnz = 128;  // item nonzeros the flat kernel prefetches

// Element k of a register array spread over the wave (element 64 m + l in lane
// l of arr[m]); k is wave-uniform.
template <int N, typename V>
__device__ __forceinline__ V wave_elem(const V (&arr)[N], int k) {
  V v = arr[0];
#pragma unroll
  for (int m = 1; m < N; m++)
    if ((k >> 6) == m) v = arr[m];
  return __builtin_bit_cast(V, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k & 63));
}

// EPL: factor elements per lane and load -- 4 (FP32 float4, or BF16 8-byte
// loads), or 8 (BF16 16-byte loads; K % 8 == 0, rows 16-byte aligned).
template <int VPL, typename TV, typename TX, bool VEC, int EPL = 4, int UNR_ = 0>
__global__ __launch_bounds__(256) void spmm_flat(SpmmKArgs a) {
  static_assert(EPL == 4 || (EPL == 8 && VEC && sizeof(TX) == 2 && VPL == 1),
                "16-byte BF16 loads only");
  constexpr int NQ = EPL / 4;  // float4 accumulators per load
  constexpr int UNR = UNR_ ? UNR_ : ((EPL == 8 || VPL == 1) ? 16 : 8);  // gathers per batch
  constexpr int MZ = kFlatMaxNnz / 64;
  constexpr int MR = (kMaxRowsPerItem + 1 + 63) / 64;
  const int lane = threadIdx.x & 63;
  const int64_t it = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (it >= a.n_items) return;
  const int K = a.K;
  const TX* X = (const TX*)a.X;
  const int4 item = a.items[it];
  const int slot = a.slot[it];
  const int r0 = item.x, nr = item.y - item.x;
  const int j0 = item.z, nz = item.w - item.z;  // nz <= kFlatMaxNnz, nr <= kMaxRowsPerItem
  int32_t pc[MZ], prp[MR];
  float pv[MZ];
#pragma unroll
  for (int m = 0; m < MZ; m++) {
    const int i = lane + 64 * m;
    pc[m] = i < nz ? a.col[j0 + i] : 0;
    pv[m] = i < nz ? ld_val<TV>(a.val, j0 + i) : 0.0f;
  }
#pragma unroll
  for (int m = 0; m < MR; m++) {
    const int i = lane + 64 * m;
    prp[m] = i <= nr ? a.rowptr[r0 + i] : 0;
  }
  // end (item-local nonzero index) of local row r; a long row's segment ends at nz
  auto row_end = [&](int r) {
    const int e = wave_elem(prp, r + 1) - j0;
    return e < nz ? e : nz;
  };
  floatx4 acc[VPL * NQ];
#pragma unroll
  for (int v = 0; v < VPL * NQ; v++) acc[v] = floatx4{0, 0, 0, 0};
  int r = 0;
  int rend = nr > 0 ? row_end(0) : nz;
  auto flush = [&]() {
    float* dst = slot >= 0 ? a.carry + (int64_t)slot * K : a.out + (int64_t)(r0 + r) * a.ldo;
#pragma unroll
    for (int v = 0; v < VPL; v++) {
      const int cb = EPL * (lane + 64 * v);
#pragma unroll
      for (int q = 0; q < NQ; q++) {
        if constexpr (VEC) {
          if (cb < K) *(floatx4*)(dst + cb + 4 * q) = acc[v * NQ + q];
        } else {
#pragma unroll
          for (int e = 0; e < 4; e++)
            if (cb + e < K) dst[cb + e] = acc[v * NQ + q][e];
        }
        acc[v * NQ + q] = floatx4{0, 0, 0, 0};
      }
    }
    r++;
    rend = r < nr ? row_end(r) : nz;
  };
  if constexpr (EPL == 8) {
    // BF16 rows kept packed until use (4 VGPRs per nonzero), so twice as
    // many gathers are in flight per wave as with unpacked floats
    for (int jb = 0; jb < nz; jb += UNR) {
      bf16x8 xb[UNR];
#pragma unroll
      for (int u = 0; u < UNR; u++) {
        const int j = jb + u;
        const int64_t col = j < nz ? wave_elem(pc, j) : 0;
        const int cb = 8 * lane;
        xb[u] = (j < nz && cb < K) ? *(const bf16x8*)((const __bf16*)X + col * a.ldx + cb)
                                   : bf16x8{};
      }
#pragma unroll
      for (int u = 0; u < UNR; u++) {
        const int j = jb + u;
        if (j < nz) {
          while (j >= rend && r < nr) flush();
          const float vv = wave_elem(pv, j);
          const bf16x8 b = xb[u];
          acc[0] += vv * floatx4{(float)b[0], (float)b[1], (float)b[2], (float)b[3]};
          acc[1] += vv * floatx4{(float)b[4], (float)b[5], (float)b[6], (float)b[7]};
        }
      }
    }
  } else {
    for (int jb = 0; jb < nz; jb += UNR) {
      floatx4 x[UNR][VPL];
#pragma unroll
      for (int u = 0; u < UNR; u++) {
        const int j = jb + u;
        const int64_t col = j < nz ? wave_elem(pc, j) : 0;
#pragma unroll
        for (int v = 0; v < VPL; v++) {
          const int cb = EPL * (lane + 64 * v);
          x[u][v] = j < nz ? ld_x4<TX, VEC>(X + col * a.ldx, cb, K) : floatx4{0, 0, 0, 0};
        }
      }
#pragma unroll
      for (int u = 0; u < UNR; u++) {
        const int j = jb + u;
        if (j < nz) {
          while (j >= rend && r < nr) flush();  // rows that end here, empty ones included
          const float vv = wave_elem(pv, j);
#pragma unroll
          for (int v = 0; v < VPL; v++) acc[v] += vv * x[u][v];
        }
      }
    }
  }
  while (r < nr) flush();
}

// One workgroup per long row: add its segments' partial rows.  Thread (v, sl)
// sums columns 4v..4v+3 over segments sl, sl + S, ... (S slices, in order, four
// loads in flight), then slice 0 adds the S slice sums in slice order: a fixed
// order for a given K and segment count, so results are bitwise reproducible.
constexpr int kFixThreads = 512;

__global__ __launch_bounds__(kFixThreads) void spmm_fixup(const int32_t* __restrict__ fix,
                                                          int64_t n_fix,
                                                          const float* __restrict__ carry,
                                                          float* __restrict__ out, int K,
                                                          int64_t ldo) {
  __shared__ floatx4 part[kFixThreads];
  const int64_t i = blockIdx.x;
  if (i >= n_fix) return;
  const int nv = (K + 3) / 4;
  const int S = kFixThreads / nv > 0 ? kFixThreads / nv : 1;
  const int t = threadIdx.x;
  const int v = t % nv, sl = t / nv;
  const int64_t r = fix[3 * i], first = fix[3 * i + 1], cnt = fix[3 * i + 2];
  const bool vec = (K % 4) == 0;
  floatx4 acc = floatx4{0, 0, 0, 0};
  if (sl < S && t < nv * S) {
    auto seg = [&](int64_t g) -> floatx4 {
      const float* p = carry + (first + g) * K + 4 * v;
      if (vec) return *(const floatx4*)p;
      floatx4 x;
#pragma unroll
      for (int e = 0; e < 4; e++) x[e] = 4 * v + e < K ? p[e] : 0.0f;
      return x;
    };
    int64_t g = sl;
    for (; g + 3 * S < cnt; g += 4 * S) {
      const floatx4 x0 = seg(g), x1 = seg(g + S), x2 = seg(g + 2 * S), x3 = seg(g + 3 * S);
      acc += x0;
      acc += x1;
      acc += x2;
      acc += x3;
    }
    for (; g < cnt; g += S) acc += seg(g);
  }
  part[t] = acc;
  __syncthreads();
  if (sl == 0 && t < nv) {
    floatx4 tot = part[v];
    for (int k = 1; k < S; k++) tot += part[k * nv + v];
    float* dst = out + r * ldo + 4 * v;
    if (vec) {
      *(floatx4*)dst = tot;
    } else {
#pragma unroll
      for (int e = 0; e < 4; e++)
        if (4 * v + e < K) dst[e] = tot[e];
    }
  }
}

template <int VPL, int LPN, typename TV, typename TX>
hipError_t launch_t(const SpmmKArgs& a, bool vec, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.n_items + 3) / 4);
  if (blocks == 0) return hipSuccess;
  if (vec) spmm_items<VPL, LPN, TV, TX, true><<<blocks, 256, 0, s>>>(a);
  else spmm_items<VPL, LPN, TV, TX, false><<<blocks, 256, 0, s>>>(a);
  return hipGetLastError();
}

template <int VPL, typename TV, typename TX>
hipError_t launch_f(const SpmmKArgs& a, bool vec, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.n_items + 3) / 4);
  if (blocks == 0) return hipSuccess;
  if (vec) spmm_flat<VPL, TV, TX, true><<<blocks, 256, 0, s>>>(a);
  else spmm_flat<VPL, TV, TX, false><<<blocks, 256, 0, s>>>(a);
  return hipGetLastError();
}

template <typename TV, typename TX>
hipError_t launch_k(const SpmmKArgs& a, bool vec, bool vec8, bool flat, hipStream_t s) {
  const int n4 = (a.K + 3) / 4;
  if constexpr (sizeof(TX) == 2) {
    // BF16 rows longer than 256 elements: one 16-byte load of 8 per lane
    if (flat && n4 > 64 && vec8) {
      const unsigned blocks = (unsigned)((a.n_items + 3) / 4);
      if (blocks == 0) return hipSuccess;
      spmm_flat<1, TV, TX, true, 8><<<blocks, 256, 0, s>>>(a);
      return hipGetLastError();
    }
  }
  if (flat && n4 > 32) return n4 <= 64 ? launch_f<1, TV, TX>(a, vec, s) : launch_f<2, TV, TX>(a, vec, s);
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

int spmm_item_nnz(int64_t nnz) {
  (void)nnz;
  return 128;
}

SpmmSizes spmm_sizes(int64_t rows, int64_t nnz, int L) {
  SpmmSizes z;
  z.items = rows + 2 * (nnz / L) + 2;
  z.fix = nnz / L + 1;
  z.seg = 2 * (nnz / L) + 2;
  return z;
}

hipError_t spmm_build(SpmmPlan* p, hipStream_t s, const uint8_t* skip) {
  const int64_t rows = p->rows;
  const int L = p->L;
  std::vector<int32_t> rp((size_t)rows + 1);
  hipError_t e = hipMemcpyAsync(rp.data(), p->rowptr, rp.size() * sizeof(int32_t),
                                hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  std::vector<int4> items;
  std::vector<int32_t> slot, fix;
  int32_t nseg = 0;
  int64_t r = 0;
  while (r < rows) {
    const int64_t len = (int64_t)rp[r + 1] - rp[r];
    if (len > L && skip && skip[r]) {  // a long row computed elsewhere: no items
      r++;
      continue;
    }
    if (len > L) {  // a long row: segments of L nonzeros, summed by the fixup pass
      const int32_t first = nseg;
      int32_t cnt = 0;
      for (int64_t j = rp[r]; j < rp[r + 1]; j += L) {
        const int64_t je = std::min<int64_t>(j + L, rp[r + 1]);
        items.push_back(make_int4((int)r, (int)r + 1, (int)j, (int)je));
        slot.push_back(nseg++);
        cnt++;
      }
      fix.push_back((int32_t)r);
      fix.push_back(first);
      fix.push_back(cnt);
      r++;
      continue;
    }
    const int64_t r0 = r, j0 = rp[r];
    while (r < rows && r - r0 < kMaxRowsPerItem && (int64_t)rp[r + 1] - rp[r] <= L &&
           (int64_t)rp[r + 1] - j0 <= L)
      r++;
    items.push_back(make_int4((int)r0, (int)r, (int)j0, (int)rp[r]));
    slot.push_back(-1);
  }
  const SpmmSizes cap = spmm_sizes(rows, p->nnz, L);
  if ((int64_t)items.size() > cap.items || (int64_t)fix.size() / 3 > cap.fix || nseg > cap.seg)
    return hipErrorInvalidValue;  // cannot happen: the bounds cover every partition
  p->n_items = (int64_t)items.size();
  p->n_fix = (int64_t)fix.size() / 3;
  p->n_seg = nseg;
  if (!items.empty()) {
    e = hipMemcpyAsync(p->items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(p->item_slot, slot.data(), slot.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
  }
  if (!fix.empty()) {
    e = hipMemcpyAsync(p->fix, fix.data(), fix.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipStreamSynchronize(s);  // the host vectors go out of scope
}

hipError_t spmm(const SpmmPlan& p, Elem t, const void* X, int K, float* out, hipStream_t s) {
  return spmm_slice(p, t, X, K, 0, K, out, K, s);
}

hipError_t spmm_slice(const SpmmPlan& p, Elem t, const void* X0, int64_t ldx, int k0, int K,
                      float* out0, int64_t ldo, hipStream_t s) {
  const size_t esz = t == Elem::F32 ? 4 : 2;
  const void* X = (const char*)X0 + (size_t)k0 * esz;
  float* out = out0 + k0;
  SpmmKArgs a;
  a.ldx = ldx;
  a.ldo = ldo;
  a.rowptr = p.rowptr;
  a.col = p.col;
  a.val = p.val;
  a.items = p.items;
  a.slot = p.item_slot;
  a.X = X;
  a.out = out;
  a.carry = p.carry;
  a.n_items = p.n_items;
  a.K = K;
  const bool vec = (K % 4 == 0) && (ldx % 4 == 0) && (ldo % 4 == 0) &&
                   (((uintptr_t)X) % (4 * esz) == 0) && ((uintptr_t)out % 16 == 0) &&
                   ((uintptr_t)p.carry % 16 == 0);
  const bool vec8 = vec && K % 8 == 0 && ldx % 8 == 0 && ((uintptr_t)X) % 16 == 0;
  const bool flat = p.L <= kFlatMaxNnz;  // the flat kernel holds a whole item in registers
  hipError_t e = t == Elem::F32 ? launch_k<float, float>(a, vec, vec8, flat, s)
                                : launch_k<__bf16, __bf16>(a, vec, vec8, flat, s);
  if (e != hipSuccess) return e;
  if (p.n_fix > 0) {
    spmm_fixup<<<(unsigned)p.n_fix, kFixThreads, 0, s>>>(p.fix, p.n_fix, p.carry, out, K, ldo);
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

// One wave per row (the last wave checks the end pointers): every nonzero is
// checked by its own lane, so the long rows of a Zipf corpus cost no more than
// a few wave steps.
__global__ __launch_bounds__(256) void csr_check(int64_t rows, int64_t cols, int64_t nnz,
                                                 const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col,
                                                 const float* __restrict__ val,
                                                 int32_t* __restrict__ flag) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r > rows) return;
  if (r == rows) {
    if (lane == 0 && (rowptr[rows] != nnz || rowptr[0] != 0)) atomicOr(flag, 1);
    return;
  }
  const int64_t a = rowptr[r], b = rowptr[r + 1];
  if (a > b || a < 0 || b > nnz) {
    if (lane == 0) atomicOr(flag, 1);
    return;
  }
  int bad = 0;
  for (int64_t j = a + lane; j < b; j += 64) {
    const int32_t c = col[j];
    if (c < 0 || c >= cols || (j > a && col[j - 1] >= c)) bad |= 2;  // in range, strictly increasing
    const float v = val[j];
    if (!(v >= 0.0f) || isinf(v)) bad |= 4;
  }
  if (bad) atomicOr(flag, bad);
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
  csr_check<<<(unsigned)((rows + 1 + 3) / 4), 256, 0, s>>>(rows, cols, nnz, rowptr, col, val, flag);
  return hipGetLastError();
}

}  // namespace plnmf
