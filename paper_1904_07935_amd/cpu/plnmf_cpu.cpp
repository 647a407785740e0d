// PL-NMF-cpu: the tiled FAST-HALS sweep (Alg. 1 reordered as Alg. 2, Eq. 4-6)
// on the host in FP64 with OpenMP -- the CPU comparison baseline of the GPU
// library.  See include/nmf_cpu.h for the interface.
#include "../../include/nmf_cpu.h"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

namespace {

constexpr int kChunks = 64;  // fixed row chunks of every reduction (thread-count independent)
constexpr int kBlock = 32;   // rows per block of the updates and Grams

struct Csr {
  std::vector<int64_t> rp;
  std::vector<int32_t> col;
  std::vector<double> val;
};

}  // namespace

struct nmf_cpu_plan_s {
  int64_t V = 0, D = 0;
  int K = 0, T = 0, threads = 1;
  double eps = 0.0;
  bool sparse = true;
  Csr A, At;                       // CSR of A (V rows) and of A^T (D rows)
  std::vector<double> dense;       // [V, D] when A is dense
  double* W = nullptr;             // [V, K]
  double* Ht = nullptr;            // [D, K]
  std::vector<double> R, P, S, Q;  // R [D,K], P [V,K], S, Q [K,K]
  std::vector<double> old;         // the half's old factor [max(V,D), K]
  std::vector<double> gpart;       // Gram partials [kChunks][K][K]
  double a2 = 0.0;
};

namespace {

int64_t chunk_lo(int64_t n, int c) { return n * c / kChunks; }

// G = X^T X for X [rows, K]: per chunk, the upper triangle accumulated four
// rows of X at a time (four FMAs per load and store of a partial row);
// chunks summed in order.
void gram(nmf_cpu_plan_s* p, const double* X, int64_t rows, double* G) {
  const int K = p->K;
  const size_t KK = (size_t)K * K;
#pragma omp parallel num_threads(p->threads)
  {
#pragma omp for schedule(dynamic, 1)
    for (int c = 0; c < kChunks; c++) {
      double* g = p->gpart.data() + (size_t)c * KK;
      std::fill(g, g + KK, 0.0);
      const int64_t r1 = chunk_lo(rows, c + 1);
      int64_t r = chunk_lo(rows, c);
      for (; r + 4 <= r1; r += 4) {
        const double* x0 = X + r * K;
        const double* x1 = x0 + K;
        const double* x2 = x1 + K;
        const double* x3 = x2 + K;
        for (int i = 0; i < K; i++) {
          const double a0 = x0[i], a1 = x1[i], a2 = x2[i], a3 = x3[i];
          double* gi = g + (size_t)i * K;
          for (int j = i; j < K; j++) gi[j] += (a0 * x0[j] + a1 * x1[j]) + (a2 * x2[j] + a3 * x3[j]);
        }
      }
      for (; r < r1; r++) {
        const double* x0 = X + r * K;
        for (int i = 0; i < K; i++) {
          const double a0 = x0[i];
          double* gi = g + (size_t)i * K;
          for (int j = i; j < K; j++) gi[j] += a0 * x0[j];
        }
      }
    }
#pragma omp for schedule(static)
    for (int i = 0; i < K; i++)
      for (int j = i; j < K; j++) {
        double s = 0.0;
        for (int c = 0; c < kChunks; c++) s += p->gpart[(size_t)c * KK + (size_t)i * K + j];
        G[(size_t)i * K + j] = s;
        G[(size_t)j * K + i] = s;
      }
  }
}

// out[r, :] = sum_j a[r, j] X[j, :] over a CSR (rows n_rows), or the dense form.
void spmm(nmf_cpu_plan_s* p, const Csr& m, int64_t n_rows, const double* X, double* out) {
  const int K = p->K;
#pragma omp parallel for schedule(dynamic, 64) num_threads(p->threads)
  for (int64_t r = 0; r < n_rows; r++) {
    double* o = out + r * K;
    std::fill(o, o + K, 0.0);
    for (int64_t j = m.rp[r]; j < m.rp[r + 1]; j++) {
      const double a = m.val[j];
      const double* x = X + (int64_t)m.col[j] * K;
      for (int k = 0; k < K; k++) o[k] += a * x[k];
    }
  }
}

// R = A^T W (dense A [V, D]): blocks of documents, all terms streamed once.
void dense_R(nmf_cpu_plan_s* p) {
  const int K = p->K;
  const int64_t V = p->V, D = p->D;
#pragma omp parallel for schedule(dynamic, 1) num_threads(p->threads)
  for (int64_t d0 = 0; d0 < D; d0 += kBlock) {
    const int nb = (int)std::min<int64_t>(kBlock, D - d0);
    double* o = p->R.data() + d0 * K;
    std::fill(o, o + (size_t)nb * K, 0.0);
    for (int64_t v = 0; v < V; v++) {
      const double* a = p->dense.data() + v * D + d0;
      const double* w = p->W + v * K;
      for (int r = 0; r < nb; r++) {
        const double c = a[r];
        double* orow = o + (size_t)r * K;
        for (int k = 0; k < K; k++) orow[k] += c * w[k];
      }
    }
  }
}

// P = A H^T (dense A): blocks of terms, all documents streamed once per block.
void dense_P(nmf_cpu_plan_s* p) {
  const int K = p->K;
  const int64_t V = p->V, D = p->D;
#pragma omp parallel for schedule(dynamic, 1) num_threads(p->threads)
  for (int64_t v0 = 0; v0 < V; v0 += kBlock) {
    const int nb = (int)std::min<int64_t>(kBlock, V - v0);
    double* o = p->P.data() + v0 * K;
    std::fill(o, o + (size_t)nb * K, 0.0);
    for (int64_t d = 0; d < D; d++) {
      const double* h = p->Ht + d * K;
      for (int r = 0; r < nb; r++) {
        const double c = p->dense[(v0 + r) * D + d];
        double* orow = o + (size_t)r * K;
        for (int k = 0; k < K; k++) orow[k] += c * h[k];
      }
    }
  }
}

// For every row r of a block of nb rows (stride K):
//   y[r, j0:j1] -= sum over l in [l0, l1) of c[r, l] * G[l, j0:j1],
// four rows of G per pass over the block (each reused by all nb rows from L1,
// four FMAs per load and store of y).
void block_axpy(double* y, const double* c, int nb, const double* G, int K, int l0, int l1, int j0,
                int j1) {
  int l = l0;
  for (; l + 4 <= l1; l += 4) {
    const double* g0 = G + (size_t)l * K;
    const double* g1 = g0 + K;
    const double* g2 = g1 + K;
    const double* g3 = g2 + K;
    for (int r = 0; r < nb; r++) {
      const double* cr = c + (size_t)r * K;
      const double c0 = cr[l], c1 = cr[l + 1], c2 = cr[l + 2], c3 = cr[l + 3];
      double* yr = y + (size_t)r * K;
      for (int j = j0; j < j1; j++) yr[j] -= ((c0 * g0[j] + c1 * g1[j]) + (c2 * g2[j] + c3 * g3[j]));
    }
  }
  for (; l < l1; l++) {
    const double* g0 = G + (size_t)l * K;
    for (int r = 0; r < nb; r++) {
      const double c0 = c[(size_t)r * K + l];
      double* yr = y + (size_t)r * K;
      for (int j = j0; j < j1; j++) yr[j] -= c0 * g0[j];
    }
  }
}

// Phase 1 (Eq. 4) for a block of nb rows of y (old values in `xo`): every
// tile's old values subtracted from the columns left of it.
void phase1(const nmf_cpu_plan_s* p, double* y, const double* xo, int nb, const double* G) {
  const int K = p->K, T = p->T;
  for (int a = T; a < K; a += T) block_axpy(y, xo, nb, G, K, a, std::min(a + T, K), 0, a);
}

// Phase 3 (Eq. 6): the finished tile [a, b) subtracted from the columns right of it.
void phase3(const nmf_cpu_plan_s* p, double* y, int nb, int a, int b, const double* G) {
  block_axpy(y, y, nb, G, p->K, a, b, b, p->K);
}

// Phase 2 (Eq. 5, +Bterm) of column t in tile [a, b) for one row.
inline double phase2(const double* yr, const double* xr, const double* g, double bterm, int a,
                     int b, int t, double eps) {
  double s = 0.0;
  for (int l = a; l < t; l++) s += yr[l] * g[l];
  for (int l = t; l < b; l++) s += xr[l] * g[l];
  return std::max(eps, yr[t] + bterm - s);
}

// The H half's update (no normalisation): rows independent, blocks in parallel.
void update_h(nmf_cpu_plan_s* p) {
  const int K = p->K, T = p->T;
  const int64_t D = p->D;
  std::copy(p->Ht, p->Ht + D * K, p->old.begin());
#pragma omp parallel for schedule(dynamic, 1) num_threads(p->threads)
  for (int64_t r0 = 0; r0 < D; r0 += kBlock) {
    const int nb = (int)std::min<int64_t>(kBlock, D - r0);
    double* y = p->Ht + r0 * K;
    const double* xo = p->old.data() + r0 * K;
    phase1(p, y, xo, nb, p->S.data());
    for (int a = 0; a < K; a += T) {
      const int b = std::min(a + T, K);
      for (int t = a; t < b; t++) {
        const double* g = p->S.data() + (size_t)t * K;
        for (int r = 0; r < nb; r++)
          y[(size_t)r * K + t] = phase2(y + (size_t)r * K, xo + (size_t)r * K, g,
                                        p->R[(r0 + r) * K + t], a, b, t, p->eps);
      }
      if (b < K) phase3(p, y, nb, a, b, p->S.data());
    }
  }
}

// The W half's update: W_new = W_old diag(Q), phase 1, then per tile phase 2
// with every column normalised over all rows (a reduction per column), phase 3.
void update_w(nmf_cpu_plan_s* p) {
  const int K = p->K, T = p->T;
  const int64_t V = p->V;
  const double* Q = p->Q.data();
  std::copy(p->W, p->W + V * K, p->old.begin());
  double part[kChunks];
  double norm = 1.0;
#pragma omp parallel num_threads(p->threads)
  {
#pragma omp for schedule(dynamic, 1)
    for (int64_t r0 = 0; r0 < V; r0 += kBlock) {
      const int nb = (int)std::min<int64_t>(kBlock, V - r0);
      double* y = p->W + r0 * K;
      const double* xo = p->old.data() + r0 * K;
      for (int r = 0; r < nb; r++)
        for (int j = 0; j < K; j++) y[(size_t)r * K + j] = xo[(size_t)r * K + j] * Q[(size_t)j * K + j];
      phase1(p, y, xo, nb, Q);
    }
    for (int a = 0; a < K; a += T) {
      const int b = std::min(a + T, K);
      for (int t = a; t < b; t++) {
        const double* g = Q + (size_t)t * K;
#pragma omp for schedule(static)
        for (int c = 0; c < kChunks; c++) {
          double ss = 0.0;
          for (int64_t r = chunk_lo(V, c); r < chunk_lo(V, c + 1); r++) {
            double* yr = p->W + r * K;
            const double v = phase2(yr, p->old.data() + r * K, g, p->P[r * K + t], a, b, t, p->eps);
            yr[t] = v;
            ss += v * v;
          }
          part[c] = ss;
        }
#pragma omp single
        {
          double s = 0.0;
          for (int c = 0; c < kChunks; c++) s += part[c];
          norm = std::sqrt(s);
        }
#pragma omp for schedule(static)
        for (int c = 0; c < kChunks; c++)
          for (int64_t r = chunk_lo(V, c); r < chunk_lo(V, c + 1); r++) p->W[r * K + t] /= norm;
      }
      if (b < K) {
#pragma omp for schedule(dynamic, 1)
        for (int64_t r0 = 0; r0 < V; r0 += kBlock)
          phase3(p, p->W + r0 * K, (int)std::min<int64_t>(kBlock, V - r0), a, b, Q);
      }
    }
  }
}

double dot_chunks(const nmf_cpu_plan_s* p, const double* x, const double* y, int64_t n) {
  double part[kChunks];
#pragma omp parallel for schedule(static) num_threads(p->threads)
  for (int c = 0; c < kChunks; c++) {
    double s = 0.0;
    for (int64_t i = chunk_lo(n, c); i < chunk_lo(n, c + 1); i++) s += x[i] * y[i];
    part[c] = s;
  }
  double s = 0.0;
  for (int c = 0; c < kChunks; c++) s += part[c];
  return s;
}

// Relative objective after a sweep: sparse A by the identity
// ||A||^2 - 2 <W, A H^T> + <W^T W, H H^T> (P and Q are this sweep's), dense A
// by the explicit residual.
double rel_objective(nmf_cpu_plan_s* p) {
  const int K = p->K;
  double e2;
  if (p->sparse) {
    std::vector<double> S2((size_t)K * K);
    gram(p, p->W, p->V, S2.data());
    e2 = p->a2 - 2.0 * dot_chunks(p, p->W, p->P.data(), p->V * K) +
         dot_chunks(p, S2.data(), p->Q.data(), (int64_t)K * K);
  } else {
    double part[kChunks];
    const int64_t V = p->V, D = p->D;
#pragma omp parallel for schedule(static) num_threads(p->threads)
    for (int c = 0; c < kChunks; c++) {
      double s = 0.0;
      for (int64_t v = chunk_lo(V, c); v < chunk_lo(V, c + 1); v++) {
        const double* w = p->W + v * K;
        for (int64_t d = 0; d < D; d++) {
          const double* h = p->Ht + d * K;
          double wh = 0.0;
          for (int k = 0; k < K; k++) wh += w[k] * h[k];
          const double e = p->dense[v * D + d] - wh;
          s += e * e;
        }
      }
      part[c] = s;
    }
    e2 = 0.0;
    for (int c = 0; c < kChunks; c++) e2 += part[c];
  }
  return std::sqrt(std::max(e2, 0.0) / p->a2);
}

void sweep(nmf_cpu_plan_s* p) {
  // H half: R = A^T W, S = W^T W, then the H loop
  gram(p, p->W, p->V, p->S.data());
  if (p->sparse) spmm(p, p->At, p->D, p->W, p->R.data());
  else dense_R(p);
  update_h(p);
  // W half: P = A H^T, Q = H H^T (the new H), then the W loop
  if (p->sparse) spmm(p, p->A, p->V, p->Ht, p->P.data());
  else dense_P(p);
  gram(p, p->Ht, p->D, p->Q.data());
  update_w(p);
}

}  // namespace

extern "C" {

int nmf_cpu_init(nmf_cpu_plan* out, int64_t V, int64_t D, const int32_t* rowptr,
                 const int32_t* col, const float* val, int K, double eps, int tile, int threads,
                 double* W, double* Ht) {
  if (!out || !val || !W || !Ht) return -1;
  *out = nullptr;
  if (V < 1 || D < 1 || K < 1 || K > std::min(V, D)) return -2;
  if (!(eps > 0.0) || !std::isfinite(eps) || tile < 0 || tile > K || threads < 0) return -1;
  nmf_cpu_plan_s* p = new (std::nothrow) nmf_cpu_plan_s();
  if (!p) return -1;
  p->V = V;
  p->D = D;
  p->K = K;
  p->eps = eps;
  p->T = tile > 0 ? tile : std::max(1, (int)std::lround(std::sqrt((double)K)));
  p->threads = threads > 0 ? threads : omp_get_max_threads();
  p->W = W;
  p->Ht = Ht;
  p->sparse = rowptr != nullptr;
  double a2 = 0.0;
  if (p->sparse) {
    if (!col || rowptr[0] != 0) {
      delete p;
      return -2;
    }
    const int64_t nnz = rowptr[V];
    p->A.rp.resize(V + 1);
    for (int64_t v = 0; v <= V; v++) {
      p->A.rp[v] = rowptr[v];
      if (v > 0 && rowptr[v] < rowptr[v - 1]) {
        delete p;
        return -2;
      }
    }
    p->A.col.assign(col, col + nnz);
    p->A.val.resize(nnz);
    for (int64_t j = 0; j < nnz; j++) {
      if (col[j] < 0 || col[j] >= D || !(val[j] >= 0.0f) || std::isinf(val[j])) {
        delete p;
        return col[j] < 0 || col[j] >= D ? -2 : -5;
      }
      p->A.val[j] = val[j];
      a2 += (double)val[j] * val[j];
    }
    // CSR of A^T by a counting sort (columns come out sorted)
    p->At.rp.assign(D + 1, 0);
    for (int64_t j = 0; j < nnz; j++) p->At.rp[col[j] + 1]++;
    for (int64_t d = 0; d < D; d++) p->At.rp[d + 1] += p->At.rp[d];
    p->At.col.resize(nnz);
    p->At.val.resize(nnz);
    std::vector<int64_t> fill(p->At.rp.begin(), p->At.rp.end() - 1);
    for (int64_t v = 0; v < V; v++)
      for (int64_t j = rowptr[v]; j < rowptr[v + 1]; j++) {
        const int64_t at = fill[col[j]]++;
        p->At.col[at] = (int32_t)v;
        p->At.val[at] = val[j];
      }
  } else {
    p->dense.resize((size_t)V * D);
    for (int64_t i = 0; i < V * D; i++) {
      if (!(val[i] >= 0.0f) || std::isinf(val[i])) {
        delete p;
        return -5;
      }
      p->dense[i] = val[i];
      a2 += (double)val[i] * val[i];
    }
  }
  if (!(a2 > 0.0)) {
    delete p;
    return -5;
  }
  p->a2 = a2;
  p->R.resize((size_t)D * K);
  p->P.resize((size_t)V * K);
  p->S.resize((size_t)K * K);
  p->Q.resize((size_t)K * K);
  p->old.resize((size_t)std::max(V, D) * K);
  p->gpart.resize((size_t)kChunks * K * K);
  // W's columns to unit norm (the initialisation reading shared with the GPU library)
  for (int k = 0; k < K; k++) {
    double s = 0.0;
    for (int64_t v = 0; v < V; v++) s += W[v * K + k] * W[v * K + k];
    if (!(s > 0.0) || !std::isfinite(s)) {
      delete p;
      return -5;
    }
    const double n = std::sqrt(s);
    for (int64_t v = 0; v < V; v++) W[v * K + k] /= n;
  }
  *out = p;
  return 0;
}

int nmf_cpu_sweep(nmf_cpu_plan p, int n_sweeps, double* rel_obj) {
  if (!p || n_sweeps < 0) return -1;
  for (int i = 0; i < n_sweeps; i++) {
    sweep(p);
    if (rel_obj) {
      rel_obj[i] = rel_objective(p);
      if (!std::isfinite(rel_obj[i])) return -5;
    }
  }
  return 0;
}

int nmf_cpu_info(nmf_cpu_plan p, int* tile, int* threads) {
  if (!p) return -1;
  if (tile) *tile = p->T;
  if (threads) *threads = p->threads;
  return 0;
}

int nmf_cpu_destroy(nmf_cpu_plan p) {
  delete p;
  return 0;
}

}  // extern "C"
