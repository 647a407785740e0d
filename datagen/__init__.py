"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and assembles input arrays; it holds
none of the factorisation's arithmetic.  Both the FP64 oracle tests and the
GPU path (tests, bench) take their inputs from here, so the two sides start
from bit-identical FP32 data.

The paper's corpora (Sec. 6.2, Table 4: 20 Newsgroups, TDT2, Reuters, AT&T,
PIE) are not available; these generators stand in for their shapes and
statistics and reproduce none of their content.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) and draws in
the order written in its docstring.  Values are produced in float64 and
rounded to float32 once.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "Csr",
    "BowCorpus",
    "dense_planted_uniform",
    "dense_planted_halfnormal",
    "uniform_init",
    "uniform_init_matched",
    "mean_value",
    "bag_of_words",
    "bag_of_words_docs",
    "planted_separable",
    "c0",
    "c1",
    "c2",
    "c3_docs",
    "c4",
]


@dataclass
class Csr:
    """Compressed sparse rows: ``rowptr`` [rows+1], ``col`` [nnz], ``val`` [nnz]."""

    rows: int
    cols: int
    rowptr: np.ndarray  # int32
    col: np.ndarray  # int32, strictly increasing within a row
    val: np.ndarray  # float32

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_dense(self, dtype=np.float32) -> np.ndarray:
        out = np.zeros((self.rows, self.cols), dtype=dtype)
        for r in range(self.rows):
            a, b = self.rowptr[r], self.rowptr[r + 1]
            out[r, self.col[a:b]] = self.val[a:b]
        return out

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.rows, self.cols))

    def transpose(self) -> "Csr":
        """Row-sorted CSR of the transpose (pure index bookkeeping)."""
        m = self.to_scipy().T.tocsr()
        m.sort_indices()
        return Csr(self.cols, self.rows, m.indptr.astype(np.int32), m.indices.astype(np.int32),
                   m.data.astype(np.float32))


@dataclass
class BowCorpus:
    """Term-by-document matrix A (V terms x D docs) in both CSR orientations."""

    A: Csr  # V rows (terms), column index = document
    At: Csr  # D rows (documents), column index = term
    perm: np.ndarray  # popularity rank -> term id
    idf: np.ndarray  # float64 [V]


# ---------------------------------------------------------------- dense ----

def dense_planted_uniform(V: int, D: int, K0: int, sigma: float, seed: int) -> np.ndarray:
    """A = W0 H0 + |N(0, sigma)|, W0, H0 ~ U[0,1).  Draw order: W0, H0, noise."""
    rng = np.random.default_rng(seed)
    W0 = rng.random((V, K0))
    H0 = rng.random((K0, D))
    noise = np.abs(rng.normal(0.0, sigma, (V, D)))
    return (W0 @ H0 + noise).astype(np.float32)


def dense_planted_halfnormal(V: int, D: int, K0: int, noise_hi: float, seed: int) -> np.ndarray:
    """A = W0 H0 + U[0, noise_hi), W0, H0 ~ |N(0,1)|.  Draw order: W0, H0, noise."""
    rng = np.random.default_rng(seed)
    W0 = np.abs(rng.normal(size=(V, K0)))
    H0 = np.abs(rng.normal(size=(K0, D)))
    A = W0 @ H0
    del W0, H0
    A += noise_hi * rng.random((V, D))
    return A.astype(np.float32)


def uniform_init(V: int, D: int, K: int, seed: int = 1):
    """Initial factors W [V,K] then H [K,D], both U[0,1), rounded to FP32.

    Returns ``(W, H)`` with H in the paper's K x D orientation.
    """
    rng = np.random.default_rng(seed)
    W = rng.random((V, K)).astype(np.float32)
    H = rng.random((K, D)).astype(np.float32)
    return W, H


def mean_value(A) -> float:
    """Mean entry of A (dense ndarray or Csr), zeros included."""
    if isinstance(A, Csr):
        return float(np.sum(A.val, dtype=np.float64)) / (A.rows * A.cols)
    return float(np.mean(A, dtype=np.float64))


def uniform_init_matched(V: int, D: int, K: int, a_mean: float, seed: int = 1):
    """``uniform_init`` with H scaled so that the initial product matches the
    data's mean entry in expectation: once W's U[0,1) columns are scaled to unit
    norm (each by about sqrt(V/3)), E[(W H)_vd] = (K/4) h / sqrt(V/3), so
    H ~ U[0,1) * h with h = a_mean * sqrt(V/3) / (K/4).  Same draws as
    ``uniform_init``; the scale is applied in float64 before the FP32 rounding."""
    rng = np.random.default_rng(seed)
    W = rng.random((V, K))
    H = rng.random((K, D))
    h = a_mean * np.sqrt(V / 3.0) / (0.25 * K)
    return W.astype(np.float32), (H * h).astype(np.float32)


def planted_separable(V: int, D: int, K: int, seed: int, scale_lo: float = 0.5):
    """Noise-free planted A = W0 H0 whose W0 and H0 each contain a scaled
    K x K identity block (separable, so the factorisation is unique up to
    permutation and scale).  Draw order: W0 rest, H0 rest, the two diagonal
    scales.  Returns ``(A, W0, H0)`` in float64."""
    rng = np.random.default_rng(seed)
    W0 = rng.random((V, K))
    H0 = rng.random((K, D))
    sw = scale_lo + rng.random(K)
    sh = scale_lo + rng.random(K)
    W0[:K, :] = np.diag(sw)
    H0[:, :K] = np.diag(sh)
    return W0 @ H0, W0, H0


# -------------------------------------------------------- bag of words ----

def _zipf_cdf(V: int, s: float) -> np.ndarray:
    r = np.arange(1, V + 1, dtype=np.float64)
    p = r ** (-s)
    return np.cumsum(p / p.sum())


def _draw_docs(rng, cdf: np.ndarray, n_terms: np.ndarray, perm: np.ndarray):
    """Per document, the first ``n`` distinct ranks of weighted draws with
    replacement (equivalent to weighted sampling without replacement), drawn in
    batches of 2n+16 uniforms.  Returns (doc_ptr, term ids) unsorted per doc."""
    V = cdf.shape[0]
    mark = np.zeros(V, dtype=bool)
    ptr = np.zeros(len(n_terms) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(n_terms)
    out = np.empty(int(ptr[-1]), dtype=np.int64)
    total = cdf[-1]
    for j, need in enumerate(n_terms):
        need = int(need)
        got = 0
        base = int(ptr[j])
        while got < need:
            u = rng.random(2 * need + 16)
            idx = np.searchsorted(cdf, u * total, side="right")
            idx = np.minimum(idx, V - 1)
            _, first = np.unique(idx, return_index=True)
            cand = idx[np.sort(first)]
            cand = cand[~mark[cand]]
            take = cand[: need - got]
            mark[take] = True
            out[base + got: base + got + take.size] = take
            got += take.size
        mark[out[base: base + need]] = False
    return ptr, perm[out]


def _assemble(D: int, V: int, ptr, terms, counts, idf) -> Csr:
    """Doc-major CSR (rows = docs) of tf-idf values, each doc L2-normalised."""
    rowptr = ptr.astype(np.int64)
    col = np.empty_like(terms)
    val = np.empty(terms.shape[0], dtype=np.float64)
    for j in range(D):
        a, b = rowptr[j], rowptr[j + 1]
        order = np.argsort(terms[a:b], kind="stable")
        t = terms[a:b][order]
        c = counts[a:b][order]
        x = c * idf[t]
        x = x / np.sqrt(np.sum(x * x))
        col[a:b] = t
        val[a:b] = x
    return Csr(D, V, rowptr.astype(np.int32), col.astype(np.int32), val.astype(np.float32))


def bag_of_words(V: int, D: int, zipf_s: float, mean_len: float, seed: int,
                 count_lam: float = 2.0) -> BowCorpus:
    """Sparse term-by-document matrix shaped like a bag-of-words corpus.

    Draw order: term permutation (popularity rank -> term id); per-document
    lengths n_j = 1 + Poisson(mean_len); per document in order, distinct terms
    with probability proportional to rank^-zipf_s; counts 1 + Poisson(count_lam)
    for every (doc, term) pair in generation order.  Value = count * idf with the
    smooth idf ln((1+D)/(1+df)) + 1, then every document (column of A) is scaled
    to unit L2 norm; FP32.
    """
    rng = np.random.default_rng(seed)
    perm = rng.permutation(V)
    cdf = _zipf_cdf(V, zipf_s)
    n = np.minimum(1 + rng.poisson(mean_len, size=D), V)
    ptr, terms = _draw_docs(rng, cdf, n, perm)
    counts = 1 + rng.poisson(count_lam, size=terms.shape[0])
    df = np.bincount(terms, minlength=V)
    idf = np.log((1.0 + D) / (1.0 + df)) + 1.0
    At = _assemble(D, V, ptr, terms, counts.astype(np.float64), idf)
    return BowCorpus(At.transpose(), At, perm, idf)


def bag_of_words_docs(D: int, zipf_s: float, mean_len: float, seed: int, perm: np.ndarray,
                      idf: np.ndarray, count_lam: float = 2.0) -> Csr:
    """New documents drawn by the same process as an existing corpus (its term
    permutation and idf vector).  Draw order: lengths, terms, counts.  Returns
    the doc-major CSR (D rows, V columns)."""
    V = perm.shape[0]
    rng = np.random.default_rng(seed)
    cdf = _zipf_cdf(V, zipf_s)
    n = np.minimum(1 + rng.poisson(mean_len, size=D), V)
    ptr, terms = _draw_docs(rng, cdf, n, perm)
    counts = 1 + rng.poisson(count_lam, size=terms.shape[0])
    return _assemble(D, V, ptr, terms, counts.astype(np.float64), idf)


# ------------------------------------------------------- named recipes ----

def c0():
    """Dense planted problem: 1000 x 800, rank 16, |N(0,0.01)| noise, seed 0."""
    return dense_planted_uniform(1000, 800, 16, 0.01, seed=0)


def c1(V: int = 26000, D: int = 11000, seed: int = 2) -> BowCorpus:
    """Bag-of-words stand-in for 20 Newsgroups / TDT2 / Reuters (about 0.3% dense)."""
    return bag_of_words(V, D, 1.1, 77.0, seed)


def c2(V: int = 10000, D: int = 10000, seed: int = 0) -> np.ndarray:
    """Dense image-shaped stand-in for PIE / AT&T: rank-300 planted + U[0,0.05)."""
    return dense_planted_halfnormal(V, D, 300, 0.05, seed)


def c3_docs(corpus: BowCorpus, D: int = 200000, seed: int = 3) -> Csr:
    """New documents for fold-in, drawn like ``c1`` with its permutation and idf."""
    return bag_of_words_docs(D, 1.1, 77.0, seed, corpus.perm, corpus.idf)


def c4(V: int = 100000, D: int = 300000, seed: int = 5) -> BowCorpus:
    """Large bag-of-words matrix, Zipf 1.05, about 0.1% dense (about 3e7 nnz)."""
    return bag_of_words(V, D, 1.05, 99.0, seed)
