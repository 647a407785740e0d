"""Data-movement model of Sec. 5 (test infrastructure only; model, not a kernel).

Volumes are counted in words moved between main memory and a cache of C words.

Readings:
* C is the cache capacity in 8-byte words (the paper's numbers are FP64): a
  35 MiB cache is C = 35 * 2**20 / 8 words.  This reproduces both printed
  volumes of Sec. 5 (the tiled one as the floor of Eq. 9).
* The printed tile sizes (Sec. 5) are Eq. 11 as printed, sqrt(K - 2/sqrt(C)),
  truncated to two decimals.  Setting the printed derivative (Eq. 10) to zero
  instead gives T = sqrt(K / (1 - 2/sqrt(C))), the exact minimiser of Eq. 9
  over real T; both are close to sqrt(K).
"""
from __future__ import annotations

import math

CACHE_35MIB_WORDS = 35 * 2 ** 20 / 8


def original_w_volume(V, K):
    """Data movement of the untiled W loop of Alg. 1: K (V K + K + 6 V + 1) (Sec. 3.2)."""
    return K * (V * K + K + 6 * V + 1)


def tiled_w_volume(V, K, T, C):
    """Eq. 9: vol(T) = V (1/T + 2/sqrt(C)) (K^2 - K T) + (K/T) T (V T)."""
    return V * (1.0 / T + 2.0 / math.sqrt(C)) * (K * K - K * T) + (K / T) * T * (V * T)


def tile_size_printed(K, C):
    """Eq. 11 as printed: T = sqrt(K - 2/sqrt(C))."""
    return math.sqrt(K - 2.0 / math.sqrt(C))


def tile_size_stationary(K, C):
    """Root of Eq. 10, T^2 (2/sqrt(C) - 1) + K = 0, i.e. T = sqrt(K / (1 - 2/sqrt(C)))."""
    return math.sqrt(K / (1.0 - 2.0 / math.sqrt(C)))
