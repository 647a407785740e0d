"""Pins of the Sec. 5 data-movement model against the paper's printed numbers
(fixture: tests/golden/sec5_model.json)."""
import json
import math
import os

import numpy as np

from oracle import tile_model as tm

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sec5_model.json")))


def test_worked_example_volumes():
    ex = GOLD["worked_example"]
    C = ex["cache_mib"] * 2 ** 20 / 8
    assert tm.original_w_volume(ex["V"], ex["K"]) == ex["original_words"]
    vol = tm.tiled_w_volume(ex["V"], ex["K"], ex["T"], C)
    assert math.floor(vol) == ex["tiled_words"]
    assert round(ex["original_words"] / vol, 1) == ex["ratio_printed"]


def test_printed_tile_sizes():
    ts = GOLD["tile_sizes"]
    C = ts["cache_mib"] * 2 ** 20 / 8
    for K, T in zip(ts["K"], ts["T_printed"]):
        assert math.floor(tm.tile_size_printed(K, C) * 100) / 100 == T


def test_stationary_point_minimises_eq9():
    """Eq. 10's root is the minimiser of Eq. 9 over real T (brute force grid)."""
    C = tm.CACHE_35MIB_WORDS
    for K in (80, 160, 240):
        grid = np.linspace(1.0, K, 400001)
        vols = tm.tiled_w_volume(11314, K, grid, C)
        t_best = grid[np.argmin(vols)]
        assert abs(t_best - tm.tile_size_stationary(K, C)) < 2e-3
