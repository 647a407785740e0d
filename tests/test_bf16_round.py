"""The test-side BF16 rounding helper against hand-computed cases (CPU)."""
import numpy as np

from tests.gpu_util import bf16_round


def test_bf16_round_cases():
    # 1 + 2^-8 is exactly halfway between bf16 1.0 and 1 + 2^-7: ties to even -> 1.0
    assert bf16_round(np.float32(1.0 + 2.0 ** -8)) == 1.0
    # 1 + 3*2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even -> 1 + 2^-6
    assert bf16_round(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6
    assert bf16_round(np.float32(1.0 + 2.0 ** -8 + 2.0 ** -20)) == 1.0 + 2.0 ** -7
    x = np.random.default_rng(0).normal(size=1000).astype(np.float32)
    r = bf16_round(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)
    assert np.all(r.astype(np.float32).view(np.uint32) & 0xFFFF == 0)
