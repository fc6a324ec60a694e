"""The device FMA-rate probe the evaluation's efficiency is quoted against."""
import pytest

from paper_2006_02501_amd import fma_rate

pytestmark = pytest.mark.gpu

# one FMA per lane per clock: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
PUBLISHED_LANE_FMA_FP64 = 78.6e12 / 2


def test_fma_rate_within_published_peak():
    r64 = fma_rate("fp64")
    r32 = fma_rate("fp32")
    assert 0.5 * PUBLISHED_LANE_FMA_FP64 <= r64 <= 1.05 * PUBLISHED_LANE_FMA_FP64, r64
    # the two-operand FP32 form may issue above one per lane per clock
    assert 0.5 * PUBLISHED_LANE_FMA_FP64 <= r32 <= 2.1 * PUBLISHED_LANE_FMA_FP64, r32
