"""Host logic of bench.py: the algorithmic flop and byte model per band pair
(against the per-configuration figures derived independently from the
method: F = 10 N log2 N + 16 N, B = 4 s N), the roofline choice, and the
kernel-rate table."""
import math
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


@pytest.mark.parametrize("L,flops_m,bytes_mb32", [(16, 0.56, 0.13), (32, 5.44, 1.05), (64, 51.4, 8.39), (72, 75.06, 11.94)])
def test_apply_model_per_pair(L, flops_m, bytes_mb32):
    m = bench.kernel_model((L, L, L), 8)
    # the reference figures carry 2-4 significant digits
    assert m["fused"]["flops"] / 1e6 == pytest.approx(flops_m, rel=1e-2)
    assert m["fused"]["bytes"] / 1e6 == pytest.approx(bytes_mb32, rel=1e-2)
    # the three-pass split adds up to the same flops
    split = m["plane"]["flops"] + m["pencil"]["flops"] + m["accumulate"]["flops"]
    assert split == pytest.approx(m["fused"]["flops"], rel=1e-12)
    # the energy path is the forward half
    n = L ** 3
    assert m["energy_fused"]["flops"] == pytest.approx(5 * n * math.log2(n) + 9 * n)


def test_roofline_picks_dominant_kernel_and_bound():
    stats = {"apply_fft_pairs": 1_000_000, "energy_fft_pairs": 500_000}
    kern = {"fused": (200.0, 2), "energy_fused": (20.0, 1), "overlap": (1.0, 1)}
    r = bench.roofline(kern, stats, (32, 32, 32), 8, 78.6)
    assert r["kernel"] == "fused" and r["launches"] == 2
    per_launch_s = 0.1
    gbs = 4 * 8 * 32768 * 1e6 / per_launch_s / 1e9
    tfl = (10 * 32768 * 15 + 16 * 32768) * 1e6 / per_launch_s / 1e12
    assert r["alt"]["hbm_gbs"] == pytest.approx(gbs, rel=1e-3)
    assert r["alt"]["alu_tflops"] == pytest.approx(tfl, rel=1e-3)
    assert r["bound"] == ("hbm" if gbs / 8000 >= tfl / 78.6 else "alu")
    rates = bench.kernel_rates(kern, stats, (32, 32, 32), 8)
    assert set(rates) == {"fused", "energy_fused"}
    assert rates["fused"]["gbs"] == pytest.approx(gbs, rel=1e-3)  # two launches of the same size
