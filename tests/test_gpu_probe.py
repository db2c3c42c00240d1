"""The FMA-rate microbenchmark behind the bench line's measured ceiling: FP32 without
packed instructions and FP64 both land between a quarter of and just above the rate the
published peaks give for one FMA per lane and cycle (78.6 TFLOP/s: 256 CUs x 4 SIMDs x
16 lanes x 2 flop x 2.4 GHz)."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_13094_amd import sdmm
    sdmm.lib()
    return torch


@pytest.mark.parametrize("bits", [32, 64])
def test_fma_probe_rate(dev, bits):
    print(f"case: FMA probe, FP{bits}", flush=True)
    from paper_2111_13094_amd import sdmm
    sdmm.probe_fma(bits, n_groups=1024, iters=64)
    rate = max(sdmm.probe_fma(bits) for _ in range(2))
    print("FP%d FMA rate %.1f TFLOP/s" % (bits, rate))
    assert 0.25 * 78.6 < rate < 1.05 * 78.6
