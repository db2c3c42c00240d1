"""Precision study on the huge workload (one cell, 2^24 samples, K = 32, weights
lognormal(0, 2.5) with no zeros: the largest weight is ~e^13 times the median), one E+M
step from the initial mixture, every running-sum variant of the E-step against the
FP64 oracle. The E-step forms products in FP32 in every variant; what differs is how
the per-lane running sums are kept:

  twosum  FP32 block sums folded every 64 steps by TwoSum into an FP32 running sum, the
          rounding error of each fold opening the next block (compensated)
  plain   one FP32 running sum per lane
  fp64    FP32 block sums folded into an FP64 running sum

and over how many samples a lane sums before the FP64 reduction across work items
(the default work item of 256 samples, or the whole cell as one item). Errors are the
parity metrics of tests/parity_utils.py (relative for pi, mu_pos and Sigma in the
oracle covariance's metric, radians for mu_dir)."""
import numpy as np
import pytest

from paper_2111_13094_amd import synth
from tests.parity_utils import compare_mixtures, state_to_torch, to_numpy, to_torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_13094_amd import sdmm
    sdmm.lib()
    return torch


def test_precision_variants_on_the_huge_cell(dev, orc):
    print("case: huge cell, 2^24 samples, K=32, oracle step (about a minute on one core)", flush=True)
    from paper_2111_13094_amd import sdmm
    torch = dev
    wl = synth.workload("huge")
    b = synth.workload_batch(wl)
    K = 32
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)
    om, ost = synth.copy_mix(mix0), orc.new_state(1, K)
    s_o = orc.fit(orc.Opts(K=K), b.offsets, b.samples, om, ost)
    print("oracle status", s_o, flush=True)
    off, smp = torch.from_numpy(b.offsets).cuda(), torch.from_numpy(b.samples).cuda()
    one_item = 1 << 24
    variants = {
        "twosum, default items": dict(),
        "fp64, default items": dict(flags=sdmm.FLAG_FP64_SUMS),
        "plain, default items": dict(flags=sdmm.FLAG_PLAIN_FP32),
        "twosum, one item": dict(min_range=one_item),
        "plain, one item": dict(min_range=one_item, flags=sdmm.FLAG_PLAIN_FP32),
    }
    res = {}
    for name, kw in variants.items():
        gm, gst = to_torch(mix0), state_to_torch(orc.new_state(1, K))
        st = sdmm.fit_mixtures(off, smp, gm, gst, sdmm.default_opts(K, **kw))
        torch.cuda.synchronize()
        assert (st.cpu().numpy() == s_o).all(), (name, st, s_o)
        res[name] = compare_mixtures(to_numpy(gm), om, K)
    print("\nvariant                     pi        mu_dir    mu_pos    Sigma")
    for name, w in res.items():
        print(f"{name:26s} {w['pi']:.2e}  {w['mu_dir']:.2e}  {w['mu_pos']:.2e}  {w['cov']:.2e}")

    def worst(w):
        return max(w["pi"], w["mu_pos"], w["cov"], 10 * w["mu_dir"])
    for name in ("twosum, default items", "fp64, default items", "twosum, one item"):
        assert worst(res[name]) < 1e-4, (name, res[name])
    # compensation is what keeps a lane's long sum exact: without it the one-item sums drift
    assert worst(res["plain, one item"]) > 3 * worst(res["twosum, one item"])
