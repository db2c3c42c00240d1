"""GPU test of the launch-configuration autotuner: it picks one of its candidates, does
not touch the caller's mixtures, caches its choice, and the tuned fit stays within the
parity tolerance of the oracle."""
import numpy as np
import pytest

from paper_2111_13094_amd import synth
from tests.parity_utils import assert_cells_close, positive_counts, state_to_torch, to_numpy, to_torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_13094_amd import sdmm
    sdmm.lib()
    return torch


def test_tuner_picks_a_candidate_and_keeps_parity(dev, orc):
    print("case: autotuner on 64 cells", flush=True)
    from paper_2111_13094_amd import sdmm, tune
    torch = dev
    wl = synth.workload("cells4k", scale=64 / 4096, seed=21)
    C = wl["grid"].n_cells
    b = synth.workload_batch(wl)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    off, smp = torch.from_numpy(b.offsets).cuda(), torch.from_numpy(b.samples).cuda()
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
    before = {k: v.clone() for k, v in gm.items()}
    opts = sdmm.default_opts(16, eta=0.1)
    cands = tune.DEFAULT_CANDIDATES[:4] + tune.FUSED_CANDIDATES[:1]
    assert all(c["schedule"] == sdmm.SCHED_BATCHED for c in tune.DEFAULT_CANDIDATES)
    tuned = tune.tune_fit(off, smp, gm, gst, opts, candidates=cands, reps=2)
    for k in gm:
        assert torch.equal(gm[k], before[k])
    chosen = {"schedule": tuned.schedule, "min_range": tuned.min_range, "waves_per_block": tuned.waves_per_block}
    assert chosen in cands
    cached = tune.tuned_config(C, 16, smp.shape[1], opts)
    assert cached is not None and cached["ms"] > 0
    again = tune.tune_fit(off, smp, gm, gst, opts, candidates=[cands[-1]])  # served from the cache
    assert again.min_range == tuned.min_range and again.schedule == tuned.schedule
    status = sdmm.fit_mixtures(off, smp, gm, gst, tuned)
    om, ost = synth.copy_mix(mix0), orc.new_state(C, 16)
    s_o = orc.fit(orc.Opts(K=16, eta=0.1), b.offsets, b.samples, om, ost)
    assert (status.cpu().numpy() == s_o).all()
    print(chosen)
    assert_cells_close(to_numpy(gm), om, 16, range(C), positive_counts(b.samples, b.offsets), what="tuned fit")
