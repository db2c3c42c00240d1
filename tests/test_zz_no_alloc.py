"""sdmm_fit_mixtures_noalloc (through the C ABI) against sdmm_fit_mixtures: the same
kernels on the library's static per-device workspace instead of the caller's, so the
results are bitwise equal. Two calls in a row, the second on a smaller batch, so that
the second runs on an array that still holds the first call's contents."""
import numpy as np
import pytest

from paper_2111_13094_amd import synth
from tests.parity_utils import assert_close, compare_mixtures, state_to_torch, to_numpy, to_torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_13094_amd import sdmm
    sdmm.lib()
    return torch


def _case(n_cells, seed):
    wl = synth.workload("cells4k", scale=n_cells / 4096, seed=seed)
    return wl, synth.workload_batch(wl), synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)


def test_noalloc_equals_fit_mixtures_on_two_calls(dev, orc):
    print("case: no-alloc fit vs fit_mixtures, 125 cells then 27 cells", flush=True)
    from paper_2111_13094_amd import sdmm
    for call, (n_cells, seed) in enumerate(((125, 5), (27, 6))):
        wl, b, mix0 = _case(n_cells, seed)
        C = wl["grid"].n_cells
        off, smp = dev.from_numpy(b.offsets).cuda(), dev.from_numpy(b.samples).cuda()
        o = sdmm.default_opts(16, iters=2, eta=0.1)
        gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
        s_ref = sdmm.fit_mixtures(off, smp, gm, gst, o)
        nm, nst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
        status = dev.full((C,), -7, dtype=dev.int32, device="cuda")
        sdmm.fit_mixtures_noalloc(off, smp, nm, nst, o, status)
        dev.cuda.synchronize()
        assert dev.equal(status, s_ref), call
        for k in gm:
            assert dev.equal(nm[k], gm[k]), (call, k)
        for k in gst:
            assert dev.equal(nst[k], gst[k]), (call, k)
        # and the oracle's bar on the no-alloc result
        om, ost = synth.copy_mix(mix0), orc.new_state(C, 16)
        s_o = orc.fit(orc.Opts(K=16, iters=2, eta=0.1), b.offsets, b.samples, om, ost)
        assert (status.cpu().numpy() == s_o).all()
        fitted = [c for c in range(C) if not s_o[c] & (1 | 2 | 4 | 32)]
        worst = compare_mixtures(to_numpy(nm), om, 16, cells=fitted)
        print(call, C, worst)
        assert_close(worst, what=f"no-alloc call {call}")


def test_noalloc_rejects_what_it_cannot_hold(dev, orc):
    """A batch whose workspace exceeds the static array is refused with
    ENOWORKSPACE before anything is enqueued; the per-cell schedule and the graph
    cache are refused with EINVAL."""
    from paper_2111_13094_amd import sdmm
    wl, b, mix0 = _case(27, 7)
    C = wl["grid"].n_cells
    off, smp = dev.from_numpy(b.offsets).cuda(), dev.from_numpy(b.samples).cuda()
    status = dev.zeros(C, dtype=dev.int32, device="cuda")
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
    for kw, msg in ((dict(schedule=sdmm.SCHED_PER_CELL), "invalid argument"), (dict(use_graph=1), "invalid argument"),
                    (dict(min_range=16, max_ranges=1 << 20), None)):
        o = sdmm.default_opts(16, **kw)
        if msg is None:
            # tiny items: more records than the array holds for this batch size
            big = sdmm.workspace_bytes(C, 16, 1 << 22, o)
            assert big > sdmm.NOALLOC_SCRATCH_BYTES
            fake = dev.zeros(7, 1 << 22, dtype=dev.float32, device="cuda")
            with pytest.raises(RuntimeError, match="workspace too small"):
                sdmm.fit_mixtures_noalloc(off, fake, gm, gst, o, status)
        else:
            with pytest.raises(RuntimeError, match=msg):
                sdmm.fit_mixtures_noalloc(off, smp, gm, gst, o, status)
    dev.cuda.synchronize()
    for k, v in to_numpy(gm).items():
        assert np.array_equal(v, mix0[k]), k
