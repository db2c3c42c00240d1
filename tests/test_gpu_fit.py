"""GPU parity of sdmm_fit_mixtures (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest

from paper_2111_13094_amd import synth
from tests.parity_utils import (assert_cells_close, assert_close, compare_mixtures, positive_counts, state_to_torch,
                                to_numpy, to_torch)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_13094_amd import sdmm
    sdmm.lib()
    return torch


def _gpu_fit(dev, batch, mix, state, **opt):
    from paper_2111_13094_amd import sdmm
    K = opt.pop("K", 16)
    o = sdmm.default_opts(K, **opt)
    off = dev.from_numpy(batch.offsets).cuda()
    smp = dev.from_numpy(batch.samples).cuda()
    status = sdmm.fit_mixtures(off, smp, mix, state, o)
    dev.cuda.synchronize()
    return status.cpu().numpy()


def _orc_opts(orc, K=16, **kw):
    return orc.Opts(K=K, **kw)


def _single(n=16384, seed=1234):
    wl = synth.workload("single", seed=seed)
    b = synth.make_batch(seed + 5, [n], wl["box_lo"], wl["box_size"], wl["lobes"], parallax=True)
    return wl, b


def test_single_cell_one_step_parity(dev, orc):
    print("case: single cell N=16384 K=16, one E+M step", flush=True)
    wl, b = _single()
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    om, ost = synth.copy_mix(mix0), orc.new_state(1, 16)
    s_o = orc.fit(_orc_opts(orc), b.offsets, b.samples, om, ost)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(1, 16))
    s_g = _gpu_fit(dev, b, gm, gst)
    assert (s_g == s_o).all(), (s_g, s_o)
    worst = compare_mixtures(to_numpy(gm), om, 16)
    print(worst)
    assert_close(worst, what="one step")
    g = to_numpy(gst)
    assert g["step"][0] == ost["step"][0] == 1
    assert abs(g["sw"][0] - ost["sw"][0]) <= 1e-6 * ost["sw"][0]
    assert np.allclose(g["s0"], ost["s0"], rtol=1e-4, atol=1e-9 * ost["sw"][0])


def test_single_cell_twenty_iterations(dev, orc):
    print("case: single cell N=16384 K=16, 20 iterations", flush=True)
    wl, b = _single(seed=99)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    om, ost = synth.copy_mix(mix0), orc.new_state(1, 16)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(1, 16))
    worst_all = []
    for it in range(20):
        orc.fit(_orc_opts(orc), b.offsets, b.samples, om, ost)
        _gpu_fit(dev, b, gm, gst)
        w = compare_mixtures(to_numpy(gm), om, 16)
        worst_all.append(max(w["pi"], w["mu_pos"], w["cov"], w["mu_dir"] * 10))
    print("per-iteration worst:", ["%.1e" % v for v in worst_all])
    assert max(worst_all) < 1e-3
    # the same 20 iterations as one call
    gm2, gst2 = to_torch(mix0), state_to_torch(orc.new_state(1, 16))
    _gpu_fit(dev, b, gm2, gst2, iters=20)
    for k in gm:
        assert dev.equal(gm[k], gm2[k]), k


def _ragged_case():
    wl = synth.workload("cells4k", scale=64 / 4096)
    C = wl["grid"].n_cells
    counts = wl["counts"].copy()
    counts[0] = 0          # empty
    counts[1] = 7          # too few
    counts[2] = 16         # exactly the minimum
    counts[3] = 20000      # several work items
    counts[4] = 65         # one more than a 64-sample multiple
    b = synth.make_batch(77, counts, wl["box_lo"], wl["box_size"], wl["lobes"])
    off = b.offsets
    smp = b.samples
    smp[6, off[2]:off[3]] = np.abs(smp[6, off[2]:off[3]]) + 0.5  # all positive
    smp[0, off[5] + 2] = np.nan                                  # bad input
    smp[6, off[6] + 1] = -2.0                                    # negative weight
    smp[6, off[7]:off[8]] = 0.0                                  # zero weights
    smp[3, off[9] + 4] = np.inf                                  # infinite position
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    cov = mix["cov"].reshape(C, 16, 15)
    cov[10, 5, 0] = -1.0                                         # non-SPD parameters
    mix["pi"].reshape(C, 16)[11, 3] = np.nan                     # non-finite weight
    return wl, b, mix


def test_ragged_cells_statuses_and_isolation(dev, orc):
    print("case: 64 ragged cells with gated / bad cells", flush=True)
    wl, b, mix0 = _ragged_case()
    C = wl["grid"].n_cells
    om, ost = synth.copy_mix(mix0), orc.new_state(C, 16)
    s_o = orc.fit(_orc_opts(orc, iters=2), b.offsets, b.samples, om, ost)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
    s_g = _gpu_fit(dev, b, gm, gst, iters=2)
    assert (s_g == s_o).all(), np.nonzero(s_g != s_o)
    assert s_o[0] == orc.SKIPPED_FEW and s_o[1] == orc.SKIPPED_FEW
    assert s_o[5] == orc.BAD_INPUT and s_o[6] == orc.BAD_INPUT and s_o[9] == orc.BAD_INPUT
    assert s_o[7] == orc.SKIPPED_FEW
    assert s_o[10] == orc.BAD_PARAMS and s_o[11] == orc.BAD_PARAMS
    got = to_numpy(gm)
    skipped = [c for c in range(C) if s_o[c] & (1 | 2 | 4 | 32)]
    for c in skipped:  # untouched, bitwise
        for k in got:
            assert np.array_equal(got[k].reshape(C, -1)[c], mix0[k].reshape(C, -1)[c], equal_nan=True)
    fitted = [c for c in range(C) if c not in skipped]
    # cells with fewer than 64 positive weights (cell 2 has 16) take the small-cell bound
    # of the whitened covariance metric; every other measure is at 1e-4
    assert_cells_close(got, om, 16, fitted, positive_counts(b.samples, b.offsets), what="ragged")


def test_schedules_and_graph_are_bitwise_equal_and_deterministic(dev, orc):
    print("case: fused vs split vs per-cell vs graph replay, 64 cells", flush=True)
    from paper_2111_13094_amd import sdmm
    wl, b, mix0 = _ragged_case()
    C = wl["grid"].n_cells
    runs = []
    for sched, graph in ((sdmm.SCHED_BATCHED, 0), (sdmm.SCHED_BATCHED, 0), (sdmm.SCHED_PER_CELL, 0),
                         (sdmm.SCHED_FUSED, 0), (sdmm.SCHED_BATCHED, 1), (sdmm.SCHED_FUSED, 1)):
        gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
        s = _gpu_fit(dev, b, gm, gst, iters=2, schedule=sched, use_graph=graph)
        runs.append((to_numpy(gm), to_numpy(gst), s))
    for m, st, s in runs[1:]:
        assert (s == runs[0][2]).all()
        for k in m:
            assert np.array_equal(m[k], runs[0][0][k], equal_nan=True), k
        for k in st:
            assert np.array_equal(st[k], runs[0][1][k], equal_nan=True), k


def test_graph_replays_match_eager(dev, orc):
    print("case: repeated graph replays vs eager", flush=True)
    wl = synth.workload("cells4k", scale=27 / 4096)
    b = synth.workload_batch(wl)
    C = wl["grid"].n_cells
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    ge, gse = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
    gg, gsg = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
    for rep in range(4):
        _gpu_fit(dev, b, ge, gse, eta=0.1)
        _gpu_fit(dev, b, gg, gsg, eta=0.1, use_graph=1)
        for k in ge:
            assert dev.equal(ge[k], gg[k]), (rep, k)


def test_cell_independence_bitwise(dev, orc):
    print("case: cells fitted together vs alone", flush=True)
    wl = synth.workload("cells4k", scale=27 / 4096)
    b = synth.workload_batch(wl)
    C = wl["grid"].n_cells
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
    _gpu_fit(dev, b, gm, gst, iters=2)
    allm = to_numpy(gm)
    for c in (0, 5, C - 1):
        i0, i1 = b.offsets[c], b.offsets[c + 1]
        sub = synth.Batch(np.ascontiguousarray(b.samples[:, i0:i1]), np.array([0, i1 - i0]), b.lobe[i0:i1])
        mc = {k: np.ascontiguousarray(v.reshape(C, -1)[c]) for k, v in mix0.items()}
        g1, s1 = to_torch(mc), state_to_torch(orc.new_state(1, 16))
        _gpu_fit(dev, sub, g1, s1, iters=2)
        for k, v in to_numpy(g1).items():
            assert np.array_equal(v, allm[k].reshape(C, -1)[c]), (c, k)


def test_stepwise_batches_parity(dev, orc):
    print("case: 27 cells, 8 batches, eta = 0.1 (decay 0.9)", flush=True)
    wl = synth.workload("cells4k", scale=27 / 4096)
    C = wl["grid"].n_cells
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    om, ost = synth.copy_mix(mix0), orc.new_state(C, 16)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
    worst = []
    for j in range(8):
        b = synth.workload_batch(wl, j)
        orc.fit(_orc_opts(orc, eta=0.1), b.offsets, b.samples, om, ost)
        _gpu_fit(dev, b, gm, gst, eta=0.1)
        w = compare_mixtures(to_numpy(gm), om, 16)
        worst.append(max(w["pi"], w["mu_pos"], w["cov"], 10 * w["mu_dir"]))
    print("per-batch worst:", ["%.1e" % v for v in worst])
    assert max(worst) < 1e-3
    g = to_numpy(gst)
    assert (g["step"] == ost["step"]).all()


@pytest.mark.parametrize("K", [5, 12, 32])
def test_other_component_counts(dev, orc, K):
    print(f"case: single cell N=8192 K={K}", flush=True)
    wl, b = _single(n=8192, seed=7 + K)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)
    om, ost = synth.copy_mix(mix0), orc.new_state(1, K)
    orc.fit(_orc_opts(orc, K=K, iters=2), b.offsets, b.samples, om, ost)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(1, K))
    _gpu_fit(dev, b, gm, gst, K=K, iters=2)
    worst = compare_mixtures(to_numpy(gm), om, K)
    print(worst)
    assert_close(worst, what=f"K={K}")


@pytest.mark.parametrize("variant", ["plain", "fp64", "jacobian", "paper_eta", "fixed_prior"])
def test_option_variants(dev, orc, variant):
    print(f"case: option variant {variant}", flush=True)
    from paper_2111_13094_amd import sdmm
    wl, b = _single(n=8192, seed=31)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    gopt, oopt = {"iters": 2}, {"iters": 2}
    if variant == "plain":
        gopt["flags"] = sdmm.FLAG_PLAIN_FP32
    elif variant == "fp64":
        gopt["flags"] = sdmm.FLAG_FP64_SUMS
    elif variant == "jacobian":
        gopt["flags"] = sdmm.FLAG_ESTEP_JACOBIAN
        oopt["estep_jacobian"] = 1
    elif variant == "paper_eta":
        gopt.update(eta_mode=sdmm.ETA_PAPER)
        oopt.update(eta_mode=1)
    elif variant == "fixed_prior":
        gopt.update(prior_mode=sdmm.PRIOR_FIXED, prior_scale=0.25)
        oopt.update(prior_mode=1, prior_scale=0.25)
    om, ost = synth.copy_mix(mix0), orc.new_state(1, 16)
    orc.fit(_orc_opts(orc, **oopt), b.offsets, b.samples, om, ost)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(1, 16))
    _gpu_fit(dev, b, gm, gst, **gopt)
    worst = compare_mixtures(to_numpy(gm), om, 16)
    print(worst)
    assert_close(worst, what=variant)


@pytest.mark.parametrize("case", ["batched", "fused", "fixed_prior_zero"])
def test_zero_weight_component(dev, orc, case):
    """A usable component of weight exactly zero takes no responsibility (Sec. 3.2: r is
    proportional to pi_k p_k): its log constant is -inf on the device, never the cell's
    largest. Caller-supplied pi = 0 in two of 16 components, one E+M step in the batched
    and fused schedules; and three iterations with a fixed prior of strength 0, where
    those components stay dead with pi = 0 and the M-step's mirror refresh carries the
    zero weight into the next iteration."""
    print(f"case: zero-weight components, {case}", flush=True)
    from paper_2111_13094_amd import sdmm
    wl, b = _single(n=8192, seed=41)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    mix0["pi"][[3, 9]] = 0.0
    mix0["pi"] /= mix0["pi"].sum()
    gopt, oopt = {}, {}
    if case == "fused":
        gopt["schedule"] = sdmm.SCHED_FUSED
    if case == "fixed_prior_zero":
        gopt.update(prior_mode=sdmm.PRIOR_FIXED, prior_scale=0.0, iters=3)
        oopt.update(prior_mode=1, prior_scale=0.0, iters=3)
    om, ost = synth.copy_mix(mix0), orc.new_state(1, 16)
    s_o = orc.fit(_orc_opts(orc, **oopt), b.offsets, b.samples, om, ost)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(1, 16))
    s_g = _gpu_fit(dev, b, gm, gst, **gopt)
    assert (s_g == s_o).all(), (s_g, s_o)
    got = to_numpy(gm)
    g = to_numpy(gst)
    if case == "fixed_prior_zero":
        assert s_o[0] & orc.DEAD_COMPONENT
        assert (got["pi"][[3, 9]] == 0.0).all() and (om["pi"][[3, 9]] == 0.0).all()
        assert (g["s0"][[3, 9]] == 0.0).all()
    else:
        # one step: the zero-weight components gathered nothing
        assert (g["s0"][[3, 9]] == 0.0).all() and (ost["s0"][[3, 9]] == 0.0).all()
    worst = compare_mixtures(got, om, 16)
    print(worst)
    assert_close(worst, what=f"zero-weight components, {case}")


@pytest.mark.parametrize("split", [dict(min_range=64), dict(max_ranges=3), dict(min_range=1 << 20)])
def test_work_split_does_not_change_results(dev, orc, split):
    """One cell of 150000 samples cut into 2344 items of 64 samples, 3 items of 50000, or
    a single item: the records are summed in item order in FP64, so every split is
    within the same tolerance of the oracle."""
    print(f"case: one cell of 150000 samples, split {split}", flush=True)
    wl, b = _single(n=150000, seed=5)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    om, ost = synth.copy_mix(mix0), orc.new_state(1, 16)
    orc.fit(_orc_opts(orc), b.offsets, b.samples, om, ost)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(1, 16))
    _gpu_fit(dev, b, gm, gst, **split)
    worst = compare_mixtures(to_numpy(gm), om, 16)
    print(worst)
    assert_close(worst, what=f"split {split}")


def test_record_tree_schedules(dev, orc):
    """Cells with more than 128 work items have their records pre-summed in a 16-ary tree
    (two levels here: a 120000-sample cell in 64-sample items, 1875 items, next to small
    cells). The batched and per-cell schedules sum in the same order (bitwise equal);
    the fused schedule sums a cell's records in one pass (equal to rounding); all match
    the oracle."""
    print("case: record tree, 120000-sample cell in 64-sample items + 7 small cells", flush=True)
    from paper_2111_13094_amd import sdmm
    wl = synth.workload("single", seed=17)
    counts = [120000, 300, 0, 5000, 64, 2000, 17, 900]
    b = synth.make_batch(19, counts, np.tile(wl["box_lo"], (8, 1)), np.tile(wl["box_size"], (8, 1)), wl["lobes"])
    C = len(counts)
    lo, size = np.tile(wl["box_lo"], (C, 1)), np.tile(wl["box_size"], (C, 1))
    mix0 = synth.initial_mixtures(lo, size, 16)
    om, ost = synth.copy_mix(mix0), orc.new_state(C, 16)
    s_o = orc.fit(_orc_opts(orc, iters=2), b.offsets, b.samples, om, ost)
    runs = {}
    for name, sched in (("batched", sdmm.SCHED_BATCHED), ("per_cell", sdmm.SCHED_PER_CELL),
                        ("fused", sdmm.SCHED_FUSED)):
        gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
        st = _gpu_fit(dev, b, gm, gst, iters=2, schedule=sched, min_range=64, max_ranges=1 << 20)
        assert (st == s_o).all(), (name, st, s_o)
        runs[name] = to_numpy(gm)
    for k in runs["batched"]:
        assert np.array_equal(runs["batched"][k], runs["per_cell"][k]), k
    fitted = [c for c in range(C) if not s_o[c] & (1 | 2 | 4 | 32)]
    m_pos = positive_counts(b.samples, b.offsets)
    for name, got in runs.items():
        assert_cells_close(got, om, 16, fitted, m_pos, what=name)


def test_max_cell_samples_hint(dev, orc):
    """The caller's bound on samples per cell only sets how many record-tree levels are
    launched. An exact bound gives the same bits as no bound; a bound below the largest
    cell launches too few levels, and the M-step then sums the item records instead of
    the level leaders: the same result up to the FP32 rounding of the leader records
    (2^-24 relative per leader), held at a tenth of the parity bar."""
    print("case: max_cell_samples hint, 120000-sample cell in 64-sample items", flush=True)
    from paper_2111_13094_amd import sdmm
    wl = synth.workload("single", seed=17)
    counts = [120000, 300, 0, 5000, 64, 2000, 17, 900]
    b = synth.make_batch(19, counts, np.tile(wl["box_lo"], (8, 1)), np.tile(wl["box_size"], (8, 1)), wl["lobes"])
    C = len(counts)
    lo, size = np.tile(wl["box_lo"], (C, 1)), np.tile(wl["box_size"], (C, 1))
    mix0 = synth.initial_mixtures(lo, size, 16)
    runs, stats = {}, {}
    # 1875 items of 64 samples in the big cell need one level; a bound of 200000 launches
    # two (the second does nothing), one of 1000 launches none
    for name, hint in (("none", 0), ("exact", 120000), ("above", 200000), ("below", 1000)):
        for sched in (sdmm.SCHED_BATCHED, sdmm.SCHED_PER_CELL):
            gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
            stats[(name, sched)] = _gpu_fit(dev, b, gm, gst, iters=2, schedule=sched, min_range=64,
                                            max_ranges=1 << 20, max_cell_samples=hint)
            runs[(name, sched)] = to_numpy(gm)
    ref = runs[("none", sdmm.SCHED_BATCHED)]
    for key, got in runs.items():
        assert (stats[key] == stats[("none", sdmm.SCHED_BATCHED)]).all(), key
        if key[0] != "below":
            for k in ref:
                assert np.array_equal(got[k], ref[k]), (key, k)
        else:
            assert_close(compare_mixtures(got, ref, 16), rtol=1e-5, ang_tol=1e-6, what=str(key))
    o = sdmm.default_opts(16, max_cell_samples=-1)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
    with pytest.raises(RuntimeError):
        sdmm.fit_mixtures(dev.from_numpy(b.offsets).cuda(), dev.from_numpy(b.samples).cuda(), gm, gst, o)


def test_unsorted_offsets_mark_every_cell_bad_input(dev, orc):
    """Offsets that decrease somewhere are rejected on the device: every cell reports
    BAD_INPUT and no parameter changes, as in the oracle."""
    print("case: 27 cells with decreasing offsets", flush=True)
    wl = synth.workload("cells4k", scale=27 / 4096)
    b = synth.workload_batch(wl)
    C = wl["grid"].n_cells
    off = b.offsets.copy()
    off[5], off[6] = off[6], off[5]
    bad = synth.Batch(b.samples, off, b.lobe)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    om, ost = synth.copy_mix(mix0), orc.new_state(C, 16)
    s_o = orc.fit(_orc_opts(orc), bad.offsets, bad.samples, om, ost)
    assert (s_o == orc.BAD_INPUT).all()
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
    s_g = _gpu_fit(dev, bad, gm, gst)
    assert (s_g == orc.BAD_INPUT).all()
    for k, v in to_numpy(gm).items():
        assert np.array_equal(v, mix0[k]), k


def test_full_size_cells4k_sampled_cells(dev, orc):
    """The 4096-cell workload at full size in the benchmark's launch configuration; the
    oracle recomputes 24 sampled cells (chosen across the count range) one by one."""
    print("case: cells4k full size, one step, 24 sampled cells", flush=True)
    wl = synth.workload("cells4k")
    b = synth.workload_batch(wl)
    C = wl["grid"].n_cells
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
    s_g = _gpu_fit(dev, b, gm, gst, eta=0.1)
    got = to_numpy(gm)
    order = np.argsort(wl["counts"])
    cells = sorted(set(order[np.linspace(0, C - 1, 24).astype(int)].tolist()))
    for c in cells:
        i0, i1 = b.offsets[c], b.offsets[c + 1]
        sub = np.ascontiguousarray(b.samples[:, i0:i1])
        mc = {k: np.ascontiguousarray(v.reshape(C, -1)[c]) for k, v in mix0.items()}
        st = orc.new_state(1, 16)
        s_o = orc.fit(_orc_opts(orc, eta=0.1), np.array([0, i1 - i0]), sub, mc, st)
        assert s_o[0] == s_g[c]
        gc = {k: v.reshape(C, -1)[c] for k, v in got.items()}
        assert_cells_close(gc, mc, 16, [0], positive_counts(sub, np.array([0, i1 - i0])), what=f"n={i1 - i0}")


# --- accurate covariance update (second pass in the new tangent spaces) ---------------

def test_accurate_sigma_parity_ragged_cells(dev, orc):
    """SDMM_FLAG_ACCURATE_SIGMA against the oracle's accurate update on the 64 ragged
    cells (gated and bad cells included), two iterations per call so that the second
    M-step's mirror refresh is used."""
    print("case: accurate covariance update, 64 ragged cells, 2 iterations", flush=True)
    from paper_2111_13094_amd import sdmm
    wl, b, mix0 = _ragged_case()
    C = wl["grid"].n_cells
    om, ost = synth.copy_mix(mix0), orc.new_state(C, 16)
    s_o = orc.fit(_orc_opts(orc, iters=2, accurate_sigma=1), b.offsets, b.samples, om, ost)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
    s_g = _gpu_fit(dev, b, gm, gst, iters=2, flags=sdmm.FLAG_ACCURATE_SIGMA)
    assert (s_g == s_o).all(), np.nonzero(s_g != s_o)
    got = to_numpy(gm)
    for c in range(C):
        if s_o[c] & (1 | 2 | 4 | 32):
            for k in got:
                assert np.array_equal(got[k].reshape(C, -1)[c], mix0[k].reshape(C, -1)[c], equal_nan=True)
    fitted = [c for c in range(C) if not s_o[c] & (1 | 2 | 4 | 32)]
    assert_cells_close(got, om, 16, fitted, positive_counts(b.samples, b.offsets), what="accurate")
    g = to_numpy(gst)
    fitted = [c for c in range(C) if not s_o[c] & (1 | 2 | 4 | 32)]
    s2g, s2o = g["s2"].reshape(C, 16, 15)[fitted], ost["s2"].reshape(C, 16, 15)[fitted]
    scale = np.abs(s2o).max(axis=2, keepdims=True) + 1e-300
    err = (np.abs(s2g - s2o) / scale).max()
    print("carried S2, worst relative to its largest entry: %.2e" % err)
    assert err < 1e-4


def test_accurate_sigma_single_cell_and_first_order_gap(dev, orc):
    """One cell of 16384 samples from the initial mixture: the GPU's accurate update
    matches the oracle's to 1e-4, while the first-order update differs from it by far
    more, so the test sees which update ran."""
    print("case: accurate covariance update, single cell N=16384", flush=True)
    from paper_2111_13094_amd import sdmm
    wl, b = _single(seed=4321)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    om, ost = synth.copy_mix(mix0), orc.new_state(1, 16)
    orc.fit(_orc_opts(orc, accurate_sigma=1), b.offsets, b.samples, om, ost)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(1, 16))
    _gpu_fit(dev, b, gm, gst, flags=sdmm.FLAG_ACCURATE_SIGMA)
    worst = compare_mixtures(to_numpy(gm), om, 16)
    print("accurate:", worst)
    assert_close(worst, what="accurate single cell")
    fm, fst = to_torch(mix0), state_to_torch(orc.new_state(1, 16))
    _gpu_fit(dev, b, fm, fst)
    gap = compare_mixtures(to_numpy(fm), om, 16)
    print("first-order vs accurate:", gap)
    assert gap["cov"] > 20 * max(worst["cov"], 1e-6)


def test_accurate_sigma_schedules_graph_and_record_tree(dev, orc):
    """Batched, per-cell and graph-replayed accurate fits are bitwise equal, with a cell
    large enough for two record-tree levels in 64-sample items; all match the oracle."""
    print("case: accurate update, record tree, batched / per-cell / graph", flush=True)
    from paper_2111_13094_amd import sdmm
    wl = synth.workload("single", seed=23)
    counts = [120000, 300, 0, 5000, 64, 2000, 17, 900]
    C = len(counts)
    lo, size = np.tile(wl["box_lo"], (C, 1)), np.tile(wl["box_size"], (C, 1))
    b = synth.make_batch(29, counts, lo, size, wl["lobes"])
    mix0 = synth.initial_mixtures(lo, size, 16)
    om, ost = synth.copy_mix(mix0), orc.new_state(C, 16)
    s_o = orc.fit(_orc_opts(orc, iters=2, accurate_sigma=1), b.offsets, b.samples, om, ost)
    runs = []
    for sched, graph in ((sdmm.SCHED_BATCHED, 0), (sdmm.SCHED_PER_CELL, 0), (sdmm.SCHED_BATCHED, 1),
                         (sdmm.SCHED_BATCHED, 1)):
        gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
        s = _gpu_fit(dev, b, gm, gst, iters=2, schedule=sched, use_graph=graph, min_range=64,
                     max_ranges=1 << 20, flags=sdmm.FLAG_ACCURATE_SIGMA)
        assert (s == s_o).all(), (sched, graph, s, s_o)
        runs.append((to_numpy(gm), to_numpy(gst)))
    for m, st in runs[1:]:
        for k in m:
            assert np.array_equal(m[k], runs[0][0][k]), k
        for k in st:
            assert np.array_equal(st[k], runs[0][1][k]), k
    fitted = [c for c in range(C) if not s_o[c] & (1 | 2 | 4 | 32)]
    assert_cells_close(runs[0][0], om, 16, fitted, positive_counts(b.samples, b.offsets), what="accurate, record tree")


def test_accurate_sigma_with_jacobian_responsibilities(dev, orc):
    print("case: accurate update with solid-angle responsibilities", flush=True)
    from paper_2111_13094_amd import sdmm
    wl, b = _single(n=8192, seed=57)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    om, ost = synth.copy_mix(mix0), orc.new_state(1, 16)
    orc.fit(_orc_opts(orc, iters=2, accurate_sigma=1, estep_jacobian=1), b.offsets, b.samples, om, ost)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(1, 16))
    _gpu_fit(dev, b, gm, gst, iters=2, flags=sdmm.FLAG_ACCURATE_SIGMA | sdmm.FLAG_ESTEP_JACOBIAN)
    worst = compare_mixtures(to_numpy(gm), om, 16)
    print(worst)
    assert_close(worst, what="accurate + Jacobian")


def test_accurate_sigma_argument_checks(dev, orc):
    """The accurate update needs batch steps (eta = 1) and a non-fused schedule; unknown
    flag bits are rejected."""
    from paper_2111_13094_amd import sdmm
    wl, b = _single(n=256, seed=3)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    for kw in (dict(eta=0.5), dict(eta_mode=sdmm.ETA_PAPER), dict(schedule=sdmm.SCHED_FUSED)):
        gm, gst = to_torch(mix0), state_to_torch(orc.new_state(1, 16))
        with pytest.raises(RuntimeError, match="invalid argument"):
            _gpu_fit(dev, b, gm, gst, flags=sdmm.FLAG_ACCURATE_SIGMA, **kw)
        for k, v in to_numpy(gm).items():
            assert np.array_equal(v, mix0[k])
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(1, 16))
    with pytest.raises(RuntimeError, match="invalid argument"):
        _gpu_fit(dev, b, gm, gst, flags=32)  # no such flag


# --- stepwise (per-sample) EM ---------------------------------------------------------

def _stepwise_pair(dev, orc, b, mix0, C, K=16, calls=2, gopt=None, oopt=None):
    """calls x (GPU stepwise, oracle stepwise) on the same batch from the same start."""
    from paper_2111_13094_amd import sdmm
    gopt = dict(gopt or {})
    oopt = dict(oopt or {})
    om, ost = synth.copy_mix(mix0), orc.new_state(C, K)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, K))
    for _ in range(calls):
        s_o = orc.fit_stepwise(_orc_opts(orc, K=K, **oopt), b.offsets, b.samples, om, ost)
        s_g = _gpu_fit(dev, b, gm, gst, K=K, schedule=sdmm.SCHED_STEPWISE, **gopt)
        assert (s_g == s_o).all(), (np.nonzero(s_g != s_o), s_g[s_g != s_o], s_o[s_g != s_o])
    return gm, gst, om, ost, s_o


def test_stepwise_parity_single_cell(dev, orc):
    """A batch step (fresh cell) and then one per-sample pass over 4096 samples, FP64 on
    both sides in the same sample order: the chain stays within 1e-10 (measured 3e-15;
    the sides differ only in the order of the lane reductions and in FP64 contraction)."""
    print("case: stepwise EM, one cell, 4096 samples, batch step then per-sample pass", flush=True)
    wl, b = _single(n=4096, seed=71)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    gm, gst, om, ost, _ = _stepwise_pair(dev, orc, b, mix0, 1, gopt=dict(eta_mode=1), oopt=dict(eta_mode=1))
    worst = compare_mixtures(to_numpy(gm), om, 16)
    print(worst)
    assert_close(worst, rtol=1e-10, ang_tol=1e-10, what="stepwise")
    g = to_numpy(gst)
    assert g["step"][0] == ost["step"][0] == 1 + (b.samples[6] > 0).sum()
    assert abs(g["sw"][0] - ost["sw"][0]) <= 1e-10 * ost["sw"][0]


@pytest.mark.parametrize("variant", ["ragged", "jacobian", "constant_eta"])
def test_stepwise_variants(dev, orc, variant):
    print(f"case: stepwise EM, {variant}", flush=True)
    if variant == "ragged":
        wl, b, mix0 = _ragged_case()
        C = wl["grid"].n_cells
        gopt, oopt = dict(eta_mode=1), dict(eta_mode=1)
    else:
        wl, b = _single(n=2048, seed=72)
        mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
        C = 1
        if variant == "jacobian":
            from paper_2111_13094_amd import sdmm
            gopt, oopt = dict(eta_mode=1, flags=sdmm.FLAG_ESTEP_JACOBIAN), dict(eta_mode=1, estep_jacobian=1)
        else:
            gopt, oopt = dict(eta=0.02), dict(eta=0.02)
    gm, gst, om, ost, s_o = _stepwise_pair(dev, orc, b, mix0, C, gopt=gopt, oopt=oopt)
    got = to_numpy(gm)
    fitted = [c for c in range(C) if not s_o[c] & (1 | 2 | 4 | 32)]
    for c in range(C):
        if c not in fitted:
            for k in got:
                assert np.array_equal(got[k].reshape(C, -1)[c], mix0[k].reshape(C, -1)[c], equal_nan=True)
    worst = compare_mixtures(got, om, 16, cells=fitted)
    print(worst)
    # measured up to 9e-11 (the constant-eta chain forgets slowest)
    assert_close(worst, rtol=1e-9, ang_tol=1e-9, what=f"stepwise {variant}")


def test_stepwise_rejects_the_accurate_update(dev, orc):
    from paper_2111_13094_amd import sdmm
    wl, b = _single(n=256, seed=3)
    gm, gst = to_torch(synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)), state_to_torch(orc.new_state(1, 16))
    with pytest.raises(RuntimeError, match="invalid argument"):
        _gpu_fit(dev, b, gm, gst, schedule=sdmm.SCHED_STEPWISE, flags=sdmm.FLAG_ACCURATE_SIGMA)


def test_stepwise_full_size_sampled_cells(dev, orc):
    """The 4096-cell batch in the launch configuration the stepwise benchmark times (a
    batch step, then a per-sample pass over the next batch); 8 sampled cells recomputed by
    the oracle one by one."""
    print("case: stepwise EM at full size, 8 sampled cells", flush=True)
    from paper_2111_13094_amd import sdmm
    wl = synth.workload("cells4k")
    b0, b1 = synth.workload_batch(wl, 0), synth.workload_batch(wl, 1)
    C = wl["grid"].n_cells
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    gm, gst = to_torch(mix0), state_to_torch(orc.new_state(C, 16))
    _gpu_fit(dev, b0, gm, gst, schedule=sdmm.SCHED_STEPWISE, eta_mode=1)
    s_g = _gpu_fit(dev, b1, gm, gst, schedule=sdmm.SCHED_STEPWISE, eta_mode=1)
    got = to_numpy(gm)
    order = np.argsort(wl["counts"])
    for c in sorted(set(order[np.linspace(0, C - 1, 8).astype(int)].tolist())):
        mc = {k: np.ascontiguousarray(v.reshape(C, -1)[c]) for k, v in mix0.items()}
        st = orc.new_state(1, 16)
        for bb in (b0, b1):
            i0, i1 = bb.offsets[c], bb.offsets[c + 1]
            s_o = orc.fit_stepwise(_orc_opts(orc, eta_mode=1), np.array([0, i1 - i0]),
                                   np.ascontiguousarray(bb.samples[:, i0:i1]), mc, st)
        assert s_o[0] == s_g[c]
        worst = compare_mixtures({k: v.reshape(C, -1)[c] for k, v in got.items()}, mc, 16)
        assert_close(worst, rtol=1e-9, ang_tol=1e-9, what=f"stepwise cell {c}")


@pytest.mark.parametrize("K", [4, 12, 32, 40])
def test_stepwise_other_component_counts(dev, orc, K):
    """The stepwise kernel's lane groups for K = 4 (G = 4, half-row DPP reductions),
    K = 12 (G = 16 with idle lanes), K = 32 (G = 32, a cross-row shuffle) and K = 40
    (G = 64, the whole wave): a batch step then a per-sample pass over one cell of 2048
    samples, FP64 on both sides in the same sample order."""
    print(f"case: stepwise EM, one cell of 2048 samples, K={K}", flush=True)
    wl, b = _single(n=2048, seed=73 + K)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)
    gm, gst, om, ost, _ = _stepwise_pair(dev, orc, b, mix0, 1, K=K, gopt=dict(eta_mode=1), oopt=dict(eta_mode=1))
    worst = compare_mixtures(to_numpy(gm), om, K)
    print(worst)
    assert_close(worst, rtol=1e-9, ang_tol=1e-9, what=f"stepwise K={K}")
    g = to_numpy(gst)
    assert g["step"][0] == ost["step"][0]
