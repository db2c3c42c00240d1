"""GPU parity of the spatial kD-tree (through the C ABI) against the FP64 oracle:
pre-subdivision, refinement rounds, mixture copies, leaf initialisation and the
reordering by leaf. Integer and index results (tree structure, leaf assignment, counts,
offsets, the reordered samples, copied mixtures) must be equal. Split positions and leaf
boxes are FP64 means whose sums run in a different order on the two sides: relative
1e-12 (a sample would have to lie within ~1e-16 of a plane for the assignment to differ).
Initial mixtures: relative 1e-14 (the same FP64 formulas, contracted differently)."""
import numpy as np
import pytest

from paper_2111_13094_amd import synth
from tests.parity_utils import assert_cells_close, positive_counts, state_to_torch, to_numpy, to_torch

pytestmark = pytest.mark.gpu

K = 16


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_13094_amd import sdmm
    sdmm.lib()
    return torch


def _samples(n, seed=0):
    rng = np.random.default_rng(seed)
    smp = np.zeros((7, n), dtype=np.float32)
    smp[3:6] = rng.beta(2, 5, size=(3, n))
    d = rng.normal(size=(3, n))
    smp[0:3] = d / np.linalg.norm(d, axis=0)
    smp[6] = np.exp(rng.normal(size=n))
    return smp


def _store(max_leaves, seed=None, n_init=0):
    mix = {k: np.zeros(max_leaves * n) for k, n in (("pi", K), ("mu_dir", 3 * K), ("mu_pos", 3 * K), ("cov", 15 * K))}
    st = {"s0": np.zeros(max_leaves * K), "s2": np.zeros(max_leaves * 15 * K), "sw": np.zeros(max_leaves),
          "step": np.zeros(max_leaves, dtype=np.int32)}
    if seed is not None:
        rng = np.random.default_rng(seed)
        for key in mix:
            w = mix[key].size // max_leaves
            mix[key][:n_init * w] = rng.random(n_init * w)
        st["sw"][:n_init] = rng.random(n_init)
        st["step"][:n_init] = rng.integers(1, 9, n_init)
    return mix, st


def _gpu_tree(dev, orc_tree):
    """Device copy of an oracle tree."""
    from paper_2111_13094_amd import sdmm
    t = sdmm.new_tree(orc_tree.max_leaves)
    for key in ("counts", "axis", "left", "leaf", "split", "leaf_node", "lo", "hi", "init"):
        t[key].copy_(dev.from_numpy(np.ascontiguousarray(getattr(orc_tree, key))))
    return t


def _assert_tree_equal(t_gpu, t_orc):
    g = {k: v.cpu().numpy() for k, v in t_gpu.items() if hasattr(v, "cpu")}
    assert np.array_equal(g["counts"], t_orc.counts)
    n, L = t_orc.n_nodes, t_orc.n_leaves
    for key in ("axis", "left", "leaf"):
        assert np.array_equal(g[key][:n], getattr(t_orc, key)[:n]), key
    assert np.array_equal(g["leaf_node"][:L], t_orc.leaf_node[:L])
    assert np.array_equal(g["init"][:L], t_orc.init[:L])
    assert np.allclose(g["split"][:n], t_orc.split[:n], rtol=1e-12, atol=0)
    assert np.allclose(g["lo"][:L], t_orc.lo[:L], rtol=1e-12, atol=0)
    assert np.allclose(g["hi"][:L], t_orc.hi[:L], rtol=1e-12, atol=0)


def test_tree_init_matches_the_oracle(dev, orc):
    print("case: pre-subdivision depth 3", flush=True)
    from paper_2111_13094_amd import sdmm
    lo, hi = [0.0, -1.0, 2.0], [1.0, 1.0, 6.0]
    t = sdmm.new_tree(1024)
    sdmm.tree_init(t, 3, lo, hi)
    ref = orc.tree_init(1024, 3, lo, hi)
    g = {k: v.cpu().numpy() for k, v in t.items() if hasattr(v, "cpu")}
    assert np.array_equal(g["counts"], ref.counts)
    for key in ("axis", "left", "leaf", "split", "leaf_node", "lo", "hi", "init"):
        n = 1023 if key in ("axis", "left", "leaf", "split") else 512
        assert np.array_equal(g[key][:n], getattr(ref, key)[:n]), key


def _refine_both(dev, orc, smp, c, max_leaves, depth=2, seed=None, n_init=0, t_orc=None, store=None):
    from paper_2111_13094_amd import sdmm
    if t_orc is None:
        t_orc = orc.tree_init(max_leaves, depth, [0, 0, 0], [1, 1, 1])
        t_orc.init[:n_init] = 1
    t_gpu = _gpu_tree(dev, t_orc)
    mix, st = store if store is not None else _store(max_leaves, seed, n_init)
    gm, gst = to_torch(mix), state_to_torch(st)
    srt_g, off_g, L, status_g = sdmm.tree_refine(t_gpu, dev.from_numpy(smp).cuda(), c, gm, gst, K)
    status_o, srt_o, off_o = orc.tree_refine(t_orc, smp, c, K, mix, st)
    return t_gpu, t_orc, (srt_g, off_g, L, status_g, gm, gst), (srt_o, off_o, status_o, mix, st)


def _assert_refine_equal(t_gpu, t_orc, g, o):
    srt_g, off_g, L, status_g, gm, gst = g
    srt_o, off_o, status_o, mix, st = o
    _assert_tree_equal(t_gpu, t_orc)
    assert L == t_orc.n_leaves and status_g == status_o
    assert np.array_equal(off_g.cpu().numpy(), off_o)
    assert np.array_equal(srt_g.cpu().numpy(), srt_o)
    gmix, gs = to_numpy(gm), to_numpy(gst)
    init_fresh = None
    for key in mix:
        assert np.allclose(gmix[key], mix[key], rtol=1e-14, atol=1e-15), key
    for key in st:
        assert np.allclose(gs[key], st[key], rtol=1e-14, atol=0), key


def test_tree_refine_matches_the_oracle(dev, orc):
    print("case: refine 300000 samples, c = 4000, 64 pre-subdivided leaves (half initialised)", flush=True)
    smp = _samples(300000, 1)
    t_gpu, t_orc, g, o = _refine_both(dev, orc, smp, 4000, 4096, seed=3, n_init=32)
    assert t_orc.n_leaves > 100
    _assert_refine_equal(t_gpu, t_orc, g, o)


def test_tree_refine_twice_matches_the_oracle(dev, orc):
    """A second iteration's samples refine the refined tree further."""
    print("case: refine twice (2 x 200000 samples)", flush=True)
    from paper_2111_13094_amd import sdmm
    t_gpu, t_orc, g, o = _refine_both(dev, orc, _samples(200000, 4), 3000, 4096, seed=5, n_init=64)
    _assert_refine_equal(t_gpu, t_orc, g, o)
    smp2 = _samples(400000, 6)
    mix, st = o[3], o[4]
    gm, gst = g[4], g[5]
    srt_g, off_g, L, status_g = sdmm.tree_refine(t_gpu, dev.from_numpy(smp2).cuda(), 3000, gm, gst, K)
    status_o, srt_o, off_o = orc.tree_refine(t_orc, smp2, 3000, K, mix, st)
    _assert_refine_equal(t_gpu, t_orc, (srt_g, off_g, L, status_g, gm, gst), (srt_o, off_o, status_o, mix, st))


def test_refine_of_a_tree_deeper_than_the_staged_top(dev, orc):
    """Walks that leave the work group's LDS copy of the oldest 4096 nodes and go on in
    global memory: a first refinement grows the tree to about 7700 nodes, and a second
    iteration's samples are located from the root through both parts (and split further,
    with a ragged last tile)."""
    print("case: refine 400000 samples (c = 150), then 300001 more from the root (c = 90)", flush=True)
    from paper_2111_13094_amd import sdmm
    t_gpu, t_orc, g, o = _refine_both(dev, orc, _samples(400000, 11), 150, 8192)
    assert t_orc.n_nodes > 7000
    _assert_refine_equal(t_gpu, t_orc, g, o)
    smp2 = _samples(300001, 12)
    mix, st = o[3], o[4]
    gm, gst = g[4], g[5]
    srt_g, off_g, L, status_g = sdmm.tree_refine(t_gpu, dev.from_numpy(smp2).cuda(), 90, gm, gst, K)
    n_before = t_orc.n_nodes
    status_o, srt_o, off_o = orc.tree_refine(t_orc, smp2, 90, K, mix, st)
    assert t_orc.n_nodes > n_before
    _assert_refine_equal(t_gpu, t_orc, (srt_g, off_g, L, status_g, gm, gst), (srt_o, off_o, status_o, mix, st))


def test_locate_on_and_beside_split_planes(dev, orc):
    """Positions on a split plane and one FP32 step to either side of it, against FP64
    splits on an FP32 value, one FP64 step to either side of that value, halfway to the
    next FP32 value, and on it: every sample must take the FP64 comparison's branch (the
    threshold is never reached, so only the location, the reordering and the leaf
    initialisation run)."""
    print("case: 60000 samples on and beside the split planes of a depth-2 tree", flush=True)
    t_orc = orc.tree_init(64, 2, [0, 0, 0], [1, 1, 1])
    rng = np.random.default_rng(13)
    inner = np.flatnonzero(t_orc.axis[:t_orc.n_nodes] >= 0)
    mid = t_orc.split[inner]
    assert np.array_equal(mid, mid.astype(np.float32))
    up32 = np.nextafter(mid.astype(np.float32), np.float32(2)).astype(np.float64)
    choice = np.stack([mid, np.nextafter(mid, 2.0), np.nextafter(mid, -1.0), 0.5 * (mid + up32), up32])
    t_orc.split[inner] = choice[rng.integers(0, 5, inner.size), np.arange(inner.size)]
    n = 60000
    base = np.array([0.25, 0.5, 0.75], dtype=np.float32)[rng.integers(0, 3, (3, n))]
    step = rng.integers(-1, 2, (3, n))
    pos = np.where(step > 0, np.nextafter(base, np.float32(2)),
                   np.where(step < 0, np.nextafter(base, np.float32(-1)), base))
    smp = _samples(n, 14)
    smp[3:6] = pos
    t_gpu, t_orc, g, o = _refine_both(dev, orc, smp, 1 << 30, 64, t_orc=t_orc)
    assert t_orc.n_leaves == 64
    _assert_refine_equal(t_gpu, t_orc, g, o)


def test_refine_rejects_a_tree_with_counts_out_of_range(dev, orc):
    """The counts are read from the device after the first round's location and sort pass
    are queued: a tree whose counts are out of range is rejected with SDMM_EINVAL and left
    as it was, and the same tree refines normally once its counts are restored."""
    print("case: refine with leaf count 0, then node count above capacity, then restored", flush=True)
    from paper_2111_13094_amd import sdmm
    t_orc = orc.tree_init(64, 1, [0, 0, 0], [1, 1, 1])
    t_gpu = _gpu_tree(dev, t_orc)
    mix, st = _store(64)
    gm, gst = to_torch(mix), state_to_torch(st)
    smp = dev.from_numpy(_samples(20000, 15)).cuda()
    before = {k: v.clone() for k, v in t_gpu.items() if hasattr(v, "clone")}
    for bad in ([t_orc.n_nodes, 0], [t_gpu["max_nodes"] + 1, t_orc.n_leaves]):
        t_gpu["counts"].copy_(dev.tensor(bad, dtype=dev.int32))
        with pytest.raises(RuntimeError, match="sdmm_tree_refine"):
            sdmm.tree_refine(t_gpu, smp, 500, gm, gst, K)
        for k, v in before.items():
            if k != "counts":
                assert dev.equal(t_gpu[k], v), k
    t_gpu["counts"].copy_(before["counts"])
    srt_g, off_g, L, status_g = sdmm.tree_refine(t_gpu, smp, 500, gm, gst, K)
    status_o, srt_o, off_o = orc.tree_refine(t_orc, smp.cpu().numpy(), 500, K, mix, st)
    _assert_refine_equal(t_gpu, t_orc, (srt_g, off_g, L, status_g, gm, gst), (srt_o, off_o, status_o, mix, st))


def test_tree_capacity_constant_positions_and_empty_input(dev, orc):
    print("case: capacity 70 leaves; constant positions; no samples", flush=True)
    t_gpu, t_orc, g, o = _refine_both(dev, orc, _samples(120000, 7), 1000, 70)
    assert o[2] & 1 and t_orc.n_leaves == 70
    _assert_refine_equal(t_gpu, t_orc, g, o)
    smp = _samples(5000, 8)
    smp[3:6] = 0.25
    t_gpu, t_orc, g, o = _refine_both(dev, orc, smp, 100, 64, depth=0)
    assert t_orc.n_leaves == 1
    _assert_refine_equal(t_gpu, t_orc, g, o)
    t_gpu, t_orc, g, o = _refine_both(dev, orc, np.zeros((7, 0), dtype=np.float32), 100, 64)
    _assert_refine_equal(t_gpu, t_orc, g, o)


def test_refine_then_fit_matches_the_oracle(dev, orc):
    """The pipeline of one rendering iteration: refine with the iteration's samples,
    initialise leaves, then one batched EM step on the leaves."""
    print("case: refine + initialise + fit, 200000 samples", flush=True)
    from paper_2111_13094_amd import sdmm
    wl = synth.workload("single", seed=9)
    b = synth.make_batch(10, [200000], np.zeros((1, 3)), np.ones((1, 3)), wl["lobes"], parallax=True)
    smp = b.samples
    t_gpu, t_orc, g, o = _refine_both(dev, orc, smp, 6000, 1024)
    _assert_refine_equal(t_gpu, t_orc, g, o)
    srt_g, off_g, L, _, gm, gst = g
    srt_o, off_o, _, mix, st = o
    view = lambda d, n: {k: v[:n * (v.numel() // 1024)] for k, v in d.items()}
    nview = lambda d, n: {k: np.ascontiguousarray(v[:n * (v.size // 1024)]) for k, v in d.items()}
    gmv, gsv = view(gm, L), view(gst, L)
    sdmm.fit_mixtures(off_g, srt_g, gmv, gsv, sdmm.default_opts(K))
    om, ost = nview(mix, L), nview(st, L)
    orc.fit(orc.Opts(K=K), off_o, srt_o, om, ost)
    fitted = [l for l in range(L) if off_o[l + 1] - off_o[l] >= 64]
    assert_cells_close(to_numpy(gmv), om, K, fitted, positive_counts(srt_o, off_o), what="refine + fit")


def test_full_size_refinement(dev, orc):
    """The 16384-cell workload's 16.6M samples in a depth-3 pre-subdivided tree with the
    paper's threshold c = 16000: the whole structure, the offsets and a million sampled
    entries of the reordered samples against the oracle."""
    print("case: refine 16.6M samples, c = 16000", flush=True)
    from paper_2111_13094_amd import sdmm
    wl = synth.workload("cells16k")
    smp = synth.workload_batch(wl).samples
    max_leaves = 8192
    t_orc = orc.tree_init(max_leaves, 3, [0, 0, 0], [1, 1, 1])
    t_gpu = _gpu_tree(dev, t_orc)
    mix, st = _store(max_leaves)
    gm, gst = to_torch(mix), state_to_torch(st)
    srt_g, off_g, L, status_g = sdmm.tree_refine(t_gpu, dev.from_numpy(smp).cuda(), 16000, gm, gst, K)
    status_o, srt_o, off_o = orc.tree_refine(t_orc, smp, 16000, K, mix, st)
    _assert_tree_equal(t_gpu, t_orc)
    assert L == t_orc.n_leaves and status_g == status_o
    assert np.array_equal(off_g.cpu().numpy(), off_o)
    assert np.diff(off_o).max() <= 16000
    pick = np.random.default_rng(2).choice(smp.shape[1], 1 << 20, replace=False)
    assert np.array_equal(srt_g[:, dev.from_numpy(pick).cuda()].cpu().numpy(), srt_o[:, pick])
    print("leaves", L, "nodes", t_orc.n_nodes)
