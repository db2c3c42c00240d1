"""Pins for the oracle's spatial kD-tree (Sec. 4.2 "Refinement of the spatial kD-tree",
Sec. 4.3 "Initialization"): the pre-subdivision, the split rule checked by numpy on the
samples of every split node, point location, stable reordering, the copies of the parent
mixture, the leaf initialisation against the synthetic-input module's recipe (separate
code), idempotence, capacity and unsplittable leaves."""
import numpy as np
import pytest

from paper_2111_13094_amd import synth

K = 16


def _samples(n, seed=0, dist="beta"):
    rng = np.random.default_rng(seed)
    smp = np.zeros((7, n), dtype=np.float32)
    if dist == "beta":
        smp[3:6] = rng.beta(2, 5, size=(3, n))
    else:
        smp[3:6] = rng.random((3, n))
    d = rng.normal(size=(3, n))
    smp[0:3] = d / np.linalg.norm(d, axis=0)
    smp[6] = np.arange(n, dtype=np.float32)  # the weight channel carries the index (exact below 2^24)
    return smp


def _store(max_leaves):
    mix = {k: np.zeros(max_leaves * n) for k, n in (("pi", K), ("mu_dir", 3 * K), ("mu_pos", 3 * K), ("cov", 15 * K))}
    st = {"s0": np.zeros(max_leaves * K), "s2": np.zeros(max_leaves * 15 * K), "sw": np.zeros(max_leaves),
          "step": np.zeros(max_leaves, dtype=np.int32)}
    return mix, st


def test_presubdivision_tiles_the_box(orc):
    t = orc.tree_init(1024, 3, [0.0, -1.0, 2.0], [1.0, 1.0, 6.0])
    assert t.n_leaves == 512 and t.n_nodes == 1023
    vol = np.prod(t.hi[:512] - t.lo[:512], axis=1)
    assert np.allclose(vol, 8.0 / 512, rtol=1e-14)
    # the boxes tile the root box: every point of a fine lattice is in exactly one box
    g = np.stack(np.meshgrid(*[np.linspace(a + 1e-3, b - 1e-3, 23) for a, b in
                               zip([0.0, -1.0, 2.0], [1.0, 1.0, 6.0])], indexing="ij"), -1).reshape(-1, 3)
    inside = np.stack([np.all((g >= t.lo[l]) & (g < t.hi[l]), axis=1) for l in range(512)])
    assert np.all(inside.sum(0) == 1)
    assert np.all(t.init[:512] == 0)


def _refined(orc, n=120000, c=3000, seed=1, max_leaves=4096, dist="beta"):
    t = orc.tree_init(max_leaves, 2, [0, 0, 0], [1, 1, 1])
    smp = _samples(n, seed, dist)
    mix, st = _store(max_leaves)
    status, srt, off = orc.tree_refine(t, smp, c, K, mix, st)
    return t, smp, mix, st, status, srt, off


def test_every_split_follows_the_rule(orc):
    """For every node the refinement split: its samples number more than c, the axis is
    the one of largest variance of their positions, and the split is their mean there."""
    c = 3000
    t, smp, mix, st, status, srt, off = _refined(orc, c=c)
    assert status == 0 and t.n_leaves > 64
    # samples of each node = samples of the leaves below it
    leaf_samples = [srt[3:6, off[l]:off[l + 1]].T.astype(np.float64) for l in range(t.n_leaves)]

    def below(n):
        if t.axis[n] < 0:
            return leaf_samples[t.leaf[n]]
        return np.concatenate([below(t.left[n]), below(t.left[n] + 1)])

    checked = 0
    for n in range(63, t.n_nodes):  # the 64 pre-subdivision leaves and the nodes made since
        if t.axis[n] < 0:
            continue
        P = below(n)
        assert P.shape[0] > c
        mean = P.mean(0)
        var = P.var(0)
        assert t.axis[n] == int(np.argmax(var))
        assert t.split[n] == pytest.approx(mean[t.axis[n]], rel=1e-13)
        checked += 1
    assert checked == t.n_leaves - 64


def test_leaves_hold_their_samples_and_respect_the_threshold(orc):
    c = 3000
    t, smp, mix, st, status, srt, off = _refined(orc, c=c)
    counts = np.diff(off)
    assert counts.sum() == smp.shape[1] and np.all(counts <= c)
    for l in range(t.n_leaves):
        P = srt[3:6, off[l]:off[l + 1]].T.astype(np.float64)
        assert np.all((P >= t.lo[l]) & ((P < t.hi[l]) | (t.hi[l] == 1.0)))
        # stable: original index order within the leaf
        idx = srt[6, off[l]:off[l + 1]]
        assert np.all(np.diff(idx) > 0)
    assert np.array_equal(np.sort(srt[6]), smp[6])


def test_new_leaves_copy_the_parent_mixture(orc):
    """Leaves made by splitting carry a copy of the mixture and Robbins-Monro state of
    the leaf they came from."""
    max_leaves = 4096
    t = orc.tree_init(max_leaves, 2, [0, 0, 0], [1, 1, 1])
    mix, st = _store(max_leaves)
    rng = np.random.default_rng(3)
    for key in mix:
        mix[key][:64 * (mix[key].size // max_leaves)] = rng.random(64 * (mix[key].size // max_leaves))
    st["sw"][:64] = rng.random(64)
    st["step"][:64] = rng.integers(1, 9, 64)
    t.init[:64] = 1
    before = {k: v.copy() for k, v in mix.items()}
    sw_before = st["sw"].copy()
    boxes_before = (t.lo[:64].copy(), t.hi[:64].copy())
    smp = _samples(100000, 4)
    orc.tree_refine(t, smp, 2500, K, mix, st)
    assert t.n_leaves > 64
    for r in range(t.n_leaves):
        centre = 0.5 * (t.lo[r] + t.hi[r])
        orig = int(np.nonzero(np.all((centre >= boxes_before[0]) & (centre < boxes_before[1]), axis=1))[0][0])
        for key in mix:
            w = mix[key].size // max_leaves
            assert np.array_equal(mix[key][r * w:(r + 1) * w], before[key][orig * w:(orig + 1) * w]), (r, key)
        assert st["sw"][r] == sw_before[orig] and t.init[r] == 1


def test_initialisation_of_leaves_with_enough_samples(orc):
    """Uninitialised leaves with at least 16 samples get the initial mixture of their box
    (the same recipe as the synthetic-input module, written separately there) and a zero
    state; leaves with fewer samples stay untouched."""
    max_leaves = 1024
    t = orc.tree_init(max_leaves, 2, [0, 0, 0], [1, 1, 1])
    mix, st = _store(max_leaves)
    mix["pi"][:] = -7.0  # marker
    smp = _samples(64 * 20, 5, dist="beta")
    _, srt, off = orc.tree_refine(t, smp, 100000, K, mix, st)
    counts = np.diff(off)
    assert (counts >= 16).any() and (counts < 16).any()
    for l in range(t.n_leaves):
        if counts[l] >= 16:
            ref = synth.initial_mixtures(t.lo[l][None], (t.hi[l] - t.lo[l])[None], K)
            for key in mix:
                w = mix[key].size // max_leaves
                assert np.allclose(mix[key][l * w:(l + 1) * w], ref[key], rtol=1e-14, atol=1e-15), (l, key)
            assert t.init[l] == 1 and st["step"][l] == 0
        else:
            assert t.init[l] == 0 and np.all(mix["pi"][l * K:(l + 1) * K] == -7.0)


@pytest.mark.parametrize("Kc", [5, 12, 32, 64])
def test_initial_leaf_mixture_other_K(orc, Kc):
    lo, hi = np.array([0.2, -1.0, 3.0]), np.array([0.7, 2.0, 3.5])
    got = orc.init_leaf(Kc, lo, hi)
    ref = synth.initial_mixtures(lo[None], (hi - lo)[None], Kc)
    for key in got:
        assert np.allclose(got[key], ref[key], rtol=1e-14, atol=1e-15), key


def test_refining_again_changes_nothing(orc):
    t, smp, mix, st, status, srt, off = _refined(orc, n=60000, c=2000, seed=7)
    nodes = t.n_nodes
    status2, srt2, off2 = orc.tree_refine(t, smp, 2000, K, mix, st)
    assert t.n_nodes == nodes and np.array_equal(off2, off) and np.array_equal(srt2, srt)


def test_capacity_and_unsplittable_leaves(orc):
    # capacity: room for 70 leaves only
    t, smp, mix, st, status, srt, off = _refined(orc, n=120000, c=1000, max_leaves=70)
    assert status & 1 and t.n_leaves == 70 and t.n_nodes <= 2 * 70 - 1
    assert np.diff(off).sum() == 120000
    # a leaf whose samples all sit at one position cannot be split
    t = orc.tree_init(64, 0, [0, 0, 0], [1, 1, 1])
    smp = _samples(5000, 8)
    smp[3:6] = 0.25
    mix, st = _store(64)
    status, srt, off = orc.tree_refine(t, smp, 100, K, mix, st)
    assert t.n_leaves == 1 and status == 0 and off[-1] == 5000
