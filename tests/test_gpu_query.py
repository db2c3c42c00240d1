"""GPU parity of conditioning, pdf and sampling (through the C ABI) against the oracle.

Both sides start from the same FP64 masters (an oracle fit). Tolerances: pi' absolute
1e-6; m and pdf relative 1e-4 (pdf wherever it exceeds 1e-6 of the query's maximum);
sampled directions 1e-5 rad. A draw whose component choice or cut-locus decision sits
within FP32 rounding of a boundary has two correct outcomes and is compared only for
validity of what was returned."""
import numpy as np
import pytest

from paper_2111_13094_amd import synth
from tests.parity_utils import CUT_LOCUS_BAND, draw_radius, to_torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_13094_amd import sdmm
    sdmm.lib()
    return torch


@pytest.fixture(scope="module")
def fitted(orc):
    """27 cells fitted by the oracle (3 iterations) + queries."""
    wl = synth.workload("cells4k", scale=27 / 4096, seed=11)
    C = wl["grid"].n_cells
    b = synth.workload_batch(wl)
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    st = orc.new_state(C, 16)
    orc.fit(orc.Opts(K=16, iters=3), b.offsets, b.samples, mix, st)
    qpos, qcell = synth.make_queries(12, wl["box_lo"], wl["box_size"], 24)
    return wl, mix, qpos, qcell


def _gpu_cond(dev, mix, C, K, qpos, qcell):
    from paper_2111_13094_amd import sdmm
    gm = to_torch(mix)
    table = sdmm.condition_prepare(gm, C, K)
    qp = dev.from_numpy(np.ascontiguousarray(qpos.T)).cuda()
    qc = dev.from_numpy(qcell).cuda()
    cw, cm = sdmm.condition(table, C, K, qp, qc)
    return table, qp, qc, cw, cm


def test_condition_parity(dev, orc, fitted):
    print("case: condition, 27 cells x 24 queries", flush=True)
    wl, mix, qpos, qcell = fitted
    C = wl["grid"].n_cells
    table, qp, qc, cw, cm = _gpu_cond(dev, mix, C, 16, qpos, qcell)
    cw, cm = cw.cpu().numpy(), cm.cpu().numpy()
    for q in range(qpos.shape[0]):
        pic, m, Sc = orc.condition(16, mix, int(qcell[q]), qpos[q].astype(np.float64))
        assert np.abs(cw[q] - pic).max() < 1e-6, (q, cw[q], pic)
        scale = np.abs(m).max(axis=1, keepdims=True) + 1e-6
        assert (np.abs(cm[q] - m) / scale).max() < 1e-4, (q, cm[q], m)


def _dirs(rng, mix, qcell, nd, K=16):
    """Half uniform directions, half near the cell's component means."""
    nq = qcell.size
    d = rng.normal(size=(nq, nd, 3))
    mus = mix["mu_dir"].reshape(-1, K, 3)
    for q in range(nq):
        ks = rng.integers(0, K, nd // 2)
        d[q, :nd // 2] = mus[qcell[q], ks] + 0.15 * rng.normal(size=(nd // 2, 3))
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return d.astype(np.float32)


def test_pdf_parity(dev, orc, fitted):
    print("case: pdf, 27 cells x 24 queries x 16 directions", flush=True)
    from paper_2111_13094_amd import sdmm
    wl, mix, qpos, qcell = fitted
    C = wl["grid"].n_cells
    nd = 16
    table, qp, qc, cw, cm = _gpu_cond(dev, mix, C, 16, qpos, qcell)
    d = _dirs(np.random.default_rng(3), mix, qcell, nd)
    gd = dev.from_numpy(np.ascontiguousarray(d.reshape(-1, 3).T)).cuda()
    got = sdmm.pdf(table, C, 16, qc, cw, cm, gd, nd).cpu().numpy().reshape(-1, nd)
    ref = orc.pdf(16, mix, qpos.astype(np.float64), qcell, d.astype(np.float64))
    for q in range(ref.shape[0]):
        big = ref[q] > 1e-6 * ref[q].max()
        rel = np.abs(got[q][big] - ref[q][big]) / ref[q][big]
        assert rel.max() < 1e-4, (q, rel.max())
        assert np.all(np.abs(got[q][~big]) <= 2e-6 * ref[q].max())


def _sample_parity(orc, mix, qpos, qcell, u, got_dirs, got_pdf, got_valid, got_comp=None):
    nq, ns = u.shape[0], u.shape[1]
    od, op, oc, ov = orc.sample(16, mix, qpos.astype(np.float64), qcell, u.astype(np.float64))
    ambiguous = 0
    for q in range(nq):
        pic, m, Sc = orc.condition(16, mix, int(qcell[q]), qpos[q].astype(np.float64))
        cdf = np.cumsum(pic)
        for t in range(ns):
            near_cdf = np.min(np.abs(cdf - u[q, t, 0])) < 2e-6
            if got_comp is not None and got_comp[q, t] != oc[q, t]:
                assert near_cdf, (q, t, got_comp[q, t], oc[q, t])
                ambiguous += 1
                continue
            if got_valid[q, t] != ov[q, t]:
                # only at the cut locus |nu| = pi
                k = oc[q, t]
                r = draw_radius(m[k], Sc[k], u[q, t].astype(np.float64))
                assert abs(r - np.pi) < CUT_LOCUS_BAND, (q, t, got_valid[q, t], ov[q, t], r)
                ambiguous += 1
                continue
            if not ov[q, t]:
                assert np.all(got_dirs[q, t] == 0) and got_pdf[q, t] == 0
                continue
            a, b = got_dirs[q, t].astype(np.float64), od[q, t]
            ang = np.arctan2(np.linalg.norm(np.cross(a, b)), a @ b)
            assert ang < 1e-5, (q, t, ang)
            assert abs(got_pdf[q, t] - op[q, t]) <= 1e-4 * op[q, t], (q, t, got_pdf[q, t], op[q, t])
    assert ambiguous <= max(2, nq * ns // 500), ambiguous


def test_sample_parity_with_caller_uniforms(dev, orc, fitted):
    print("case: sample, 27 cells x 24 queries x 8 draws", flush=True)
    from paper_2111_13094_amd import sdmm
    wl, mix, qpos, qcell = fitted
    C = wl["grid"].n_cells
    ns = 8
    nq = qcell.size
    table, qp, qc, cw, cm = _gpu_cond(dev, mix, C, 16, qpos, qcell)
    u = synth.make_uniforms(21, nq * ns)
    gu = dev.from_numpy(np.ascontiguousarray(u.T)).cuda()
    dirs, pdfv, valid, comp = sdmm.sample(table, C, 16, qc, cw, cm, ns, uniforms=gu, with_comp=True)
    _sample_parity(orc, mix, qpos, qcell, u.reshape(nq, ns, 3),
                   dirs.cpu().numpy().T.reshape(nq, ns, 3), pdfv.cpu().numpy().reshape(nq, ns),
                   valid.cpu().numpy().reshape(nq, ns), comp.cpu().numpy().reshape(nq, ns))
    # the fused path gives the same draws
    fd, fp, fv = sdmm.condition_sample_pdf(table, C, 16, qp, qc, ns, uniforms=gu)
    assert dev.equal(fv, valid)
    assert np.allclose(fd.cpu().numpy(), dirs.cpu().numpy(), rtol=0, atol=1e-6)
    assert np.allclose(fp.cpu().numpy(), pdfv.cpu().numpy(), rtol=1e-6, atol=0)


def test_device_generator_matches_the_oracle_generator(dev, orc, fitted):
    print("case: sample with the device Philox generator", flush=True)
    from paper_2111_13094_amd import sdmm
    wl, mix, qpos, qcell = fitted
    C = wl["grid"].n_cells
    ns = 4
    nq = qcell.size
    table, qp, qc, cw, cm = _gpu_cond(dev, mix, C, 16, qpos, qcell)
    seed = 0x1234_5678_9ABC
    d1, p1, v1, _ = sdmm.sample(table, C, 16, qc, cw, cm, ns, uniforms=None, seed=seed)
    u = orc.draw_uniforms(seed, nq * ns).astype(np.float32)
    gu = dev.from_numpy(np.ascontiguousarray(u.T)).cuda()
    d2, p2, v2, _ = sdmm.sample(table, C, 16, qc, cw, cm, ns, uniforms=gu)
    assert dev.equal(d1, d2) and dev.equal(p1, p2) and dev.equal(v1, v2)
    f1, fp1, fv1 = sdmm.condition_sample_pdf(table, C, 16, qp, qc, ns, uniforms=None, seed=seed)
    assert dev.equal(fv1, v1)


def test_invalid_query_cells_give_zero(dev, orc, fitted):
    print("case: queries with out-of-range cells", flush=True)
    from paper_2111_13094_amd import sdmm
    wl, mix, qpos, qcell = fitted
    C = wl["grid"].n_cells
    qc_bad = qcell[:8].copy()
    qc_bad[[1, 4]] = -1
    qc_bad[[2, 6]] = C
    table, qp, qc, cw, cm = _gpu_cond(dev, mix, C, 16, qpos[:8], qc_bad)
    cw = cw.cpu().numpy()
    assert np.all(cw[[1, 2, 4, 6]] == 0)
    assert np.allclose(cw[[0, 3, 5, 7]].sum(1), 1.0, atol=1e-5)
    d, p, v = sdmm.condition_sample_pdf(table, C, 16, qp, qc, 4, uniforms=None, seed=1)
    v = v.cpu().numpy().reshape(8, 4)
    assert not v[[1, 2, 4, 6]].any()
    assert v[[0, 3, 5, 7]].sum() >= 12


@pytest.mark.parametrize("K", [8, 32])
def test_condition_and_pdf_other_K(dev, orc, K):
    print(f"case: condition + pdf with K={K}", flush=True)
    from paper_2111_13094_amd import sdmm
    wl = synth.workload("single", seed=4)
    b = synth.make_batch(9, [4096], wl["box_lo"], wl["box_size"], wl["lobes"])
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)
    orc.fit(orc.Opts(K=K, iters=3), b.offsets, b.samples, mix, orc.new_state(1, K))
    qpos, qcell = synth.make_queries(3, wl["box_lo"], wl["box_size"], 32)
    gm = to_torch(mix)
    table = sdmm.condition_prepare(gm, 1, K)
    qp = dev.from_numpy(np.ascontiguousarray(qpos.T)).cuda()
    qc = dev.from_numpy(qcell).cuda()
    cw, cm = sdmm.condition(table, 1, K, qp, qc)
    d = _dirs(np.random.default_rng(5), mix, qcell, 8, K=K)
    gd = dev.from_numpy(np.ascontiguousarray(d.reshape(-1, 3).T)).cuda()
    got = sdmm.pdf(table, 1, K, qc, cw, cm, gd, 8).cpu().numpy().reshape(-1, 8)
    ref = orc.pdf(K, mix, qpos.astype(np.float64), qcell, d.astype(np.float64))
    for q in range(ref.shape[0]):
        big = ref[q] > 1e-6 * ref[q].max()
        assert (np.abs(got[q][big] - ref[q][big]) / ref[q][big]).max() < 1e-4


@pytest.mark.parametrize("K,ns", [(16, 3), (16, 5), (16, 12), (8, 2), (32, 4), (32, 20)])
def test_fused_path_matches_the_separate_calls(dev, orc, K, ns):
    """The fused condition + sample + pdf call batches the draws of several rounds of
    queries when a query has at most half a lane group of draws, and runs one round
    otherwise; both must give the draws of the separate condition, sample and pdf calls
    on the same caller uniforms (43 queries: a ragged last pass)."""
    print(f"case: fused vs separate, K={K}, ns={ns}", flush=True)
    from paper_2111_13094_amd import sdmm
    wl = synth.workload("single", seed=6)
    b = synth.make_batch(13, [4096], wl["box_lo"], wl["box_size"], wl["lobes"])
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)
    orc.fit(orc.Opts(K=K, iters=3), b.offsets, b.samples, mix, orc.new_state(1, K))
    qpos, qcell = synth.make_queries(5, wl["box_lo"], wl["box_size"], 43)
    qcell = qcell.copy()
    qcell[[3, 17]] = -1  # unusable queries give no draws on either path
    table, qp, qc, cw, cm = _gpu_cond(dev, mix, 1, K, qpos, qcell)
    nq = qcell.size
    u = synth.make_uniforms(23, nq * ns)
    gu = dev.from_numpy(np.ascontiguousarray(u.T)).cuda()
    dirs, pdfv, valid, _ = sdmm.sample(table, 1, K, qc, cw, cm, ns, uniforms=gu)
    fd, fp, fv = sdmm.condition_sample_pdf(table, 1, K, qp, qc, ns, uniforms=gu)
    assert dev.equal(fv, valid)
    assert int(valid.sum()) >= (nq - 2) * ns // 2
    assert not valid.view(nq, ns)[[3, 17]].any()
    assert np.allclose(fd.cpu().numpy(), dirs.cpu().numpy(), rtol=0, atol=1e-6)
    assert np.allclose(fp.cpu().numpy(), pdfv.cpu().numpy(), rtol=1e-6, atol=0)
    # the device generator: the same draws through both paths
    d1, p1, v1, _ = sdmm.sample(table, 1, K, qc, cw, cm, ns, uniforms=None, seed=77)
    f1, q1, w1 = sdmm.condition_sample_pdf(table, 1, K, qp, qc, ns, uniforms=None, seed=77)
    assert dev.equal(w1, v1)
    assert np.allclose(f1.cpu().numpy(), d1.cpu().numpy(), rtol=0, atol=1e-6)
