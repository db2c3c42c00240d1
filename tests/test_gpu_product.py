"""GPU parity of product sampling with a conditioned BSDF mixture (through the C ABI)
against the FP64 oracle.

Both sides start from the same FP64 masters (an oracle fit of the radiance cells, random
BSDF models) and the same FP32 query inputs. Tolerances: sampled directions 1e-5 rad
and their pdf relative 2e-4; pdf at given directions relative 2e-4 wherever it exceeds
1e-6 of the query's largest value. The FP32 chain behind them: conditioning (relative
1e-6 in the offsets), the rotation to world and the transfer Jacobian (1e-6), the 2x2
products and Cholesky factors of C (relative 1e-6 times cond(S), up to ~1e2 here), then
a quadratic form q of up to ~30 whose absolute error of a few 1e-6 changes exp(-q/2) by
as much relative, and log2 normalisers from the hardware logarithm (1 ulp). Measured on
MI355X: 6.8e-7 rad and 1.3e-5 relative. A draw whose pair choice
sits within FP32 rounding of a CDF boundary, or a query whose second and third BSDF
weights tie within rounding, has two correct outcomes and is compared only for validity
of what was returned."""
import numpy as np
import pytest

from paper_2111_13094_amd import synth
from tests.parity_utils import CUT_LOCUS_BAND, draw_radius, to_torch

pytestmark = pytest.mark.gpu

DIR_TOL = 1e-5
PDF_RTOL = 2e-4


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_13094_amd import sdmm
    sdmm.lib()
    return torch


@pytest.fixture(scope="module")
def scene(orc):
    """27 radiance cells fitted by the oracle, 3 BSDF models of 8 components, 8 queries
    per cell with BSDF inputs, model indices and shading frames."""
    wl = synth.workload("cells4k", scale=27 / 4096, seed=11)
    C = wl["grid"].n_cells
    b = synth.workload_batch(wl)
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    orc.fit(orc.Opts(K=16, iters=3), b.offsets, b.samples, mix, orc.new_state(C, 16))
    qpos, qcell = synth.make_queries(12, wl["box_lo"], wl["box_size"], 8)
    bmix = synth.bsdf_mixtures(31, 3, 8)
    bpar, bcell, F = synth.bsdf_queries(32, qcell.size, 3)
    return dict(C=C, K=16, mix=mix, CB=3, Kb=8, bmix=bmix, qpos=qpos.astype(np.float32), qcell=qcell,
                bpar=bpar.astype(np.float32), bcell=bcell, F=F.astype(np.float32))


def _gpu_inputs(dev, sc):
    from paper_2111_13094_amd import sdmm
    table = sdmm.condition_prepare(to_torch(sc["mix"]), sc["C"], sc["K"])
    btable = sdmm.condition_prepare(to_torch(sc["bmix"]), sc["CB"], sc["Kb"])
    t = lambda a: dev.from_numpy(np.ascontiguousarray(a)).cuda()
    nq = sc["qcell"].size
    return dict(table=table, btable=btable, qpos=t(sc["qpos"].T), qcell=t(sc["qcell"]), bpar=t(sc["bpar"].T),
                bcell=t(sc["bcell"]), frames=t(sc["F"].reshape(nq, 9).T))


def _gpu_sample(dev, sc, g, ns, uniforms=None, seed=0):
    from paper_2111_13094_amd import sdmm
    gu = None if uniforms is None else dev.from_numpy(np.ascontiguousarray(uniforms.reshape(-1, 3).T)).cuda()
    d, p, v, pr = sdmm.product_sample(g["table"], sc["C"], sc["K"], g["qpos"], g["qcell"], g["btable"], sc["CB"],
                                      sc["Kb"], g["bpar"], g["bcell"], g["frames"], ns, uniforms=gu, seed=seed,
                                      with_pair=True)
    nq = sc["qcell"].size
    return (d.cpu().numpy().T.reshape(nq, ns, 3), p.cpu().numpy().reshape(nq, ns), v.cpu().numpy().reshape(nq, ns),
            pr.cpu().numpy().reshape(nq, ns))


def _orc_args(sc):
    return (sc["K"], sc["mix"], sc["Kb"], sc["bmix"], sc["qpos"].astype(np.float64), sc["qcell"],
            sc["bpar"].astype(np.float64), sc["bcell"], sc["F"].astype(np.float64))


def _ambiguous_query(orc, sc, q):
    """True when the BSDF components ranked second and third (or first and second) tie
    within FP32 rounding, so the pruning has two correct outcomes."""
    bpic, _, _ = orc.condition(sc["Kb"], sc["bmix"], int(sc["bcell"][q]), sc["bpar"][q].astype(np.float64))
    w = np.sort(bpic)[::-1]
    return any(abs(w[i] - w[i + 1]) <= 1e-5 * w[i] for i in range(min(2, w.size - 1)))


def _compare(orc, sc, u, got, stats):
    gd, gp, gv, gpair = got
    nq, ns = u.shape[0], u.shape[1]
    od, op, opair, ov = orc.product_sample(*_orc_args(sc), u.astype(np.float64))
    ambiguous = 0
    for q in range(nq):
        if _ambiguous_query(orc, sc, q):
            ambiguous += ns
            continue
        pr = orc.product_pairs(sc["K"], sc["mix"], int(sc["qcell"][q]), sc["Kb"], sc["bmix"], int(sc["bcell"][q]),
                               sc["qpos"][q].astype(np.float64), sc["bpar"][q].astype(np.float64),
                               sc["F"][q].astype(np.float64))
        P = np.exp(pr["logw"] - pr["logw"].max())
        cdf = np.cumsum(P / P.sum())
        for t in range(ns):
            if gpair[q, t] != opair[q, t]:
                assert np.min(np.abs(cdf - u[q, t, 0])) < 1e-5, (q, t, gpair[q, t], opair[q, t])
                ambiguous += 1
                continue
            if gv[q, t] != ov[q, t]:  # only at the cut locus |nu| = pi
                p = opair[q, t]
                r = draw_radius(pr["c"][p], pr["C"][p], u[q, t].astype(np.float64))
                assert abs(r - np.pi) < CUT_LOCUS_BAND, (q, t, gv[q, t], ov[q, t], r)
                ambiguous += 1
                continue
            if not ov[q, t]:
                assert np.all(gd[q, t] == 0) and gp[q, t] == 0
                continue
            a, b = gd[q, t].astype(np.float64), od[q, t]
            ang = np.arctan2(np.linalg.norm(np.cross(a, b)), a @ b)
            rel = abs(gp[q, t] - op[q, t]) / op[q, t]
            stats["ang"] = max(stats.get("ang", 0.0), ang)
            stats["pdf"] = max(stats.get("pdf", 0.0), rel)
            assert ang < DIR_TOL, (q, t, ang)
            assert rel < PDF_RTOL, (q, t, gp[q, t], op[q, t])
    return ambiguous


def test_product_sample_parity_with_caller_uniforms(dev, orc, scene):
    print("case: product sampling, 27 cells x 8 queries x 8 draws, 3 BSDF models (Kb = 8)", flush=True)
    sc = scene
    nq, ns = sc["qcell"].size, 8
    g = _gpu_inputs(dev, sc)
    u = synth.make_uniforms(41, nq * ns).reshape(nq, ns, 3)
    stats = {}
    amb = _compare(orc, sc, u, _gpu_sample(dev, sc, g, ns, uniforms=u), stats)
    print("worst direction angle %.2e rad, worst pdf relative %.2e, ambiguous %d" %
          (stats["ang"], stats["pdf"], amb))
    assert amb <= max(2, nq * ns // 100), amb


def test_product_device_generator_matches_the_oracle_generator(dev, orc, scene):
    print("case: product sampling with the device Philox generator", flush=True)
    sc = scene
    nq, ns = sc["qcell"].size, 4
    g = _gpu_inputs(dev, sc)
    seed = 0xFEED_0123_4567
    got = _gpu_sample(dev, sc, g, ns, uniforms=None, seed=seed)
    u = orc.draw_uniforms(seed, nq * ns).astype(np.float32).reshape(nq, ns, 3)
    again = _gpu_sample(dev, sc, g, ns, uniforms=u)
    for a, b in zip(got, again):
        assert np.array_equal(a, b)
    _compare(orc, sc, u, got, {})


def test_product_pdf_parity(dev, orc, scene):
    print("case: product pdf, 216 queries x 16 directions", flush=True)
    from paper_2111_13094_amd import sdmm
    sc = scene
    nq, nd = sc["qcell"].size, 16
    g = _gpu_inputs(dev, sc)
    rng = np.random.default_rng(7)
    d = rng.normal(size=(nq, nd, 3))
    # half of them near the sampled directions, where the density lives
    u = synth.make_uniforms(43, nq * 8).reshape(nq, 8, 3)
    od, _, _, ov = orc.product_sample(*_orc_args(sc), u.astype(np.float64))
    d[:, :8] = od + 0.05 * rng.normal(size=(nq, 8, 3))
    d[:, :8][~ov.astype(bool)] = rng.normal(size=(int((~ov.astype(bool)).sum()), 3))
    d = (d / np.linalg.norm(d, axis=-1, keepdims=True)).astype(np.float32)
    gd = dev.from_numpy(np.ascontiguousarray(d.reshape(-1, 3).T)).cuda()
    got = sdmm.product_pdf(g["table"], sc["C"], sc["K"], g["qpos"], g["qcell"], g["btable"], sc["CB"], sc["Kb"],
                           g["bpar"], g["bcell"], g["frames"], gd).cpu().numpy().reshape(nq, nd)
    ref = orc.product_pdf(*_orc_args(sc), d.astype(np.float64))
    worst = 0.0
    for q in range(nq):
        if _ambiguous_query(orc, sc, q):
            continue
        big = ref[q] > 1e-6 * ref[q].max()
        rel = np.abs(got[q][big] - ref[q][big]) / ref[q][big]
        worst = max(worst, rel.max())
        assert rel.max() < PDF_RTOL, (q, rel.max())
        assert np.all(np.abs(got[q][~big]) <= 2e-6 * ref[q].max())
    print("worst pdf relative %.2e" % worst)


@pytest.mark.parametrize("K,Kb,ns", [(5, 12, 6), (32, 3, 6), (16, 1, 6), (4, 3, 4), (6, 8, 3), (16, 16, 20),
                                     (64, 2, 1)])
def test_product_other_component_counts(dev, orc, K, Kb, ns):
    """K not a power of two with more BSDF than radiance lanes, a 32-lane group with a
    3-component BSDF model, a single BSDF component (the second pair is empty), groups of
    4, 8 and 64 lanes, and more draws per query than one wave pass holds (the kernel that
    draws on the query's own lanes)."""
    print(f"case: product sampling K={K} Kb={Kb} ns={ns}", flush=True)
    wl = synth.workload("single", seed=4)
    b = synth.make_batch(9, [4096], wl["box_lo"], wl["box_size"], wl["lobes"])
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)
    orc.fit(orc.Opts(K=K, iters=3), b.offsets, b.samples, mix, orc.new_state(1, K))
    qpos, qcell = synth.make_queries(3, wl["box_lo"], wl["box_size"], 48)
    qpos, qcell = qpos[:45], qcell[:45]  # a ragged last wave pass
    bpar, bcell, F = synth.bsdf_queries(5, qcell.size, 2)
    sc = dict(C=1, K=K, mix=mix, CB=2, Kb=Kb, bmix=synth.bsdf_mixtures(6, 2, Kb), qpos=qpos.astype(np.float32),
              qcell=qcell, bpar=bpar.astype(np.float32), bcell=bcell, F=F.astype(np.float32))
    nq = qcell.size
    g = _gpu_inputs(dev, sc)
    u = synth.make_uniforms(44 + K, nq * ns).reshape(nq, ns, 3)
    got = _gpu_sample(dev, sc, g, ns, uniforms=u)
    amb = _compare(orc, sc, u, got, {})
    assert amb <= max(2, nq * ns // 100), amb
    if Kb == 1:
        pair = got[3]
        assert np.all(pair[got[2] == 1] % 2 == 0)


def test_product_invalid_indices_give_zero(dev, orc, scene):
    print("case: product sampling with out-of-range cell and model indices", flush=True)
    from paper_2111_13094_amd import sdmm
    sc = dict(scene)
    nq = 8
    for key in ("qpos", "qcell", "bpar", "bcell", "F"):
        sc[key] = sc[key][:nq].copy()
    sc["qcell"][[1, 4]] = -1
    sc["qcell"][2] = sc["C"]
    sc["bcell"][[5, 6]] = [sc["CB"], -3]
    g = _gpu_inputs(dev, sc)
    d, p, v, pr = _gpu_sample(dev, sc, g, 4, uniforms=None, seed=3)
    bad = [1, 2, 4, 5, 6]
    assert not v[bad].any() and np.all(p[bad] == 0) and np.all(d[bad] == 0) and np.all(pr[bad] == -1)
    assert v[[0, 3, 7]].sum() >= 8
    gd = dev.from_numpy(np.ascontiguousarray(np.tile([[0.0], [0.0], [1.0]], (1, nq * 2)).astype(np.float32))).cuda()
    pdf = sdmm.product_pdf(g["table"], sc["C"], sc["K"], g["qpos"], g["qcell"], g["btable"], sc["CB"], sc["Kb"],
                           g["bpar"], g["bcell"], g["frames"], gd).cpu().numpy().reshape(nq, 2)
    assert np.all(pdf[bad] == 0)


def test_product_full_size_sampled_queries(dev, orc):
    """The launch configuration of the product benchmark: 16384 radiance cells (the
    initial mixtures, K = 16), 8 BSDF models of 16 components, 2^22 queries, 4 draws
    each; 48 sampled queries recomputed by the oracle."""
    print("case: product sampling at full size (2^22 queries), 48 sampled queries", flush=True)
    wl = synth.workload("cells16k")
    C = wl["grid"].n_cells
    mix = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    qpos, qcell = synth.make_queries(5, wl["box_lo"], wl["box_size"], 256)
    nq = qcell.size
    assert nq == 1 << 22
    bpar, bcell, F = synth.bsdf_queries(6, nq, 8)
    sc = dict(C=C, K=16, mix=mix, CB=8, Kb=16, bmix=synth.bsdf_mixtures(7, 8, 16), qpos=qpos.astype(np.float32),
              qcell=qcell, bpar=bpar.astype(np.float32), bcell=bcell, F=F.astype(np.float32))
    ns = 4
    g = _gpu_inputs(dev, sc)
    seed = 99
    gd, gp, gv, gpair = _gpu_sample(dev, sc, g, ns, uniforms=None, seed=seed)
    pick = np.random.default_rng(1).choice(nq, 48, replace=False)
    u_all = orc.draw_uniforms(seed, nq * ns)  # the device generator's uniforms
    sub = {k: (v[pick] if k in ("qpos", "qcell", "bpar", "bcell", "F") else v) for k, v in sc.items()}
    u = u_all.reshape(nq, ns, 3)[pick].astype(np.float32)
    amb = _compare(orc, sub, u, (gd[pick], gp[pick], gv[pick], gpair[pick]), {})
    assert amb <= 2, amb
