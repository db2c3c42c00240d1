"""Benchmark of the spatio-directional mixture EM on one MI355X.

Headline (default): EM sample x component updates per second on the 4096-cell workload
(16^3 cells of the unit cube, K = 16, cell counts lognormal(6.45, 1) clipped to
[64, 8192], about 4.2M samples per batch, 8 resident batches, stepwise EM with decay 0.9:
eta = 0.1 after the first batch), batched schedule (one E launch and one M launch per
batch over all cells; each call's last M-step writes the next call's E-step mirrors, so
after the first call no setup kernel runs) in the launch configuration the autotuner picks
on the first batch, replayed through the library's hipGraph cache.
A step is one E+M pass over one resident batch; inputs are generated on the host and
copied to HBM before the timed region. The default warm-up (200 untimed steps, about
40 ms) lets the GPU clock settle: from an idle GPU the E kernel takes about 200 us for
its first steps and settles near 150 us after some 200 steps. The autotuner times its
candidates after as many untimed steps on scratch copies of the mixtures. The same steps launched eagerly, with HIP events
around every E-step and M-step launch, give the roofline's kernel time ("eager").

The JSON line also carries:
  roofline      the E-step statistics kernel (the dominant kernel): algorithmic FP32
                flops per launch (140 per sample-component pair) over its average
                event-timed duration, against the FP32 vector peak; its
                measured_ceiling is the FMA rate the chip sustains for code built like
                the library's (sdmm_probe_fma, no packed FP32), measured after the timed
                region, with the kernel's rate as a fraction of it;
  plain         the same updates/s for the plain per-cell GPU EM (one E and one M launch
                per cell), same tolerance;
  cpu_baseline  the FP64 oracle, single thread, on a bounded sample of the workload, and
                its OpenMP build over cells on all host cores ("all_cores").

Other workloads (--workload), each printing its own line: single (1 cell, N = 16384,
20 iterations, hipGraph), cells16k (16384 cells, geometric counts, then 2^22 query
positions x 4 draws through the fused conditioning + sampling + pdf kernel), product
(the same queries, product-sampled with a conditioned 16-component BSDF mixture), huge
(1 cell, 2^24 samples, K = 32, the three running-sum variants), grad (the adjoint on
the 4096-cell state after 8 batches, plus 10 refinement steps), accurate (the two-pass
covariance update), stepwise (per-sample EM on the 4096-cell batches), tree (kD-tree
refinement of the cells16k samples; its roofline is the first-round point location,
with the HBM traffic of the committed counter summary while the tree source is
unchanged). --sweep times launch configurations of the headline workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# launch configurations the headline run lets the autotuner choose from (batched schedule:
# work-item size, waves per work group)
TUNE_CANDIDATES = [{"schedule": 0, "min_range": p, "waves_per_block": w} for p in (256, 512, 1024) for w in (1, 2)]

FLOPS_PER_PAIR = 140.0       # algorithmic FP32 flops per (sample, component) per E+M pass
FP32_PEAK_TFLOPS = 157.3     # MI355X vector FP32 (published)
HBM_PEAK_GBS = 8000.0


def _kernel_source_hash(files=("estep.hpp", "device_math.hpp", "fit.hip")):
    """Hash of the code (comment lines and trailing comments dropped) of the sources that
    build a kernel (by default the E-step's), so that a counter record names the kernel it
    was taken on."""
    h = hashlib.sha256()
    for f in files:
        for line in open(os.path.join(ROOT, "paper_2111_13094_amd", "csrc", f)):
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def _traffic_record(items, waves_per_block):
    """HBM bytes per launch of the E-step kernel from the committed counter summary, if
    it was taken on the current kernel source in the launch configuration timed here
    (work-item size, waves per work group); else None."""
    path = os.path.join(ROOT, "profiles", "estep_cells4k_traffic.json")
    try:
        data = json.load(open(path))
    except (OSError, ValueError):
        return None
    if data.get("source_hash") != _kernel_source_hash():
        return None
    for rec in data.get("records", []):
        if rec.get("items") == items and rec.get("waves_per_block") == waves_per_block:
            return rec.get("bytes_per_launch")
    return None


def _tree_traffic_record():
    """HBM bytes per launch of the first-round point location of the tree workload from
    the committed counter summary, if it was taken on the current tree source; else None."""
    path = os.path.join(ROOT, "profiles", "tree_locate_traffic.json")
    try:
        data = json.load(open(path))
    except (OSError, ValueError):
        return None
    if data.get("source_hash") != _kernel_source_hash(("tree.hip", "common.hpp")):
        return None
    return data.get("bytes_per_launch")


def _copy_probe(torch, dev, mib):
    """A plain device copy of known size, to scale the HBM byte counters of a profiler run."""
    src = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    _sync(torch)
    return src.numel() * 4


def _estep_kernel_name(items, G=16, adjoint=False):
    """The E-step kernel the library launches for the compensated sums (of the EM pass, or
    of the adjoint's pass): items whose lane share fits one fold block (64 steps of 64 / G
    samples) run the plain-sum kernel, bit for bit the same."""
    acc = 1 if items // (64 // G) <= 64 else 0
    return f"estep_kernel<{G}, {acc}, false, {'true' if adjoint else 'false'}>"


def _sync(torch):
    torch.cuda.synchronize()


_GEN_CACHE = {}


def _gen_cells4k(n_batches):
    from paper_2111_13094_amd import synth
    if n_batches not in _GEN_CACHE:
        wl = synth.workload("cells4k")
        _GEN_CACHE[n_batches] = (wl, [synth.workload_batch(wl, j) for j in range(n_batches)])
    return _GEN_CACHE[n_batches]


def cpu_baseline(wl, batch, target_s=12.0, orc_kw=None):
    """The oracle (single thread, FP64) on a bounded sample of the workload: a subset of
    cells of one batch, one E+M step each, sized to about target_s seconds."""
    orc_kw = {"eta": 0.1} if orc_kw is None else orc_kw
    from oracle import oracle as orc
    from paper_2111_13094_amd import synth
    C = wl["grid"].n_cells
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    rng = np.random.default_rng(0)
    order = rng.permutation(C)

    def run(cells):
        pairs, t = 0, 0.0
        for c in cells:
            i0, i1 = batch.offsets[c], batch.offsets[c + 1]
            sub = np.ascontiguousarray(batch.samples[:, i0:i1])
            mc = {k: np.ascontiguousarray(v.reshape(C, -1)[c]) for k, v in mix0.items()}
            st = orc.new_state(1, 16)
            t0 = time.perf_counter()
            orc.fit(orc.Opts(K=16, **orc_kw), np.array([0, i1 - i0]), sub, mc, st)
            t += time.perf_counter() - t0
            pairs += (i1 - i0) * 16
        return pairs, t

    p0, t0 = run(order[:16])
    n = int(min(C - 16, max(16, 16 * target_s / max(t0, 1e-3))))
    p1, t1 = run(order[16:16 + n])
    pairs, t = p0 + p1, t0 + t1
    return {"value": pairs / t, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{16 + n} of {C} cells of one batch, one E+M step each, FP64, single thread, {t:.1f} s",
            "host": host_description()}


def host_description():
    """nproc, the CPUs this process may run on, and the CPU model."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline_all_cores(wl, batches, target_s=12.0, orc_kw=None):
    """The same oracle source built with OpenMP over cells, on every CPU this process
    may use (capped by OMP_NUM_THREADS when set): whole batches, one E+M step each from
    the initial mixtures, repeated over the resident batches until about target_s
    seconds of wall time have passed."""
    orc_kw = {"eta": 0.1} if orc_kw is None else orc_kw
    from oracle import oracle as orc
    from paper_2111_13094_amd import synth
    C = wl["grid"].n_cells
    want = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        want = min(want, int(os.environ["OMP_NUM_THREADS"]))
    threads = orc.threads_in_use(want)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    pairs, t, nb = 0, 0.0, 0
    while t < target_s and nb < 4 * len(batches):
        b = batches[nb % len(batches)]
        mix, st = synth.copy_mix(mix0), orc.new_state(C, 16)
        t0 = time.perf_counter()
        orc.fit(orc.Opts(K=16, **orc_kw), b.offsets, b.samples, mix, st, threads=threads)
        t += time.perf_counter() - t0
        pairs += b.samples.shape[1] * 16
        nb += 1
    return {"value": pairs / t, "unit": "updates/s", "cores": threads, "kind": "oracle (OpenMP over cells)",
            "sample": f"{nb} whole batches of {C} cells, one E+M step each, FP64, {threads} threads, {t:.1f} s"}


def measured_ceiling(torch, bits, achieved):
    """The vector FMA rate the chip reaches for code built like the library's kernels
    (sdmm_probe_fma: FP32 without packed instructions, or FP64), best of three runs after
    a warm-up, and the kernel's achieved rate as a fraction of it. Measured after the timed
    region; the published peak stays the roofline's `peak`."""
    from paper_2111_13094_amd import sdmm
    sdmm.probe_fma(bits)
    best = max(sdmm.probe_fma(bits) for _ in range(3))
    return {"kind": "fp32 FMA, no packed instructions" if bits == 32 else "fp64 FMA", "value": best,
            "unit": "TFLOP/s", "frac": (achieved / best) if achieved else None}


def measured_copy_rate(torch, achieved, mib=1024):
    """HBM rate of a plain device copy of `mib` MiB (read + write bytes over the event-timed
    copy), best of three after a warm-up, and the kernel's achieved rate as a fraction of
    it. Measured after the timed region."""
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = 0.0
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = max(best, 2 * src.numel() * 4 / (a.elapsed_time(b) * 1e-3) / 1e9)
    return {"kind": "device copy (read + write)", "value": best, "unit": "GB/s",
            "frac": (achieved / best) if achieved else None}


def bench_cells4k(args, torch):
    from paper_2111_13094_amd import sdmm, synth
    n_batches = 8
    wl, batches = _gen_cells4k(n_batches)
    C, K = wl["grid"].n_cells, 16
    dev = torch.device("cuda", 0)
    offs = [torch.from_numpy(b.offsets).to(dev) for b in batches]
    smps = [torch.from_numpy(b.samples).to(dev) for b in batches]
    N = [b.samples.shape[1] for b in batches]
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)

    def fresh():
        return {k: torch.from_numpy(v).to(dev) for k, v in mix0.items()}, sdmm.new_state(C, K, dev)

    opts = sdmm.default_opts(K, eta=0.1, schedule=sdmm.SCHED_FUSED if args.schedule == "fused" else sdmm.SCHED_BATCHED)
    if args.min_range:
        opts.min_range = args.min_range
    if args.max_ranges:
        opts.max_ranges = args.max_ranges
    if args.wpb:
        opts.waves_per_block = args.wpb
    opts.flags = {"twosum": 0, "plain": sdmm.FLAG_PLAIN_FP32, "fp64": sdmm.FLAG_FP64_SUMS}[args.sums]
    # the caller's bound on samples per cell (the largest cell of its batches, from the
    # host-side offsets): with at most 8192 samples no cell needs the record tree, so
    # its launches are left out
    max_cell = max(int(np.diff(b.offsets).max()) for b in batches)
    opts.max_cell_samples = max_cell
    tuned = None
    if args.tune:
        # the autotuner's pick on the first batch (untimed); the timed runs use it. It times
        # its candidates after the same number of untimed steps on scratch copies, so that
        # every candidate runs at the settled clock
        from paper_2111_13094_amd import tune
        m_w, s_w = fresh()
        for w in range(args.warmup):
            sdmm.fit_mixtures(offs[w % n_batches], smps[w % n_batches], m_w, s_w, opts)
        del m_w, s_w
        m_t, s_t = fresh()
        opts = tune.tune_fit(offs[0], smps[0], m_t, s_t, opts, candidates=TUNE_CANDIDATES, reps=3)
        cfg = tune.tuned_config(C, K, N[0], opts)
        tuned = {"items": int(opts.min_range), "waves_per_block": int(opts.waves_per_block or 1),
                 "e_plus_m_ms": cfg["ms"] if cfg else None, "candidates": len(TUNE_CANDIDATES)}
        del m_t, s_t
    if args.carry:
        # a fitting loop whose mixtures change only through its own calls: each call's
        # last M-step writes the next call's E-step mirrors, so no setup kernel runs
        opts.flags |= sdmm.FLAG_CARRY_MIRRORS
    status = torch.empty(C, dtype=torch.int32, device=dev)
    ws = torch.empty(max(sdmm.workspace_bytes(C, K, n, opts) for n in N), dtype=torch.uint8, device=dev)
    mix, st = fresh()
    L = sdmm.lib()
    import ctypes as C_

    def run(o, steps, events):
        """steps E+M steps over the resident batches (after the warm-up's), timed by the
        wall clock between two device synchronisations; with events, the library's own
        HIP events around every E-step and M-step launch."""
        tot, cnt, mtot, mcnt = C_.c_double(), C_.c_int64(), C_.c_double(), C_.c_int64()
        if events:
            L.sdmm_timing_enable(1)
            L.sdmm_timing_read(0, C_.byref(tot), C_.byref(cnt), 1)
            L.sdmm_timing_read(1, C_.byref(mtot), C_.byref(mcnt), 1)
        _sync(torch)
        t0 = time.perf_counter()
        npairs = 0
        for s_ in range(steps):
            j = (args.warmup + s_) % n_batches
            sdmm.fit_mixtures(offs[j], smps[j], mix, st, o, status, ws)
            npairs += N[j] * K
        _sync(torch)
        wall = time.perf_counter() - t0
        e_ms = m_ms = None
        if events:
            L.sdmm_timing_read(0, C_.byref(tot), C_.byref(cnt), 1)
            L.sdmm_timing_read(1, C_.byref(mtot), C_.byref(mcnt), 1)
            L.sdmm_timing_enable(0)
            e_ms = tot.value / max(cnt.value, 1)
            m_ms = mtot.value / max(mcnt.value, 1) if mcnt.value else None
        return npairs, wall, e_ms, m_ms

    for w in range(args.warmup):
        sdmm.fit_mixtures(offs[w % n_batches], smps[w % n_batches], mix, st, opts, status, ws)
    # eager launches with event timing: the E-step kernel's duration for the roofline
    epairs, ewall, est_ms, m_ms = run(opts, args.steps, True)
    # the headline: the same launches replayed through the library's hipGraph cache (one
    # graph per batch, all captured before the timed region; a replay records no events)
    gopts = sdmm.FitOpts.from_buffer_copy(opts)
    gopts.use_graph = 1 if args.graph else 0
    if args.graph:
        for j in range(n_batches):
            sdmm.fit_mixtures(offs[j], smps[j], mix, st, gopts, status, ws)
    pairs, wall, _, _ = run(gopts, args.steps, False)
    value = pairs / wall
    flops_per_launch = FLOPS_PER_PAIR * (epairs / args.steps)
    achieved = flops_per_launch / (est_ms * 1e-3) / 1e12
    items, wpb = int(opts.min_range or 256), int(opts.waves_per_block or 1)
    traffic = _traffic_record(items, wpb)
    out = {
        "metric": "EM sample x component updates/s, 4096 cells K=16 (batched)",
        "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "cells4k: 4096 cells (16^3 grid of the unit cube), K=16, counts "
                               "lognormal(6.45,1) clipped to [64,8192], 8 resident batches, stepwise EM "
                               "eta=0.1, FP32 E-step with compensated sums, FP64 M-step",
                   "n_cells": C, "K": K, "samples_per_batch": int(np.mean(N)), "batches": n_batches,
                   "schedule": "fused" if opts.schedule == sdmm.SCHED_FUSED else "batched",
                   "min_range": items, "max_ranges": int(opts.max_ranges or 65536), "waves_per_block": wpb,
                   "hipgraph": bool(args.graph), "carried_mirrors": bool(args.carry), "running_sums": args.sums,
                   "max_cell_samples": max_cell,
                   "autotuned": tuned},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": ("fused_kernel<16, 0, false>" if opts.schedule == sdmm.SCHED_FUSED
                                else _estep_kernel_name(items)),
                     "kernel_ms": est_ms, "flops_per_launch": flops_per_launch},
        "mstep_ms": m_ms,
        "eager": {"value": epairs / ewall, "unit": "updates/s", "ms_per_step": ewall * 1e3 / args.steps},
    }
    if not args.no_plain:
        popts = sdmm.default_opts(K, eta=0.1, schedule=sdmm.SCHED_PER_CELL)
        ws = torch.empty(max(sdmm.workspace_bytes(C, K, n, popts) for n in N), dtype=torch.uint8, device=dev)
        pmix, pst = fresh()
        sdmm.fit_mixtures(offs[0], smps[0], pmix, pst, popts, status, ws)
        _sync(torch)
        t0 = time.perf_counter()
        psteps = 2
        ppairs = 0
        for s in range(psteps):
            j = (1 + s) % n_batches
            sdmm.fit_mixtures(offs[j], smps[j], pmix, pst, popts, status, ws)
            ppairs += N[j] * K
        _sync(torch)
        pt = time.perf_counter() - t0
        out["plain"] = {"value": ppairs / pt, "unit": "updates/s", "ms_per_step": pt * 1e3 / psteps,
                        "speedup_batched_over_plain": value / (ppairs / pt)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, batches[0], target_s=args.cpu_seconds)
        out["cpu_baseline"]["all_cores"] = cpu_baseline_all_cores(wl, batches, target_s=args.cpu_seconds)
    if args.copy_probe:
        out["copy_probe_bytes"] = _copy_probe(torch, dev, args.copy_probe_mib)
    return out


def bench_accurate(args, torch):
    """Batch EM (eta = 1) with the accurate covariance update on the 4096-cell batches:
    per step one E-step pass, the weight and mean update, a second E-step pass in the new
    tangent spaces and the covariance update. The first-order update on the same steps is
    timed beside it. The roofline is that of the E-step kernel over both of its launches."""
    from paper_2111_13094_amd import sdmm, synth
    import ctypes as C_
    n_batches = 8
    wl, batches = _gen_cells4k(n_batches)
    C, K = wl["grid"].n_cells, 16
    dev = torch.device("cuda", 0)
    offs = [torch.from_numpy(b.offsets).to(dev) for b in batches]
    smps = [torch.from_numpy(b.samples).to(dev) for b in batches]
    N = [b.samples.shape[1] for b in batches]
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)
    status = torch.empty(C, dtype=torch.int32, device=dev)
    L = sdmm.lib()

    def run(flags):
        opts = sdmm.default_opts(K, flags=flags)
        ws = torch.empty(max(sdmm.workspace_bytes(C, K, n, opts) for n in N), dtype=torch.uint8, device=dev)
        mix = {k: torch.from_numpy(v).to(dev) for k, v in mix0.items()}
        st = sdmm.new_state(C, K, dev)
        for w in range(args.warmup):
            sdmm.fit_mixtures(offs[w % n_batches], smps[w % n_batches], mix, st, opts, status, ws)
        _sync(torch)
        L.sdmm_timing_enable(1)
        tot, cnt = C_.c_double(), C_.c_int64()
        for cls in range(5):
            L.sdmm_timing_read(cls, C_.byref(tot), C_.byref(cnt), 1)
        _sync(torch)
        t0 = time.perf_counter()
        pairs = 0
        for s_ in range(args.steps):
            j = (args.warmup + s_) % n_batches
            sdmm.fit_mixtures(offs[j], smps[j], mix, st, opts, status, ws)
            pairs += N[j] * K
        _sync(torch)
        wall = time.perf_counter() - t0
        ms, e_tot, e_cnt = {}, 0.0, 0
        for cls, name in ((0, "estep"), (1, "mstep"), (4, "second_pass")):
            L.sdmm_timing_read(cls, C_.byref(tot), C_.byref(cnt), 1)
            ms[name] = tot.value / cnt.value if cnt.value else None
            if cls in (0, 4):
                e_tot, e_cnt = e_tot + tot.value, e_cnt + cnt.value
        ms["estep_kernel_avg"] = e_tot / max(e_cnt, 1)
        L.sdmm_timing_enable(0)
        return pairs, wall, ms

    pairs, wall, ms = run(sdmm.FLAG_ACCURATE_SIGMA)
    fpairs, fwall, fms = run(0)
    # how far the first-order covariance lands from the accurate one after one step from
    # the initial mixtures (relative Frobenius distance per component)
    covs = {}
    for flags in (sdmm.FLAG_ACCURATE_SIGMA, 0):
        mix = {k: torch.from_numpy(v).to(dev) for k, v in mix0.items()}
        sdmm.fit_mixtures(offs[0], smps[0], mix, sdmm.new_state(C, K, dev), sdmm.default_opts(K, flags=flags), status)
        covs[flags] = mix["cov"].reshape(-1, 15).double()
    tri_w = torch.tensor([1.0 if d == e else 2.0 for d in range(5) for e in range(d + 1)], device=dev,
                         dtype=torch.float64)
    diff = ((covs[0] - covs[sdmm.FLAG_ACCURATE_SIGMA]) ** 2 * tri_w).sum(1).sqrt()
    ref = ((covs[sdmm.FLAG_ACCURATE_SIGMA] ** 2) * tri_w).sum(1).sqrt()
    rel = (diff / ref).cpu().numpy()
    per_launch = pairs / args.steps
    achieved = FLOPS_PER_PAIR * per_launch / (ms["estep_kernel_avg"] * 1e-3) / 1e12
    out = {
        "metric": "EM sample x component updates/s, 4096 cells K=16, batch EM with the accurate covariance update",
        "value": pairs / wall, "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "accurate: the 4096-cell batches (lognormal(6.45,1) counts clipped to "
                               "[64,8192]), batch EM (eta=1) from the initial mixtures, one iteration per "
                               "step with the second pass in the new tangent spaces",
                   "n_cells": C, "K": K, "samples_per_batch": int(np.mean(N)), "batches": n_batches},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                     "kernel": _estep_kernel_name(256), "kernel_ms": ms["estep_kernel_avg"],
                     "flops_per_launch": FLOPS_PER_PAIR * per_launch},
        "kernel_ms": ms,
        "first_order": {"value": fpairs / fwall, "unit": "updates/s", "ms_per_step": fwall * 1e3 / args.steps,
                        "kernel_ms": fms,
                        "cov_rel_distance_after_one_step": {"median": float(np.median(rel)),
                                                            "p90": float(np.quantile(rel, 0.9)),
                                                            "max": float(rel.max())}},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, batches[0], target_s=args.cpu_seconds,
                                           orc_kw={"eta": 1.0, "accurate_sigma": 1})
    return out


def query_flops(K, ns):
    """Algorithmic FP32 flops of the fused conditioning + sampling + pdf path per query
    (an FMA counts 2): conditioning 31 per component (offset 3, L_xx^-1 d 9, |u|^2 5,
    m = A d 10, log weight 1, softmax 3); per draw the component CDF (K), one candidate
    (Box-Muller 4, nu = m + L' z 6, exp map 25, validity 3) and the pdf of the whole
    mixture at the drawn direction, 56 per component (rotation 15, log map 25, |nu|^2 3,
    nu - m 2, L'^-1 5, quadratic form 3, weight x exp x 1/sinc 2, sum 1)."""
    return 31 * K + ns * (K + 38 + 56 * K)


def bench_cells16k(args, torch):
    """Conditioning + sampling + pdf on the 16384-cell workload (32x32x16 cells of the unit
    cube, K = 16, geometric counts, 2^22 query positions sorted by cell, 4 draws each with
    the device Philox generator), after one batched E+M step on the workload's samples."""
    import ctypes as C_
    from paper_2111_13094_amd import sdmm, synth
    wl = synth.workload("cells16k")
    b = synth.workload_batch(wl)
    C, K, ns = wl["grid"].n_cells, 16, 4
    dev = torch.device("cuda", 0)
    off, smp = torch.from_numpy(b.offsets).to(dev), torch.from_numpy(b.samples).to(dev)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)
    mix = {k: torch.from_numpy(v).to(dev) for k, v in mix0.items()}
    st = sdmm.new_state(C, K, dev)
    opts = sdmm.default_opts(K)
    status = sdmm.fit_mixtures(off, smp, mix, st, opts)
    _sync(torch)
    table = sdmm.condition_prepare(mix, C, K)
    qpos, qcell = synth.make_queries(7, wl["box_lo"], wl["box_size"], 256)
    nq = qcell.size
    qp = torch.from_numpy(np.ascontiguousarray(qpos.T)).to(dev)
    qc = torch.from_numpy(qcell).to(dev)
    out = (torch.empty(3, nq * ns, dtype=torch.float32, device=dev), torch.empty(nq * ns, dtype=torch.float32, device=dev),
           torch.empty(nq * ns, dtype=torch.uint8, device=dev))
    for w in range(args.warmup):
        sdmm.condition_sample_pdf(table, C, K, qp, qc, ns, seed=w, out=out)
    _sync(torch)
    t_fit = fit_time(args, torch, off, smp, mix0, C, K, opts)
    L = sdmm.lib()
    L.sdmm_timing_enable(1)
    tot, cnt = C_.c_double(), C_.c_int64()
    L.sdmm_timing_read(2, C_.byref(tot), C_.byref(cnt), 1)
    _sync(torch)
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        sdmm.condition_sample_pdf(table, C, K, qp, qc, ns, seed=1000 + s_, out=out)
    _sync(torch)
    wall = time.perf_counter() - t0
    L.sdmm_timing_read(2, C_.byref(tot), C_.byref(cnt), 1)
    L.sdmm_timing_enable(0)
    k_ms = tot.value / max(cnt.value, 1)
    fl = query_flops(K, ns) * nq
    achieved = fl / (k_ms * 1e-3) / 1e12
    valid_frac = float(out[2].float().mean().item())
    return {"metric": "guided draws/s (conditioning + sampling + pdf), 16384 cells K=16, 4 draws per query",
            "value": nq * ns * args.steps / wall, "unit": "draws/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "cells16k: 16384 cells (32x32x16), K=16, counts 16+Geom(1/1009)-1 clipped to "
                                   "[16,32768], 2^22 query positions (256 per cell), 4 draws each (Philox4x32-10), "
                                   "fused conditioning + sampling + pdf after one E+M step",
                       "n_cells": C, "K": K, "queries": nq, "draws_per_query": ns,
                       "samples": int(smp.shape[1]), "valid_fraction": valid_frac,
                       "fitted_cells": int(((status.cpu().numpy() & (1 | 2 | 4 | 32)) == 0).sum())},
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                         "kernel": ("cond_sample_pdf_lanes_kernel<16>" if (64 // 16) * ns <= 64
                                    else "cond_sample_pdf_kernel<16>"), "kernel_ms": k_ms, "flops_per_launch": fl},
            "fit": {"value": smp.shape[1] * K / t_fit, "unit": "updates/s", "ms_per_step": t_fit * 1e3}}


def product_flops(K, Kb, ns):
    """Algorithmic FP32 flops of product sampling per query (an FMA counts 2): conditioning
    of both mixtures, 31 per component; the two kept BSDF components rotated to world
    and prepared, 171 each (mean 15, frame 12, in-plane rotation 50, offset and covariance
    28, centre and exp-map Jacobian 66); per pair (2K of them) 217 (centre in the tangent
    space 40, log-map Jacobian 13, transfer 50, J S J^T 21, weight 25, product mean and
    covariance 51, Cholesky factor, inverse and normaliser 17) and 3 to normalise; per
    draw the pair CDF (2K), one candidate (Box-Muller 6, nu 5, exp map 25, validity 3) and
    the density, 71 per radiance component (rotation 15, log map 25, |nu|^2 3, two
    quadratic forms with weight 26, 1/sinc and sum 2)."""
    return 31 * K + 31 * Kb + 2 * 171 + 2 * K * (217 + 3) + ns * (2 * K + 39 + 71 * K)


def bench_product(args, torch):
    """Product sampling with a conditioned BSDF mixture on the 16384-cell workload: the
    radiance mixtures after one batched E+M step (as cells16k), a BSDF model (16
    components over incident direction, outgoing polar angle, azimuth and roughness)
    fitted by the same EM to 2^20 GGX training samples, then 2^22 queries (positions
    sorted by cell, random BSDF inputs and shading frames) x 4 draws with the device
    Philox generator, timed."""
    import ctypes as C_
    from paper_2111_13094_amd import sdmm, synth
    wl = synth.workload("cells16k")
    b = synth.workload_batch(wl)
    C, K, Kb, ns = wl["grid"].n_cells, 16, 16, 4
    dev = torch.device("cuda", 0)
    off, smp = torch.from_numpy(b.offsets).to(dev), torch.from_numpy(b.samples).to(dev)
    mix = {k: torch.from_numpy(v).to(dev) for k, v in synth.initial_mixtures(wl["box_lo"], wl["box_size"], K).items()}
    sdmm.fit_mixtures(off, smp, mix, sdmm.new_state(C, K, dev), sdmm.default_opts(K))
    table = sdmm.condition_prepare(mix, C, K)
    # the BSDF model, fitted like any cell
    tb = synth.ggx_training_batch(17, 1 << 20)
    lo, hi = synth.BSDF_PAR_LO[None], synth.BSDF_PAR_HI[None]
    bmix = {k: torch.from_numpy(v).to(dev) for k, v in synth.initial_mixtures(lo, hi - lo, Kb).items()}
    bst = sdmm.fit_mixtures(torch.from_numpy(tb.offsets).to(dev), torch.from_numpy(tb.samples).to(dev), bmix,
                            sdmm.new_state(1, Kb, dev), sdmm.default_opts(Kb, iters=40))
    btable = sdmm.condition_prepare(bmix, 1, Kb)
    qpos, qcell = synth.make_queries(7, wl["box_lo"], wl["box_size"], 256)
    nq = qcell.size
    bpar, bcell, F = synth.bsdf_queries(8, nq, 1)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).astype(dt)).to(dev)
    qp, qc = t(qpos.T, np.float32), t(qcell, np.int32)
    bp, bc, fr = t(bpar.T, np.float32), t(bcell, np.int32), t(F.reshape(nq, 9).T, np.float32)
    out = (torch.empty(3, nq * ns, dtype=torch.float32, device=dev), torch.empty(nq * ns, dtype=torch.float32, device=dev),
           torch.empty(nq * ns, dtype=torch.uint8, device=dev), None)
    for w in range(args.warmup):
        sdmm.product_sample(table, C, K, qp, qc, btable, 1, Kb, bp, bc, fr, ns, seed=w, out=out)
    _sync(torch)
    L = sdmm.lib()
    L.sdmm_timing_enable(1)
    tot, cnt = C_.c_double(), C_.c_int64()
    L.sdmm_timing_read(5, C_.byref(tot), C_.byref(cnt), 1)
    _sync(torch)
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        sdmm.product_sample(table, C, K, qp, qc, btable, 1, Kb, bp, bc, fr, ns, seed=1000 + s_, out=out)
    _sync(torch)
    wall = time.perf_counter() - t0
    L.sdmm_timing_read(5, C_.byref(tot), C_.byref(cnt), 1)
    L.sdmm_timing_enable(0)
    k_ms = tot.value / max(cnt.value, 1)
    fl = product_flops(K, Kb, ns) * nq
    achieved = fl / (k_ms * 1e-3) / 1e12
    return {"metric": "product-sampled draws/s (radiance x BSDF mixture), 16384 cells K=16, BSDF Kb=16, "
                      "4 draws per query",
            "value": nq * ns * args.steps / wall, "unit": "draws/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "product: the cells16k radiance mixtures after one E+M step; one BSDF model "
                                   "(Kb=16) fitted by 40 EM iterations to 2^20 GGX training samples; 2^22 queries "
                                   "(256 per cell) with uniform BSDF inputs and random shading frames, 4 draws each "
                                   "(Philox4x32-10), pruned to 2 BSDF components",
                       "n_cells": C, "K": K, "Kb": Kb, "queries": nq, "draws_per_query": ns,
                       "valid_fraction": float(out[2].float().mean().item()),
                       "bsdf_fit_status": int(bst.cpu().numpy()[0])},
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                         "kernel": "product_sample_lanes_kernel<16>", "kernel_ms": k_ms, "flops_per_launch": fl}}


def bench_tree(args, torch):
    """One rendering iteration's tree work on the 16384-cell workload's samples (16.6M
    positions): refine a depth-3 pre-subdivided tree (512 leaves) with the paper's
    threshold c = 16000, initialise the leaves, reorder the samples by leaf; then one
    batched E+M step on the leaves. Each timed step starts from a fresh pre-subdivided
    tree (re-initialised before the step, outside the timed region)."""
    from paper_2111_13094_amd import sdmm, synth
    wl = synth.workload("cells16k")
    smp_np = synth.workload_batch(wl).samples
    dev = torch.device("cuda", 0)
    smp = torch.from_numpy(smp_np).to(dev)
    N, K, max_leaves, c = smp.shape[1], 16, 8192, 16000
    t = sdmm.new_tree(max_leaves)
    mix = {k: torch.zeros(max_leaves * K * n, dtype=torch.float64, device=dev)
           for k, n in (("pi", 1), ("mu_dir", 3), ("mu_pos", 3), ("cov", 15))}
    st = sdmm.new_state(max_leaves, K, dev)
    ws = torch.empty(sdmm.lib().sdmm_tree_workspace_size(N, max_leaves), dtype=torch.uint8, device=dev)
    opts = sdmm.default_opts(K)
    import ctypes as C_
    L_ = sdmm.lib()
    tot, cnt = C_.c_double(), C_.c_int64()
    refine_ms, fit_ms, leaves = [], [], 0
    for s_ in range(args.warmup + args.steps):
        if s_ == args.warmup:
            L_.sdmm_timing_enable(1)
            L_.sdmm_timing_read(6, C_.byref(tot), C_.byref(cnt), 1)
        sdmm.tree_init(t, 3, [0, 0, 0], [1, 1, 1])
        _sync(torch)
        t0 = time.perf_counter()
        srt, off, L, status = sdmm.tree_refine(t, smp, c, mix, st, K, workspace=ws)
        _sync(torch)
        t1 = time.perf_counter()
        view = {k: v[:L * (v.numel() // max_leaves)] for k, v in mix.items()}
        sview = {k: v[:L * (v.numel() // max_leaves)] for k, v in st.items()}
        sdmm.fit_mixtures(off, srt, view, sview, opts)
        _sync(torch)
        t2 = time.perf_counter()
        if s_ >= args.warmup:
            refine_ms.append((t1 - t0) * 1e3)
            fit_ms.append((t2 - t1) * 1e3)
        leaves = L
    L_.sdmm_timing_read(6, C_.byref(tot), C_.byref(cnt), 1)
    L_.sdmm_timing_enable(0)
    loc_ms = tot.value / max(cnt.value, 1)
    # the first locate launch walks every sample from the root: it reads 12 B of position
    # and writes the node and leaf index, 8 B, per sample
    loc_bytes = 20.0 * N
    achieved = loc_bytes / (loc_ms * 1e-3) / 1e9
    r_ms, f_ms = float(np.mean(refine_ms)), float(np.mean(fit_ms))
    traffic = _tree_traffic_record()
    extra = {"copy_probe_bytes": _copy_probe(torch, dev, args.copy_probe_mib)} if args.copy_probe else {}
    return {**extra,
            "metric": "kD-tree refinement: samples/s (locate, split rounds, reorder by leaf, initialise), "
                      "16.6M samples, c=16000",
            "value": N / (r_ms * 1e-3), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": r_ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "tree: the cells16k samples (32x32x16 grid counts, 16.6M) refined from a "
                                   "depth-3 pre-subdivided tree (512 leaves) with c=16000, K=16; wall time of "
                                   "the host call, which synchronises once per round",
                       "samples": N, "leaves": leaves, "max_leaves": max_leaves, "fit_after_refine_ms": f_ms},
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "locate_kernel (first round)",
                         "kernel_ms": loc_ms, "bytes_per_launch": loc_bytes}}


STEPWISE_FLOPS_PER_PAIR = 510.0  # FP64: the E-step's 140 + a per-sample M-step of about 370


def bench_stepwise(args, torch):
    """Stepwise (per-sample) EM on the 4096-cell batches: after a batch step on the first
    batch (untimed), each step is one per-sample pass over the next resident batch with
    the paper's Robbins-Monro schedule per sample; the mini-batch step on the same
    batches is timed beside it."""
    import ctypes as C_
    from paper_2111_13094_amd import sdmm, synth
    n_batches = 8
    wl, batches = _gen_cells4k(n_batches)
    C, K = wl["grid"].n_cells, 16
    dev = torch.device("cuda", 0)
    offs = [torch.from_numpy(b.offsets).to(dev) for b in batches]
    smps = [torch.from_numpy(b.samples).to(dev) for b in batches]
    N = [b.samples.shape[1] for b in batches]
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)
    L = sdmm.lib()
    tot, cnt = C_.c_double(), C_.c_int64()

    def run(schedule, steps, timer):
        opts = sdmm.default_opts(K, eta_mode=sdmm.ETA_PAPER, schedule=schedule)
        mix = {k: torch.from_numpy(v).to(dev) for k, v in mix0.items()}
        st = sdmm.new_state(C, K, dev)
        sdmm.fit_mixtures(offs[0], smps[0], mix, st, opts)  # the batch step of fresh cells
        _sync(torch)
        L.sdmm_timing_enable(1)
        L.sdmm_timing_read(timer, C_.byref(tot), C_.byref(cnt), 1)
        t0 = time.perf_counter()
        pairs = 0
        for s_ in range(steps):
            j = 1 + s_ % (n_batches - 1)
            sdmm.fit_mixtures(offs[j], smps[j], mix, st, opts)
            pairs += N[j] * K
        _sync(torch)
        wall = time.perf_counter() - t0
        L.sdmm_timing_read(timer, C_.byref(tot), C_.byref(cnt), 1)
        L.sdmm_timing_enable(0)
        return pairs, wall, tot.value / max(cnt.value, 1)

    pairs, wall, k_ms = run(sdmm.SCHED_STEPWISE, args.steps, 7)
    bpairs, bwall, _ = run(sdmm.SCHED_BATCHED, args.steps, 0)
    fl = STEPWISE_FLOPS_PER_PAIR * pairs / args.steps
    achieved = fl / (k_ms * 1e-3) / 1e12
    return {"metric": "stepwise EM sample x component updates/s, 4096 cells K=16 (one M-step per sample)",
            "value": pairs / wall, "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
            "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "stepwise: the 4096-cell batches (lognormal(6.45,1) counts clipped to "
                                   "[64,8192]); after a batch step on the first, one per-sample pass per step over "
                                   "the next resident batch, eta_j = (0.1 j + 1)^-0.5 per sample",
                       "n_cells": C, "K": K, "samples_per_batch": int(np.mean(N))},
            "roofline": {"bound": "alu", "achieved": achieved, "peak": 78.6, "unit": "TFLOP/s",
                         "frac": achieved / 78.6, "traffic": None, "kernel": "stepwise_kernel",
                         "kernel_ms": k_ms, "flops_per_launch": fl,
                         "note": "FP64 vector peak; one wave per cell runs a sequential chain of samples"},
            "mini_batch": {"value": bpairs / bwall, "unit": "updates/s", "ms_per_step": bwall * 1e3 / args.steps}}


def bench_grad(args, torch):
    """Adjoint on the 4096-cell workload: the state after 8 stepwise batches, then the
    FP32 gradient pass (value + gradient of the penalised log-likelihood per cell) timed
    over the next batch, the FP64 verification pass timed once, and 10 Adam refinement
    steps through the autograd binding with the change in F."""
    import ctypes as C_
    from paper_2111_13094_amd import autograd, sdmm, synth
    n_batches = 9
    wl, batches = _gen_cells4k(n_batches)
    C, K = wl["grid"].n_cells, 16
    dev = torch.device("cuda", 0)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)
    mix = {k: torch.from_numpy(v).to(dev) for k, v in mix0.items()}
    st = sdmm.new_state(C, K, dev)
    opts = sdmm.default_opts(K, eta=0.1)
    for j in range(8):
        b = batches[j]
        sdmm.fit_mixtures(torch.from_numpy(b.offsets).to(dev), torch.from_numpy(b.samples).to(dev), mix, st, opts)
    b = batches[8]
    off, smp = torch.from_numpy(b.offsets).to(dev), torch.from_numpy(b.samples).to(dev)
    N = smp.shape[1]
    gopts = sdmm.default_opts(K, prior_mode=sdmm.PRIOR_FIXED, prior_scale=1e-3)
    for _ in range(args.warmup):
        sdmm.fit_grad(off, smp, mix, gopts)
    _sync(torch)
    L = sdmm.lib()
    L.sdmm_timing_enable(1)
    tot, cnt = C_.c_double(), C_.c_int64()
    L.sdmm_timing_read(3, C_.byref(tot), C_.byref(cnt), 1)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = sdmm.fit_grad(off, smp, mix, gopts)
    _sync(torch)
    wall = time.perf_counter() - t0
    L.sdmm_timing_read(3, C_.byref(tot), C_.byref(cnt), 1)
    k_ms = tot.value / max(cnt.value, 1)
    g64 = sdmm.default_opts(K, prior_mode=sdmm.PRIOR_FIXED, prior_scale=1e-3, flags=sdmm.FLAG_FP64_SUMS)
    sdmm.fit_grad(off, smp, mix, g64)
    _sync(torch)
    L.sdmm_timing_read(3, C_.byref(tot), C_.byref(cnt), 1)
    k64_ms = tot.value / max(cnt.value, 1)
    L.sdmm_timing_enable(0)
    status = out["status"].cpu().numpy()
    ok = (status & (1 | 2 | 4 | 32)) == 0
    _, F0, F1, rst = autograd.refine(mix, C, K, off, smp, gopts, steps=10, lr=1e-4)
    _sync(torch)
    F0, F1 = F0.cpu().numpy(), F1.cpu().numpy()
    good = ok & ((rst.cpu().numpy() & (1 | 2 | 4 | 32)) == 0)
    fl = FLOPS_PER_PAIR * N * K
    achieved = fl / (k_ms * 1e-3) / 1e12
    return {"metric": "adjoint sample x component pairs/s, 4096 cells K=16 (value + gradient per cell)",
            "value": N * K * args.steps / wall, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "grad: 4096-cell workload after 8 stepwise batches (eta=0.1), gradient of the "
                                   "penalised log-likelihood on the 9th batch, fixed prior beta=1e-3",
                       "n_cells": C, "K": K, "samples": int(N), "cells_with_gradient": int(ok.sum())},
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                         "kernel": _estep_kernel_name(256, adjoint=True), "kernel_ms": k_ms,
                         "flops_per_launch": fl, "note": "140 flop/pair of the statistics pass; the adjoint "
                                                         "terms are extra work not counted"},
            "fp64_mode_ms": k64_ms,
            "refinement": {"steps": 10, "optimizer": "Adam lr=1e-4", "cells": int(good.sum()),
                           "mean_dF": float(np.mean((F1 - F0)[good])),
                           "cells_improved": int(((F1 > F0) & good).sum())}}


def bench_huge(args, torch):
    """One cell of 2^24 samples, K = 32, lognormal(0, 2.5) weights: one batched E+M step
    per timed step for each running-sum variant of the E-step (the precision study's
    throughput side; its errors against the FP64 oracle come from the GPU test suite)."""
    from paper_2111_13094_amd import sdmm, synth
    wl = synth.workload("huge")
    b = synth.workload_batch(wl)
    K = 32
    dev = torch.device("cuda", 0)
    off, smp = torch.from_numpy(b.offsets).to(dev), torch.from_numpy(b.samples).to(dev)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], K)
    N = smp.shape[1]
    import ctypes as C_
    L = sdmm.lib()
    tot, cnt = C_.c_double(), C_.c_int64()
    res = {}
    for name, flags in (("twosum", 0), ("plain", sdmm.FLAG_PLAIN_FP32), ("fp64", sdmm.FLAG_FP64_SUMS)):
        opts = sdmm.default_opts(K, flags=flags)
        fit_time(args, torch, off, smp, mix0, 1, K, opts, steps=max(1, args.warmup // 4))  # untimed: clock settles
        if name == "twosum":  # E-step kernel time of the headline variant by HIP events
            L.sdmm_timing_enable(1)
            L.sdmm_timing_read(0, C_.byref(tot), C_.byref(cnt), 1)
        t = fit_time(args, torch, off, smp, mix0, 1, K, opts, steps=max(3, args.steps // 4))
        if name == "twosum":
            L.sdmm_timing_read(0, C_.byref(tot), C_.byref(cnt), 1)
            L.sdmm_timing_enable(0)
        res[name] = {"updates_per_s": N * K / t, "ms_per_step": t * 1e3}
    v = res["twosum"]
    k_ms = tot.value / max(cnt.value, 1)
    fl = float(N) * K * FLOPS_PER_PAIR
    achieved = fl / (k_ms * 1e-3) / 1e12
    return {"metric": "EM sample x component updates/s, 1 cell of 2^24 samples K=32 (compensated FP32 E-step)",
            "value": v["updates_per_s"], "unit": "updates/s", "n_gpus": 1, "steps": max(3, args.steps // 4),
            "warmup": max(1, args.warmup // 4), "ms_per_step": v["ms_per_step"], "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "huge: 1 cell, 2^24 samples, K=32, weights lognormal(0,2.5), one E+M step "
                                   "from the initial mixture per step"},
            "variants": res,
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                         "kernel": _estep_kernel_name(256, G=32), "kernel_ms": k_ms, "flops_per_launch": fl}}


def fit_time(args, torch, off, smp, mix0, C, K, opts, steps=5):
    """Average wall time of one batched E+M step from fresh mixtures and state."""
    from paper_2111_13094_amd import sdmm
    dev = smp.device
    m = {k: torch.from_numpy(v).to(dev) for k, v in mix0.items()}
    sdmm.fit_mixtures(off, smp, m, sdmm.new_state(C, K, dev), opts)  # warm-up (module load, first launch)
    _sync(torch)
    tot = 0.0
    for _ in range(steps):
        m = {k: torch.from_numpy(v).to(dev) for k, v in mix0.items()}
        s = sdmm.new_state(C, K, dev)
        _sync(torch)
        t1 = time.perf_counter()
        sdmm.fit_mixtures(off, smp, m, s, opts)
        _sync(torch)
        tot += time.perf_counter() - t1
    return tot / steps


def bench_single(args, torch):
    from paper_2111_13094_amd import sdmm, synth
    wl = synth.workload("single")
    b = synth.workload_batch(wl)
    dev = torch.device("cuda", 0)
    off, smp = torch.from_numpy(b.offsets).to(dev), torch.from_numpy(b.samples).to(dev)
    mix0 = synth.initial_mixtures(wl["box_lo"], wl["box_size"], 16)
    opts = sdmm.default_opts(16, iters=20, use_graph=1)
    for w in range(args.warmup + 1):
        mix = {k: torch.from_numpy(v).to(dev) for k, v in mix0.items()}
        st = sdmm.new_state(1, 16, dev)
        sdmm.fit_mixtures(off, smp, mix, st, opts)
    _sync(torch)
    t0 = time.perf_counter()
    for s in range(args.steps):
        sdmm.fit_mixtures(off, smp, mix, st, opts)
    _sync(torch)
    wall = time.perf_counter() - t0
    pairs = smp.shape[1] * 16 * 20 * args.steps
    return {"metric": "EM sample x component updates/s, 1 cell N=16384 K=16, 20 iterations", "value": pairs / wall,
            "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "single: 1 cell, N=16384, K=16, 20 EM iterations per step, hipGraph"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed steps first (the GPU clock settles over the first ~50 ms of load)")
    ap.add_argument("--workload", default="cells4k", choices=["cells4k", "cells16k", "grad", "huge", "single",
                                                                    "accurate", "product", "tree", "stepwise"])
    ap.add_argument("--schedule", default="batched", choices=["batched", "fused"])
    ap.add_argument("--min-range", type=int, default=0, help="E-step item size floor (0: library default)")
    ap.add_argument("--max-ranges", type=int, default=0, help="E-step range count cap (0: library default)")
    ap.add_argument("--wpb", type=int, default=0, help="E-step waves per work group (0: library default)")
    ap.add_argument("--sums", default="twosum", choices=["twosum", "plain", "fp64"],
                    help="E-step running sums: compensated FP32 (default), plain FP32, FP64 fold")
    ap.add_argument("--tune", type=int, default=1, help="1: let the autotuner pick the launch configuration")
    ap.add_argument("--graph", type=int, default=1, help="1: replay the fit through the library's hipGraph cache")
    ap.add_argument("--carry", type=int, default=1, help="1: calls carry the E-step mirrors to the next call "
                                                          "(SDMM_FLAG_CARRY_MIRRORS)")
    ap.add_argument("--sweep", default="", help="comma-separated schedule:items[:waves_per_block] points, "
                                                "e.g. batched:256:1,fused:512")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe", action="store_true", help="also run a device copy of known size")
    ap.add_argument("--copy-probe-mib", type=int, default=1024)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the cells are independent, so more GPUs would each fit their "
              "own share with no communication; run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.sweep:  # launch-configuration sweep on the cells4k workload, one line per point
        for point in args.sweep.split(","):
            sched, p, *w = point.split(":")
            args.schedule, args.min_range, args.max_ranges = sched, int(p), 1 << 20
            args.wpb = int(w[0]) if w else 0
            args.sums = w[1] if len(w) > 1 else "twosum"
            args.no_plain = args.no_cpu = True
            args.tune = 0
            print(json.dumps(bench_cells4k(args, torch)), flush=True)
        return
    if args.workload == "cells4k":
        out = bench_cells4k(args, torch)
    elif args.workload == "cells16k":
        out = bench_cells16k(args, torch)
    elif args.workload == "grad":
        out = bench_grad(args, torch)
    elif args.workload == "huge":
        out = bench_huge(args, torch)
    elif args.workload == "accurate":
        out = bench_accurate(args, torch)
    elif args.workload == "product":
        out = bench_product(args, torch)
    elif args.workload == "tree":
        out = bench_tree(args, torch)
    elif args.workload == "stepwise":
        out = bench_stepwise(args, torch)
    else:
        out = bench_single(args, torch)
    roof = out.get("roofline") or {}
    if roof.get("bound") == "alu":
        roof["measured_ceiling"] = measured_ceiling(torch, 64 if roof.get("peak") == 78.6 else 32,
                                                    roof.get("achieved"))
    elif roof.get("bound") == "hbm":
        roof["measured_ceiling"] = measured_copy_rate(torch, roof.get("achieved"))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
