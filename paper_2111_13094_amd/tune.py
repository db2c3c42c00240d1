"""Autotuner for the launch configuration of sdmm_fit_mixtures.

The batched fit has three free launch parameters that change its speed but not what it
computes beyond FP32 rounding:

  * the E-step work-item size P (min_range, with max_ranges large so that P = min_range
    rounded up to a power of two): small items balance the waves across the 256 compute
    units; large items cost fewer records and M-step reads;
  * the schedule. The default candidates are all SCHED_BATCHED (one E launch, then one M
    launch): the fused launch, in which the last wave of each cell runs its M-step
    (SCHED_FUSED), measured 3-5x slower per step on the 4096-cell batch, because each
    wave's device-scope release and acquire writes back and invalidates the L2 that the
    sample stream runs through. A caller may still pass fused candidates;
  * the waves per work group of the E-step launch (1, 2 or 4), which changes how soon a
    compute unit can start new items when items end at different times.

tune_fit times every candidate on the caller's own batch, with HIP events on the
stream the library launches on, using copies of the mixtures and state, and returns
the options of the fastest candidate. Results are cached per (cells, K, sample-count
bucket, flags, iterations) for the life of the process, and optionally in a JSON file.
"""
from __future__ import annotations

import json
import os

import torch

from . import sdmm

_CACHE: dict = {}

DEFAULT_CANDIDATES = [
    {"schedule": sdmm.SCHED_BATCHED, "min_range": P, "waves_per_block": wpb}
    for P in (128, 256, 512, 1024) for wpb in (1, 2, 4)
]
FUSED_CANDIDATES = [{"schedule": sdmm.SCHED_FUSED, "min_range": P, "waves_per_block": 4} for P in (256, 1024)]


def _key(n_cells, K, N, opts):
    return (int(n_cells), int(K), int(N).bit_length(), int(opts.flags), int(opts.iters))


def _apply(opts, cand):
    o = type(opts).from_buffer_copy(opts)
    o.schedule = cand["schedule"]
    o.min_range = cand["min_range"]
    o.max_ranges = 1 << 20
    o.waves_per_block = cand.get("waves_per_block", 0)
    return o


def _time_once(cell_offsets, samples, mix, state, opts, workspace, reps):
    # the copies are fresh arrays every time: carried mirrors would never apply, so every
    # candidate is timed with its setup kernel
    opts = type(opts).from_buffer_copy(opts)
    opts.flags &= ~sdmm.FLAG_CARRY_MIRRORS
    m = {k: v.clone() for k, v in mix.items()}
    st = {k: v.clone() for k, v in state.items()}
    status = torch.empty(cell_offsets.numel() - 1, dtype=torch.int32, device=samples.device)
    sdmm.fit_mixtures(cell_offsets, samples, m, st, opts, status, workspace)  # warm-up
    best = float("inf")
    for _ in range(reps):
        m2 = {k: v.clone() for k, v in mix.items()}
        st2 = {k: v.clone() for k, v in state.items()}
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sdmm.fit_mixtures(cell_offsets, samples, m2, st2, opts, status, workspace)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune_fit(cell_offsets, samples, mix: dict, state: dict, opts, candidates=None, reps=3, cache_file=None,
             verbose=False):
    """Options (a copy of `opts`) with the fastest launch configuration for this batch
    shape. `mix` and `state` are not modified."""
    n_cells = cell_offsets.numel() - 1
    N = samples.shape[1]
    key = _key(n_cells, opts.K, N, opts)
    if key not in _CACHE and cache_file and os.path.exists(cache_file):
        for k, v in json.load(open(cache_file)).items():
            _CACHE.setdefault(tuple(json.loads(k)), v)
    if key in _CACHE:
        return _apply(opts, _CACHE[key])
    cands = candidates or DEFAULT_CANDIDATES
    if opts.flags & sdmm.FLAG_ACCURATE_SIGMA:  # the accurate update has no fused schedule
        cands = [c for c in cands if c["schedule"] != sdmm.SCHED_FUSED]
    nbytes = max(sdmm.workspace_bytes(n_cells, opts.K, N, _apply(opts, c)) for c in cands)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=samples.device)
    timings = []
    for c in cands:
        ms = _time_once(cell_offsets, samples, mix, state, _apply(opts, c), ws, reps)
        timings.append((ms, c))
        if verbose:
            print(f"tune: {c} {ms:.3f} ms", flush=True)
    best_ms, best = min(timings, key=lambda t: t[0])
    _CACHE[key] = dict(best, ms=best_ms)
    if cache_file:
        data = {json.dumps(list(k)): v for k, v in _CACHE.items()}
        with open(cache_file, "w") as f:
            json.dump(data, f, indent=1)
    return _apply(opts, best)


def tuned_config(n_cells, K, N, opts):
    """The cached choice for this shape, or None."""
    return _CACHE.get(_key(n_cells, K, N, opts))
