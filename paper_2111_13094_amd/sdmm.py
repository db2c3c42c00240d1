"""Python binding of libsdmm (argument marshalling only).

Every function here takes torch tensors that already live on the GPU, passes their
device pointers and the current HIP stream to the C ABI declared in include/sdmm.h, and
returns. All arithmetic runs in the library's HIP kernels; there is no CPU fallback, and
loading fails loudly when the built library is missing.

Names follow the C ABI: fit_mixtures, condition_prepare, condition, pdf, sample,
condition_sample_pdf, fit_grad.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libsdmm.so")

OK, EINVAL, EDEVICE, ENOWORKSPACE = 0, -1, -2, -3
SKIPPED_FEW, SKIPPED_ZERO_W, BAD_INPUT, DEAD_COMPONENT, CHOL_FAIL_KEPT_PREV, BAD_PARAMS = 1, 2, 4, 8, 16, 32
ETA_CONSTANT, ETA_PAPER = 0, 1
PRIOR_ETA_OVER_M, PRIOR_FIXED = 0, 1
FLAG_ESTEP_JACOBIAN, FLAG_PLAIN_FP32, FLAG_FP64_SUMS, FLAG_ACCURATE_SIGMA, FLAG_CARRY_MIRRORS = 1, 2, 4, 8, 16
SCHED_BATCHED, SCHED_PER_CELL, SCHED_FUSED, SCHED_STEPWISE = 0, 1, 2, 3
COND_TABLE_STRIDE = 32


class Tree(C.Structure):
    _fields_ = [("max_nodes", C.c_int32), ("max_leaves", C.c_int32), ("counts", C.c_void_p), ("axis", C.c_void_p),
                ("left", C.c_void_p), ("leaf", C.c_void_p), ("split", C.c_void_p), ("leaf_node", C.c_void_p),
                ("lo", C.c_void_p), ("hi", C.c_void_p), ("init", C.c_void_p)]


class FitOpts(C.Structure):
    _fields_ = [
        ("K", C.c_int32), ("iters", C.c_int32), ("eta_mode", C.c_int32), ("prior_mode", C.c_int32),
        ("flags", C.c_int32), ("min_samples", C.c_int32), ("schedule", C.c_int32), ("min_range", C.c_int32),
        ("max_ranges", C.c_int32), ("use_graph", C.c_int32), ("waves_per_block", C.c_int32),
        ("max_cell_samples", C.c_int32),
        ("eta", C.c_double), ("rm_alpha", C.c_double), ("rm_beta", C.c_double), ("prior_scale", C.c_double),
        ("prior_q", C.c_double), ("prior_a", C.c_double), ("prior_b", C.c_double * 5),
        ("dead_threshold", C.c_double),
    ]


class Mixtures(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("K", C.c_int32), ("weights", C.c_void_p), ("mean_dir", C.c_void_p),
                ("mean_pos", C.c_void_p), ("cov", C.c_void_p)]


class EmState(C.Structure):
    _fields_ = [("s0", C.c_void_p), ("s2", C.c_void_p), ("sw", C.c_void_p), ("step", C.c_void_p)]


_lib = None


def lib():
    """Load libsdmm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libsdmm.so not found at {LIB_PATH}; build it with "
                               "`python -m paper_2111_13094_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_size_t
        P = C.POINTER
        L.sdmm_fit_workspace_size.argtypes = [i32, i32, i64, P(FitOpts)]
        L.sdmm_fit_workspace_size.restype = sz
        L.sdmm_fit_mixtures.argtypes = [vp, vp, i64, P(Mixtures), P(EmState), P(FitOpts), vp, vp, sz, vp]
        L.sdmm_fit_mixtures_noalloc.argtypes = [vp, vp, i64, P(Mixtures), P(EmState), P(FitOpts), vp, vp]
        L.sdmm_condition_prepare.argtypes = [P(Mixtures), vp, vp]
        L.sdmm_condition.argtypes = [vp, i32, i32, vp, vp, i64, vp, vp, vp]
        L.sdmm_pdf.argtypes = [vp, i32, i32, vp, i64, vp, vp, i32, vp, vp, vp]
        L.sdmm_sample.argtypes = [vp, i32, i32, vp, i64, vp, vp, i32, vp, u64, vp, vp, vp, vp, vp]
        L.sdmm_condition_sample_pdf.argtypes = [vp, i32, i32, vp, vp, i64, i32, vp, u64, vp, vp, vp, vp]
        L.sdmm_product_sample.argtypes = [vp, i32, i32, vp, vp, vp, i32, i32, vp, vp, vp, i64, i32, vp, u64, vp, vp,
                                          vp, vp, vp]
        L.sdmm_product_pdf.argtypes = [vp, i32, i32, vp, vp, vp, i32, i32, vp, vp, vp, i64, i32, vp, vp, vp]
        L.sdmm_tree_init.argtypes = [P(Tree), i32, vp, vp, vp]
        L.sdmm_tree_workspace_size.argtypes = [i64, i32]
        L.sdmm_tree_workspace_size.restype = sz
        L.sdmm_tree_refine.argtypes = [P(Tree), vp, i64, i32, i32, P(Mixtures), P(EmState), vp, vp, vp, vp, vp, sz,
                                       vp]
        L.sdmm_fit_grad.argtypes = [vp, vp, i64, P(Mixtures), P(FitOpts), vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.sdmm_mixture_from_params.argtypes = [i32, i32, vp, vp, vp, vp, vp, P(Mixtures), vp, vp]
        L.sdmm_grad_to_params.argtypes = [i32, i32, vp, vp, vp, vp, vp]
        L.sdmm_params_from_mixture.argtypes = [P(Mixtures), vp, vp, vp, vp]
        L.sdmm_probe_fma.argtypes = [i32, i32, i32, vp, P(C.c_double), vp]
        L.sdmm_status_string.argtypes = [C.c_int]
        L.sdmm_status_string.restype = C.c_char_p
        L.sdmm_version.restype = C.c_char_p
        _lib = L
    return _lib


def _ptr(t: torch.Tensor | None, dtype=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors passed to libsdmm must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors passed to libsdmm must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


def _need(t: torch.Tensor | None, n: int, what: str, dtype=None):
    """Size and element-type check before a launch: the C ABI takes bare pointers, so a
    tensor smaller than its documented layout, or of a narrower element type, would let a
    kernel access memory past its end."""
    if t is None:
        return
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if t.numel() < n:
        raise ValueError(f"{what} has {t.numel()} elements, needs {n}")


def _state_ptrs(state: dict, n_cells: int, K: int):
    for key, n, dt in (("s0", n_cells * K, torch.float64), ("s2", n_cells * K * 15, torch.float64),
                       ("sw", n_cells, torch.float64), ("step", n_cells, torch.int32)):
        _need(state[key], n, f"state[{key!r}]", dt)
    st = EmState()
    st.s0, st.s2 = _ptr(state["s0"], torch.float64), _ptr(state["s2"], torch.float64)
    st.sw, st.step = _ptr(state["sw"], torch.float64), _ptr(state["step"], torch.int32)
    return st


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _check(rc: int, what: str):
    if rc != OK:
        raise RuntimeError(f"{what} failed: {lib().sdmm_status_string(rc).decode()} ({rc})")


def default_opts(K: int = 16, **kw) -> FitOpts:
    """Options with the paper's constants (Sec. 4.3): q = 1/K, a = 5/K,
    B = a diag(0.1, 0.1, 1, 1, 1) 1e-4, Robbins-Monro alpha = 0.5, beta = 0.1, and the
    minimum of 16 samples per leaf (Sec. 4.2)."""
    o = FitOpts()
    o.K = K
    o.iters = 1
    o.eta_mode = ETA_CONSTANT
    o.eta = 1.0
    o.rm_alpha, o.rm_beta = 0.5, 0.1
    o.prior_mode = PRIOR_ETA_OVER_M
    o.prior_scale = 0.0
    o.prior_q = 1.0 / K
    o.prior_a = 5.0 / K
    for i, v in enumerate((0.1, 0.1, 1.0, 1.0, 1.0)):
        o.prior_b[i] = o.prior_a * v * 1e-4
    o.min_samples = 16
    o.dead_threshold = 1e-12
    o.schedule = SCHED_BATCHED
    for k, v in kw.items():
        if k == "prior_b":
            for i in range(5):
                o.prior_b[i] = v[i]
        else:
            setattr(o, k, v)
    return o


def _mixtures(mix: dict, n_cells: int, K: int) -> Mixtures:
    for key, n in (("pi", 1), ("mu_dir", 3), ("mu_pos", 3), ("cov", 15)):
        _need(mix[key], 0, f"mixture array {key}", torch.float64)
        if mix[key].numel() != n_cells * K * n:
            raise ValueError(f"mixture array {key} has {mix[key].numel()} values, expected {n_cells * K * n}")
    m = Mixtures()
    m.n_cells, m.K = n_cells, K
    m.weights = _ptr(mix["pi"], torch.float64)
    m.mean_dir = _ptr(mix["mu_dir"], torch.float64)
    m.mean_pos = _ptr(mix["mu_pos"], torch.float64)
    m.cov = _ptr(mix["cov"], torch.float64)
    return m


def new_state(n_cells: int, K: int, device="cuda") -> dict:
    return {"s0": torch.zeros(n_cells * K, dtype=torch.float64, device=device),
            "s2": torch.zeros(n_cells * K * 15, dtype=torch.float64, device=device),
            "sw": torch.zeros(n_cells, dtype=torch.float64, device=device),
            "step": torch.zeros(n_cells, dtype=torch.int32, device=device)}


_ws_cache: dict = {}


def workspace_bytes(n_cells: int, K: int, n_samples: int, opts: FitOpts) -> int:
    return int(lib().sdmm_fit_workspace_size(n_cells, K, n_samples, C.byref(opts)))


def _workspace(nbytes: int, device) -> torch.Tensor:
    key = (str(device),)
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = ws
    return ws


def fit_mixtures(cell_offsets: torch.Tensor, samples: torch.Tensor, mix: dict, state: dict, opts: FitOpts,
                 status: torch.Tensor | None = None, workspace: torch.Tensor | None = None, stream=None):
    """opts.iters E+M iterations of every cell (sdmm_fit_mixtures). ``samples`` is
    float32 [7, N]; ``cell_offsets`` int64 [C+1]; ``mix``/``state`` dicts of device
    tensors updated in place. Returns the int32 per-cell status tensor."""
    n_cells = cell_offsets.numel() - 1
    K = opts.K
    if samples.dim() != 2 or samples.shape[0] != 7:
        raise ValueError("samples must be [7, N]")
    N = samples.shape[1]
    if status is None:
        status = torch.empty(n_cells, dtype=torch.int32, device=samples.device)
    _need(status, n_cells, "status", torch.int32)
    _need(cell_offsets, n_cells + 1, "cell_offsets", torch.int64)
    _need(samples, 7 * N, "samples", torch.float32)
    nbytes = workspace_bytes(n_cells, K, N, opts)
    if workspace is None:
        if opts.flags & FLAG_CARRY_MIRRORS:
            raise ValueError("FLAG_CARRY_MIRRORS needs a workspace that the caller keeps between calls")
        workspace = _workspace(nbytes, samples.device)
    m = _mixtures(mix, n_cells, K)
    st = _state_ptrs(state, n_cells, K)
    rc = lib().sdmm_fit_mixtures(_ptr(cell_offsets, torch.int64), _ptr(samples, torch.float32), N, C.byref(m),
                                 C.byref(st), C.byref(opts), _ptr(status, torch.int32),
                                 _ptr(workspace, torch.uint8), workspace.numel(), _stream(stream))
    _check(rc, "sdmm_fit_mixtures")
    return status


NOALLOC_SCRATCH_BYTES = 64 << 20


def fit_mixtures_noalloc(cell_offsets: torch.Tensor, samples: torch.Tensor, mix: dict, state: dict,
                         opts: FitOpts, status: torch.Tensor, stream=None):
    """sdmm_fit_mixtures_noalloc: fit_mixtures on the library's static per-device
    workspace (at most NOALLOC_SCRATCH_BYTES; no per-cell schedule, no graph cache).
    The caller passes every output, including ``status`` (int32 [C])."""
    n_cells = cell_offsets.numel() - 1
    K = opts.K
    if samples.dim() != 2 or samples.shape[0] != 7:
        raise ValueError("samples must be [7, N]")
    N = samples.shape[1]
    _need(status, n_cells, "status", torch.int32)
    _need(cell_offsets, n_cells + 1, "cell_offsets", torch.int64)
    _need(samples, 7 * N, "samples", torch.float32)
    m = _mixtures(mix, n_cells, K)
    st = _state_ptrs(state, n_cells, K)
    rc = lib().sdmm_fit_mixtures_noalloc(_ptr(cell_offsets, torch.int64), _ptr(samples, torch.float32), N,
                                         C.byref(m), C.byref(st), C.byref(opts), _ptr(status, torch.int32),
                                         _stream(stream))
    _check(rc, "sdmm_fit_mixtures_noalloc")
    return status


def condition_prepare(mix: dict, n_cells: int, K: int, table: torch.Tensor | None = None, stream=None):
    if table is None:
        table = torch.empty(n_cells * K * COND_TABLE_STRIDE, dtype=torch.float32, device=mix["pi"].device)
    _need(table, n_cells * K * COND_TABLE_STRIDE, "table")
    m = _mixtures(mix, n_cells, K)
    _check(lib().sdmm_condition_prepare(C.byref(m), _ptr(table, torch.float32), _stream(stream)),
           "sdmm_condition_prepare")
    return table


def condition(table, n_cells, K, qpos, qcell, stream=None):
    """qpos float32 [3, nq]; qcell int32 [nq]. Returns (cond_w [nq, K], cond_m [nq, K, 2])."""
    nq = qcell.numel()
    _need(qcell, nq, "qcell", torch.int32)
    _need(table, n_cells * K * COND_TABLE_STRIDE, "table", torch.float32)
    _need(qpos, 3 * nq, "qpos", torch.float32)
    cw = torch.empty(nq, K, dtype=torch.float32, device=qcell.device)
    cm = torch.empty(nq, K, 2, dtype=torch.float32, device=qcell.device)
    _check(lib().sdmm_condition(_ptr(table, torch.float32), n_cells, K, _ptr(qpos, torch.float32),
                                _ptr(qcell, torch.int32), nq, _ptr(cw, torch.float32), _ptr(cm, torch.float32), _stream(stream)),
           "sdmm_condition")
    return cw, cm


def pdf(table, n_cells, K, qcell, cond_w, cond_m, dirs, nd, stream=None):
    """dirs float32 [3, nq*nd]. Returns pdf float32 [nq*nd]."""
    nq = qcell.numel()
    _need(qcell, nq, "qcell", torch.int32)
    _need(table, n_cells * K * COND_TABLE_STRIDE, "table", torch.float32)
    _need(cond_w, nq * K, "cond_w", torch.float32)
    _need(cond_m, nq * K * 2, "cond_m", torch.float32)
    _need(dirs, 3 * nq * nd, "dirs", torch.float32)
    out = torch.empty(nq * nd, dtype=torch.float32, device=qcell.device)
    _check(lib().sdmm_pdf(_ptr(table, torch.float32), n_cells, K, _ptr(qcell, torch.int32), nq,
                          _ptr(cond_w, torch.float32), _ptr(cond_m, torch.float32), nd, _ptr(dirs, torch.float32),
                          _ptr(out, torch.float32), _stream(stream)), "sdmm_pdf")
    return out


def sample(table, n_cells, K, qcell, cond_w, cond_m, ns, uniforms=None, seed=0, with_comp=False, stream=None):
    """ns draws per query. uniforms float32 [3, nq*ns] or None (device Philox4x32-10).
    Returns (dirs [3, nq*ns], pdf [nq*ns], valid uint8 [nq*ns], comp int32 or None)."""
    nq = qcell.numel()
    dev = qcell.device
    n = nq * ns
    _need(qcell, nq, "qcell", torch.int32)
    _need(table, n_cells * K * COND_TABLE_STRIDE, "table", torch.float32)
    _need(cond_w, nq * K, "cond_w", torch.float32)
    _need(cond_m, nq * K * 2, "cond_m", torch.float32)
    _need(uniforms, 3 * n, "uniforms", torch.float32)
    dirs = torch.empty(3, n, dtype=torch.float32, device=dev)
    pdfv = torch.empty(n, dtype=torch.float32, device=dev)
    valid = torch.empty(n, dtype=torch.uint8, device=dev)
    comp = torch.empty(n, dtype=torch.int32, device=dev) if with_comp else None
    _check(lib().sdmm_sample(_ptr(table, torch.float32), n_cells, K, _ptr(qcell, torch.int32), nq,
                             _ptr(cond_w, torch.float32), _ptr(cond_m, torch.float32), ns,
                             _ptr(uniforms, torch.float32), seed, _ptr(dirs, torch.float32),
                             _ptr(pdfv, torch.float32), _ptr(valid, torch.uint8), _ptr(comp, torch.int32),
                             _stream(stream)), "sdmm_sample")
    return dirs, pdfv, valid, comp


def condition_sample_pdf(table, n_cells, K, qpos, qcell, ns, uniforms=None, seed=0, out=None, stream=None):
    """Fused conditioning + sampling + pdf. Returns (dirs [3, nq*ns], pdf, valid)."""
    nq = qcell.numel()
    dev = qcell.device
    n = nq * ns
    if out is None:
        out = (torch.empty(3, n, dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.float32, device=dev),
               torch.empty(n, dtype=torch.uint8, device=dev))
    dirs, pdfv, valid = out
    _need(qcell, nq, "qcell", torch.int32)
    _need(table, n_cells * K * COND_TABLE_STRIDE, "table", torch.float32)
    _need(qpos, 3 * nq, "qpos", torch.float32)
    _need(uniforms, 3 * n, "uniforms", torch.float32)
    for t, m, what, dt in ((dirs, 3 * n, "dirs", torch.float32), (pdfv, n, "pdf", torch.float32),
                           (valid, n, "valid", torch.uint8)):
        _need(t, m, what, dt)
    _check(lib().sdmm_condition_sample_pdf(_ptr(table, torch.float32), n_cells, K, _ptr(qpos, torch.float32),
                                           _ptr(qcell, torch.int32), nq, ns, _ptr(uniforms, torch.float32), seed,
                                           _ptr(dirs, torch.float32), _ptr(pdfv, torch.float32),
                                           _ptr(valid, torch.uint8), _stream(stream)),
           "sdmm_condition_sample_pdf")
    return dirs, pdfv, valid


def _product_checks(table, n_cells, K, qpos, qcell, btable, n_bsdf, Kb, bpar, bcell, frames, nq):
    _need(qcell, nq, "qcell", torch.int32)
    _need(table, n_cells * K * COND_TABLE_STRIDE, "table", torch.float32)
    _need(btable, n_bsdf * Kb * COND_TABLE_STRIDE, "btable", torch.float32)
    _need(qpos, 3 * nq, "qpos", torch.float32)
    _need(bpar, 3 * nq, "bpar", torch.float32)
    _need(bcell, nq, "bcell", torch.int32)
    _need(frames, 9 * nq, "frames", torch.float32)


def product_sample(table, n_cells, K, qpos, qcell, btable, n_bsdf, Kb, bpar, bcell, frames, ns, uniforms=None, seed=0,
                   with_pair=False, out=None, stream=None):
    """Product sampling with a conditioned BSDF mixture. qpos, bpar float32 [3, nq];
    frames float32 [9, nq] (row-major local-to-world rotation per query). Returns
    (dirs [3, nq*ns], pdf [nq*ns], valid uint8 [nq*ns], pair int32 or None)."""
    nq = qcell.numel()
    dev = qcell.device
    n = nq * ns
    if out is None:
        out = (torch.empty(3, n, dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.float32, device=dev),
               torch.empty(n, dtype=torch.uint8, device=dev),
               torch.empty(n, dtype=torch.int32, device=dev) if with_pair else None)
    dirs, pdfv, valid, pair = out
    _product_checks(table, n_cells, K, qpos, qcell, btable, n_bsdf, Kb, bpar, bcell, frames, nq)
    _need(uniforms, 3 * n, "uniforms", torch.float32)
    for t, m, what, dt in ((dirs, 3 * n, "dirs", torch.float32), (pdfv, n, "pdf", torch.float32),
                           (valid, n, "valid", torch.uint8), (pair, n, "pair", torch.int32)):
        _need(t, m, what, dt)
    _check(lib().sdmm_product_sample(_ptr(table, torch.float32), n_cells, K, _ptr(qpos, torch.float32),
                                     _ptr(qcell, torch.int32), _ptr(btable, torch.float32), n_bsdf, Kb,
                                     _ptr(bpar, torch.float32), _ptr(bcell, torch.int32), _ptr(frames, torch.float32),
                                     nq, ns, _ptr(uniforms, torch.float32), seed, _ptr(dirs, torch.float32),
                                     _ptr(pdfv, torch.float32), _ptr(valid, torch.uint8), _ptr(pair, torch.int32),
                                     _stream(stream)), "sdmm_product_sample")
    return dirs, pdfv, valid, pair


def product_pdf(table, n_cells, K, qpos, qcell, btable, n_bsdf, Kb, bpar, bcell, frames, dirs, stream=None):
    """Product density at dirs float32 [3, nq*nd]. Returns pdf [nq*nd]."""
    nq = qcell.numel()
    nd = dirs.shape[1] // max(nq, 1)
    _product_checks(table, n_cells, K, qpos, qcell, btable, n_bsdf, Kb, bpar, bcell, frames, nq)
    _need(dirs, 3 * nq * nd, "dirs", torch.float32)
    out = torch.empty(nq * nd, dtype=torch.float32, device=qcell.device)
    _check(lib().sdmm_product_pdf(_ptr(table, torch.float32), n_cells, K, _ptr(qpos, torch.float32),
                                  _ptr(qcell, torch.int32), _ptr(btable, torch.float32), n_bsdf, Kb,
                                  _ptr(bpar, torch.float32), _ptr(bcell, torch.int32), _ptr(frames, torch.float32),
                                  nq, nd, _ptr(dirs, torch.float32), _ptr(out, torch.float32), _stream(stream)),
           "sdmm_product_pdf")
    return out


def new_tree(max_leaves, device="cuda"):
    """Device arrays of a kD-tree with room for max_leaves leaves (a dict of tensors)."""
    n = 2 * max_leaves - 1
    i32 = dict(dtype=torch.int32, device=device)
    f64 = dict(dtype=torch.float64, device=device)
    return {"counts": torch.zeros(2, **i32), "axis": torch.full((n,), -1, **i32), "left": torch.full((n,), -1, **i32),
            "leaf": torch.full((n,), -1, **i32), "split": torch.zeros(n, **f64),
            "leaf_node": torch.full((max_leaves,), -1, **i32), "lo": torch.zeros(max_leaves, 3, **f64),
            "hi": torch.zeros(max_leaves, 3, **f64), "init": torch.zeros(max_leaves, **i32),
            "max_leaves": max_leaves, "max_nodes": n}


def _tree(t: dict) -> Tree:
    return Tree(t["max_nodes"], t["max_leaves"], _ptr(t["counts"], torch.int32), _ptr(t["axis"], torch.int32),
                _ptr(t["left"], torch.int32), _ptr(t["leaf"], torch.int32), _ptr(t["split"], torch.float64),
                _ptr(t["leaf_node"], torch.int32), _ptr(t["lo"], torch.float64), _ptr(t["hi"], torch.float64),
                _ptr(t["init"], torch.int32))


def tree_init(t: dict, depth, lo, hi, stream=None):
    lo_ = (C.c_double * 3)(*[float(v) for v in lo])
    hi_ = (C.c_double * 3)(*[float(v) for v in hi])
    tt = _tree(t)
    _check(lib().sdmm_tree_init(C.byref(tt), depth, lo_, hi_, _stream(stream)), "sdmm_tree_init")


def tree_refine(t: dict, samples, split_threshold, mix: dict, state: dict, K, min_init=16, workspace=None,
                stream=None):
    """Refines the tree with samples float32 [7, N]; mix / state hold max_leaves cells.
    Returns (sorted samples [7, N], cell offsets int64 [n_leaves + 1], n_leaves, status)."""
    if samples.dim() != 2 or samples.shape[0] != 7:
        raise ValueError("samples must be [7, N]")
    N = samples.shape[1]
    dev = samples.device
    sorted_ = torch.empty_like(samples)
    offsets = torch.empty(t["max_leaves"] + 1, dtype=torch.int64, device=dev)
    nbytes = lib().sdmm_tree_workspace_size(N, t["max_leaves"])
    if workspace is None:
        workspace = _workspace(nbytes, dev)
    m = _mixtures(mix, t["max_leaves"], K)
    st = _state_ptrs(state, t["max_leaves"], K)
    nl, status = C.c_int32(0), C.c_int32(0)
    tt = _tree(t)
    _check(lib().sdmm_tree_refine(C.byref(tt), _ptr(samples, torch.float32), N, split_threshold, min_init, C.byref(m),
                                  C.byref(st), _ptr(sorted_, torch.float32), _ptr(offsets, torch.int64), C.byref(nl),
                                  C.byref(status), _ptr(workspace, torch.uint8), workspace.numel(), _stream(stream)),
           "sdmm_tree_refine")
    return sorted_, offsets[:nl.value + 1], nl.value, status.value


def fit_grad(cell_offsets, samples, mix, opts: FitOpts, workspace=None, stream=None):
    """F and its gradient per cell (sdmm_fit_grad). Returns a dict of device tensors."""
    n_cells = cell_offsets.numel() - 1
    K = opts.K
    if samples.dim() != 2 or samples.shape[0] != 7:
        raise ValueError("samples must be [7, N]")
    N = samples.shape[1]
    dev = samples.device
    out = {"F": torch.empty(n_cells, dtype=torch.float64, device=dev),
           "alpha": torch.empty(n_cells, K, dtype=torch.float64, device=dev),
           "mu_pos": torch.empty(n_cells, K, 3, dtype=torch.float64, device=dev),
           "delta": torch.empty(n_cells, K, 2, dtype=torch.float64, device=dev),
           "L": torch.empty(n_cells, K, 15, dtype=torch.float64, device=dev),
           "status": torch.empty(n_cells, dtype=torch.int32, device=dev)}
    nbytes = workspace_bytes(n_cells, K, N, opts)
    if workspace is None:
        workspace = _workspace(nbytes, dev)
    m = _mixtures(mix, n_cells, K)
    rc = lib().sdmm_fit_grad(_ptr(cell_offsets, torch.int64), _ptr(samples, torch.float32), N, C.byref(m),
                             C.byref(opts), _ptr(out["F"], torch.float64), _ptr(out["alpha"], torch.float64),
                             _ptr(out["mu_pos"], torch.float64), _ptr(out["delta"], torch.float64),
                             _ptr(out["L"], torch.float64), _ptr(out["status"], torch.int32),
                             _ptr(workspace, torch.uint8), workspace.numel(), _stream(stream))
    _check(rc, "sdmm_fit_grad")
    return out


def mixture_from_params(alpha, mu_dir0, delta, mu_pos, L, out=None, with_jac=True, stream=None):
    """Mixture (pi, mu_dir, mu_pos, cov) from the refinement parameters
    (sdmm_mixture_from_params); returns (mixture dict, 2x2 Jacobians or None)."""
    n_cells, K = alpha.shape[0], alpha.shape[1]
    dev = alpha.device
    for t, m, what in ((alpha, n_cells * K, "alpha"), (mu_dir0, n_cells * K * 3, "mu_dir0"),
                       (delta, n_cells * K * 2, "delta"), (mu_pos, n_cells * K * 3, "mu_pos"),
                       (L, n_cells * K * 15, "L")):
        _need(t, m, what, torch.float64)
    if out is None:
        out = {"pi": torch.empty(n_cells * K, dtype=torch.float64, device=dev),
               "mu_dir": torch.empty(n_cells * K * 3, dtype=torch.float64, device=dev),
               "mu_pos": torch.empty(n_cells * K * 3, dtype=torch.float64, device=dev),
               "cov": torch.empty(n_cells * K * 15, dtype=torch.float64, device=dev)}
    jac = torch.empty(n_cells, K, 4, dtype=torch.float64, device=dev) if with_jac else None
    m = _mixtures(out, n_cells, K)
    f64 = torch.float64
    rc = lib().sdmm_mixture_from_params(n_cells, K, _ptr(alpha, f64), _ptr(mu_dir0, f64), _ptr(delta, f64),
                                        _ptr(mu_pos, f64), _ptr(L, f64), C.byref(m), _ptr(jac, f64),
                                        _stream(stream))
    _check(rc, "sdmm_mixture_from_params")
    return out, jac


def grad_to_params(L, jac, g_delta, g_L, stream=None):
    """In-place pull-back of sdmm_fit_grad's delta and L gradients (sdmm_grad_to_params)."""
    n_cells, K = L.shape[0], L.shape[1]
    for t, m, what in ((L, n_cells * K * 15, "L"), (jac, n_cells * K * 4, "jac"), (g_delta, n_cells * K * 2, "g_delta"),
                       (g_L, n_cells * K * 15, "g_L")):
        _need(t, m, what, torch.float64)
    f64 = torch.float64
    rc = lib().sdmm_grad_to_params(n_cells, K, _ptr(L, f64), _ptr(jac, f64), _ptr(g_delta, f64), _ptr(g_L, f64),
                                   _stream(stream))
    _check(rc, "sdmm_grad_to_params")


def params_from_mixture(mix, n_cells, K, stream=None):
    """Refinement parameters of a mixture (sdmm_params_from_mixture): returns
    (alpha [C,K], L [C,K,15], status [C]) as device tensors."""
    dev = mix["pi"].device
    alpha = torch.empty(n_cells, K, dtype=torch.float64, device=dev)
    L = torch.empty(n_cells, K, 15, dtype=torch.float64, device=dev)
    status = torch.empty(n_cells, dtype=torch.int32, device=dev)
    m = _mixtures(mix, n_cells, K)
    rc = lib().sdmm_params_from_mixture(C.byref(m), _ptr(alpha, torch.float64), _ptr(L, torch.float64),
                                        _ptr(status, torch.int32), _stream(stream))
    _check(rc, "sdmm_params_from_mixture")
    return alpha, L, status


def probe_fma(bits=32, n_groups=8192, iters=1024, device="cuda", stream=None):
    """Measured vector FMA rate (sdmm_probe_fma) in TFLOP/s: FP32 as the library's kernels
    are built (no packed FP32) for bits=32, FP64 for bits=64."""
    dt = torch.float32 if bits == 32 else torch.float64
    out = torch.empty(n_groups * 256, dtype=dt, device=device)
    ms = C.c_double()
    rc = lib().sdmm_probe_fma(int(bits), int(n_groups), int(iters), _ptr(out, dt), C.byref(ms), _stream(stream))
    _check(rc, "sdmm_probe_fma")
    return n_groups * 256.0 * iters * 16 * 2 / (ms.value * 1e-3) / 1e12
