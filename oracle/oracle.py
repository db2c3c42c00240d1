"""ctypes front end of the FP64 CPU oracle (``sdmm_oracle.c``).

TEST INFRASTRUCTURE: imported only by the tests, the package smoke check and the
benchmark's CPU-baseline leg. It shares no code with the GPU library and does not import
the product package. Arguments are numpy arrays; this module only marshals them.

The arithmetic lives in ``sdmm_oracle.c``; see its header for the paper passages each
function follows and the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sdmm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")  # the same source with OpenMP over cells

SKIPPED_FEW, SKIPPED_ZERO_W, BAD_INPUT, DEAD_COMPONENT, CHOL_FAIL_KEPT_PREV, BAD_PARAMS = (
    1, 2, 4, 8, 16, 32)


def build(force: bool = False, omp: bool = False) -> str:
    """Compile the oracle with gcc: -O2, no fast-math, FP64 throughout. omp=True builds the
    same source with OpenMP, whose fit spreads independent cells over threads (the
    all-cores CPU baseline); the single-threaded library is the reference."""
    out = LIB_OMP if omp else LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
        tmp = out + ".tmp%d" % os.getpid()
        flags = ["-fopenmp"] if omp else []
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", *flags, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, out)
    return out


class _Opts(C.Structure):
    _fields_ = [
        ("K", C.c_int32), ("iters", C.c_int32), ("eta_mode", C.c_int32), ("prior_mode", C.c_int32),
        ("estep_jacobian", C.c_int32), ("euclidean", C.c_int32), ("min_samples", C.c_int32),
        ("accurate_sigma", C.c_int32),
        ("eta", C.c_double), ("rm_alpha", C.c_double), ("rm_beta", C.c_double),
        ("prior_scale", C.c_double), ("prior_q", C.c_double), ("prior_a", C.c_double),
        ("prior_b", C.c_double * 5), ("dead_threshold", C.c_double),
    ]


@dataclass
class Opts:
    """Fit options. Defaults: the paper's prior constants q = 1/K, a = 5/K,
    B = a diag(0.1, 0.1, 1, 1, 1) 1e-4 and Robbins-Monro alpha = 0.5, beta = 0.1 (Sec. 4.3)."""
    K: int = 16
    iters: int = 1
    eta_mode: int = 0          # 0: constant eta after the first batch; 1: (rm_beta j + 1)^-rm_alpha
    eta: float = 1.0
    rm_alpha: float = 0.5
    rm_beta: float = 0.1
    prior_mode: int = 0        # 0: beta_j = eta_j / M_j; 1: beta_j = prior_scale
    prior_scale: float = 0.0
    prior_q: float | None = None
    prior_a: float | None = None
    prior_b: tuple | None = None
    estep_jacobian: int = 0
    euclidean: int = 0
    min_samples: int = 16
    dead_threshold: float = 1e-12
    accurate_sigma: int = 0    # 1: covariance from a second pass in the new tangent spaces (eta = 1)

    def to_c(self) -> _Opts:
        q = 1.0 / self.K if self.prior_q is None else self.prior_q
        a = 5.0 / self.K if self.prior_a is None else self.prior_a
        b = tuple(a * v * 1e-4 for v in (0.1, 0.1, 1, 1, 1)) if self.prior_b is None else tuple(self.prior_b)
        o = _Opts()
        o.K, o.iters, o.eta_mode, o.prior_mode = self.K, self.iters, self.eta_mode, self.prior_mode
        o.estep_jacobian, o.euclidean, o.min_samples = self.estep_jacobian, self.euclidean, self.min_samples
        o.eta, o.rm_alpha, o.rm_beta, o.prior_scale = self.eta, self.rm_alpha, self.rm_beta, self.prior_scale
        o.prior_q, o.prior_a = q, a
        for i in range(5):
            o.prior_b[i] = b[i]
        o.dead_threshold = self.dead_threshold
        o.accurate_sigma = self.accurate_sigma
        return o


_lib = None
_lib_omp = None


def lib_omp():
    """The OpenMP build (fit over cells on all threads), for the all-cores baseline."""
    global _lib_omp
    if _lib_omp is None:
        L = C.CDLL(build(omp=True))
        L.orc_fit.argtypes = [C.POINTER(_Opts), C.c_int32] + [C.c_void_p] * 2 + [C.c_int64] + [C.c_void_p] * 9
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = C.c_int
        _lib_omp = L
    return _lib_omp


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d, i32, i64, vp = C.c_double, C.c_int32, C.c_int64, C.c_void_p
        P = C.POINTER
        _lib.orc_frame.argtypes = [vp, vp]
        _lib.orc_log_map.argtypes = [vp, vp, vp]
        _lib.orc_exp_map.argtypes = [vp, vp, vp]
        _lib.orc_transfer_jacobian.argtypes = [vp, vp, vp]
        _lib.orc_eta.argtypes = [P(_Opts), i32]
        _lib.orc_eta.restype = d
        _lib.orc_cell_stats.argtypes = [P(_Opts), i32, vp, i64, i64, i64, vp, vp, vp, vp,
                                        vp, vp, vp, vp, vp, vp]
        _lib.orc_responsibilities.argtypes = [P(_Opts), i32, vp, vp, vp, vp, vp, vp, vp]
        _lib.orc_fit.argtypes = [P(_Opts), i32, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        _lib.orc_objective.argtypes = [P(_Opts), i32, vp, i64, i64, i64, vp, vp, vp, vp, d]
        _lib.orc_objective.restype = d
        _lib.orc_grad.argtypes = [P(_Opts), i32, vp, i64, i64, i64, vp, vp, vp, vp, d, vp, vp, vp, vp]
        _lib.orc_condition.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp]
        _lib.orc_pdf_conditioned.argtypes = [i32, vp, vp, vp, vp, vp]
        _lib.orc_pdf_conditioned.restype = d
        _lib.orc_pdf.argtypes = [i32, vp, vp, vp, vp, i64, vp, vp, i32, vp, vp]
        _lib.orc_sample.argtypes = [i32, vp, vp, vp, vp, i64, vp, vp, i32, vp, vp, vp, vp, vp]
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "arrays must be C-contiguous"
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --- maps -----------------------------------------------------------------

def frame(mu):
    mu = _f64(mu)
    R = np.zeros(9)
    lib().orc_frame(_p(mu), _p(R))
    return R.reshape(3, 3)


def log_map(mu, w):
    R = _f64(frame(mu))
    w = _f64(w)
    nu = np.zeros(2)
    lib().orc_log_map(_p(R), _p(w), _p(nu))
    return nu


def exp_map(mu, nu):
    R = _f64(frame(mu))
    nu = _f64(nu)
    w = np.zeros(3)
    lib().orc_exp_map(_p(R), _p(nu), _p(w))
    return w


def transfer_jacobian(mu, m):
    mu, m = _f64(mu), _f64(m)
    J = np.zeros(4)
    lib().orc_transfer_jacobian(_p(mu), _p(m), _p(J))
    return J.reshape(2, 2)


def eta(opts: Opts, j: int) -> float:
    o = opts.to_c()
    return lib().orc_eta(C.byref(o), j)


# --- mixtures -------------------------------------------------------------

def new_state(n_cells: int, K: int) -> dict:
    return {"s0": np.zeros(n_cells * K), "s2": np.zeros(n_cells * K * 15),
            "sw": np.zeros(n_cells), "step": np.zeros(n_cells, dtype=np.int32)}


def fit(opts: Opts, offsets, samples, mix: dict, state: dict, threads: int = 0) -> np.ndarray:
    """``opts.iters`` E+M iterations on one batch; ``mix`` (pi, mu_dir, mu_pos, cov) and
    ``state`` (s0, s2, sw, step) are updated in place. Returns per-cell status bits.
    threads > 0 runs the OpenMP build of the same source with that many threads (cells
    spread over them; every cell's result is the same as with one thread)."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    samples = np.ascontiguousarray(samples, dtype=np.float32)
    n_cells = offsets.shape[0] - 1
    status = np.zeros(n_cells, dtype=np.int32)
    for key in ("pi", "mu_dir", "mu_pos", "cov"):
        assert mix[key].dtype == np.float64 and mix[key].flags["C_CONTIGUOUS"]
    o = opts.to_c()
    L = lib()
    if threads > 0:
        L = lib_omp()
        L.orc_set_threads(int(threads))
    rc = L.orc_fit(C.byref(o), n_cells, _p(offsets), _p(samples), samples.shape[1],
                       _p(mix["pi"]), _p(mix["mu_dir"]), _p(mix["mu_pos"]), _p(mix["cov"]),
                       _p(state["s0"]), _p(state["s2"]), _p(state["sw"]), _p(state["step"]),
                       _p(status))
    if rc != 0:
        raise ValueError("orc_fit failed (%d)" % rc)
    return status


def fit_stepwise(opts: Opts, offsets, samples, mix: dict, state: dict) -> np.ndarray:
    """Stepwise (per-sample) EM on one batch; arguments as fit()."""
    L = lib()
    L.orc_fit_stepwise.argtypes = L.orc_fit.argtypes
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    samples = np.ascontiguousarray(samples, dtype=np.float32)
    n_cells = offsets.shape[0] - 1
    status = np.zeros(n_cells, dtype=np.int32)
    o = opts.to_c()
    rc = L.orc_fit_stepwise(C.byref(o), n_cells, _p(offsets), _p(samples), samples.shape[1],
                            _p(mix["pi"]), _p(mix["mu_dir"]), _p(mix["mu_pos"]), _p(mix["cov"]),
                            _p(state["s0"]), _p(state["s2"]), _p(state["sw"]), _p(state["step"]), _p(status))
    if rc != 0:
        raise ValueError("orc_fit_stepwise failed (%d)" % rc)
    return status


def _cell_params(mix, c, K):
    s = slice(c * K, (c + 1) * K)
    return (_f64(mix["pi"][s]), _f64(mix["mu_dir"].reshape(-1, 3)[s]), _f64(mix["mu_pos"].reshape(-1, 3)[s]),
            _f64(mix["cov"].reshape(-1, 15)[s]))


def cell_stats(opts: Opts, samples, i0, i1, mix, cell=0):
    """Unnormalised statistics of samples [i0, i1) about the cell's current parameters."""
    samples = np.ascontiguousarray(samples, dtype=np.float32)
    K = opts.K
    pi, mud, mux, cov = _cell_params(mix, cell, K)
    S0, S1, S2 = np.zeros(K), np.zeros(K * 5), np.zeros(K * 15)
    W, LL = np.zeros(1), np.zeros(1)
    M = np.zeros(1, dtype=np.int64)
    o = opts.to_c()
    st = lib().orc_cell_stats(C.byref(o), K, _p(samples), samples.shape[1], i0, i1, _p(pi), _p(mud),
                              _p(mux), _p(cov), _p(S0), _p(S1), _p(S2), _p(W), _p(M), _p(LL))
    return {"S0": S0, "S1": S1.reshape(K, 5), "S2": S2.reshape(K, 15), "W": W[0], "M": int(M[0]),
            "LL": LL[0], "status": st}


def responsibilities(opts: Opts, w, p, mix, cell=0):
    K = opts.K
    pi, mud, mux, cov = _cell_params(mix, cell, K)
    r = np.zeros(K)
    o = opts.to_c()
    lib().orc_responsibilities(C.byref(o), K, _p(_f64(w)), _p(_f64(p)), _p(pi), _p(mud), _p(mux),
                               _p(cov), _p(r))
    return r


def objective(opts: Opts, samples, i0, i1, mix, beta, cell=0) -> float:
    samples = np.ascontiguousarray(samples, dtype=np.float32)
    K = opts.K
    pi, mud, mux, cov = _cell_params(mix, cell, K)
    o = opts.to_c()
    return lib().orc_objective(C.byref(o), K, _p(samples), samples.shape[1], i0, i1, _p(pi), _p(mud),
                               _p(mux), _p(cov), beta)


def grad(opts: Opts, samples, i0, i1, mix, beta, cell=0) -> dict:
    samples = np.ascontiguousarray(samples, dtype=np.float32)
    K = opts.K
    pi, mud, mux, cov = _cell_params(mix, cell, K)
    ga, gx, gd, gL = np.zeros(K), np.zeros(3 * K), np.zeros(2 * K), np.zeros(15 * K)
    o = opts.to_c()
    st = lib().orc_grad(C.byref(o), K, _p(samples), samples.shape[1], i0, i1, _p(pi), _p(mud), _p(mux),
                        _p(cov), beta, _p(ga), _p(gx), _p(gd), _p(gL))
    if st:
        raise ValueError("orc_grad status %d" % st)
    return {"alpha": ga, "mu_pos": gx.reshape(K, 3), "delta": gd.reshape(K, 2), "L": gL.reshape(K, 15)}


def condition(K, mix, cell, x):
    pi, mud, mux, cov = _cell_params(mix, cell, K)
    pic, m, Sc = np.zeros(K), np.zeros(2 * K), np.zeros(3 * K)
    rc = lib().orc_condition(K, _p(pi), _p(mux), _p(cov), _p(_f64(x)), _p(pic), _p(m), _p(Sc))
    if rc:
        raise ValueError("conditioning failed")
    return pic, m.reshape(K, 2), Sc.reshape(K, 3)


def pdf_conditioned(K, mud, pic, m, Sc, w) -> float:
    return lib().orc_pdf_conditioned(K, _p(_f64(mud)), _p(_f64(pic)), _p(_f64(m)), _p(_f64(Sc)),
                                     _p(_f64(w)))


def pdf(K, mix, qpos, qcell, dirs):
    """dirs: (nq, nd, 3). Returns (nq, nd) FP64 pdf values."""
    qpos = _f64(qpos)
    qcell = np.ascontiguousarray(qcell, dtype=np.int32)
    dirs = _f64(dirs)
    nq, nd = dirs.shape[0], dirs.shape[1]
    out = np.zeros((nq, nd))
    rc = lib().orc_pdf(K, _p(_f64(mix["pi"])), _p(_f64(mix["mu_dir"])), _p(_f64(mix["mu_pos"])),
                       _p(_f64(mix["cov"])), nq, _p(qpos), _p(qcell), nd, _p(dirs), _p(out))
    if rc:
        raise ValueError("orc_pdf failed")
    return out


def sample(K, mix, qpos, qcell, uniforms):
    """uniforms: (nq, ns, 3) in [0,1). Returns dirs (nq,ns,3), pdf (nq,ns), comp, valid."""
    qpos = _f64(qpos)
    qcell = np.ascontiguousarray(qcell, dtype=np.int32)
    u = _f64(uniforms)
    nq, ns = u.shape[0], u.shape[1]
    dirs, pdfv = np.zeros((nq, ns, 3)), np.zeros((nq, ns))
    comp = np.zeros((nq, ns), dtype=np.int32)
    valid = np.zeros((nq, ns), dtype=np.uint8)
    rc = lib().orc_sample(K, _p(_f64(mix["pi"])), _p(_f64(mix["mu_dir"])), _p(_f64(mix["mu_pos"])),
                          _p(_f64(mix["cov"])), nq, _p(qpos), _p(qcell), ns, _p(u), _p(dirs), _p(pdfv),
                          _p(comp), _p(valid))
    if rc:
        raise ValueError("orc_sample failed")
    return dirs, pdfv, comp, valid


# --- product sampling with a conditioned BSDF mixture ----------------------------------

def pair_transfer(mu1, mu2, m2):
    """Centre a = log_mu1(exp_mu2(m2)) and Jacobian J (2x2) of log_mu1 o exp_mu2 at m2."""
    L = lib()
    L.orc_pair_transfer.argtypes = [C.c_void_p] * 5
    a, J = np.zeros(2), np.zeros(4)
    L.orc_pair_transfer(_p(_f64(mu1)), _p(_f64(mu2)), _p(_f64(m2)), _p(a), _p(J))
    return a, J.reshape(2, 2)


def rotate_component(F, mu, m, S):
    """Component (mu, offset m, packed 2x2 covariance S) rotated by F (world = F local)."""
    L = lib()
    L.orc_rotate_component.argtypes = [C.c_void_p] * 7
    muw, mw, Sw = np.zeros(3), np.zeros(2), np.zeros(3)
    L.orc_rotate_component(_p(_f64(np.asarray(F).ravel())), _p(_f64(mu)), _p(_f64(m)), _p(_f64(S)), _p(muw),
                           _p(mw), _p(Sw))
    return muw, mw, Sw


def _product_args(K, mix, Kb, bmix, qpos, qcell, bpar, bcell, frames):
    return (K, _p(_f64(mix["pi"])), _p(_f64(mix["mu_dir"])), _p(_f64(mix["mu_pos"])), _p(_f64(mix["cov"])),
            Kb, _p(_f64(bmix["pi"])), _p(_f64(bmix["mu_dir"])), _p(_f64(bmix["mu_pos"])), _p(_f64(bmix["cov"])))


def product_pairs(K, mix, cell, Kb, bmix, bcell, x, bx, F):
    """The 2K pairs of one query: dict of arrays logw (2K), mu (2K, 3), c (2K, 2), C (2K, 3)
    in pair order 2k + j."""
    L = lib()
    i32, vp = C.c_int32, C.c_void_p
    L.orc_product_pairs.argtypes = [i32, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
    pi, mud, mux, cov = _cell_params(mix, cell, K)
    bpi, bmud, bmux, bcov = _cell_params(bmix, bcell, Kb)
    out = np.zeros((2 * K, 9))
    rc = L.orc_product_pairs(K, _p(pi), _p(mud), _p(mux), _p(cov), _p(_f64(x)), Kb, _p(bpi), _p(bmud), _p(bmux),
                             _p(bcov), _p(_f64(bx)), _p(_f64(np.asarray(F).ravel())), _p(out))
    if rc:
        raise ValueError("orc_product_pairs failed")
    return {"logw": out[:, 0], "mu": out[:, 1:4], "c": out[:, 4:6], "C": out[:, 6:9]}


def product_sample(K, mix, Kb, bmix, qpos, qcell, bpar, bcell, frames, uniforms):
    """Product sampling. qpos, bpar: (nq, 3); frames: (nq, 3, 3) local-to-world;
    uniforms: (nq, ns, 3). Returns dirs (nq, ns, 3), pdf (nq, ns), pair, valid."""
    L = lib()
    i32, i64, vp = C.c_int32, C.c_int64, C.c_void_p
    L.orc_product_sample.argtypes = [i32, vp, vp, vp, vp, i32, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, i32, vp,
                                     vp, vp, vp, vp]
    qpos, bpar, F = _f64(qpos), _f64(bpar), _f64(frames)
    qcell = np.ascontiguousarray(qcell, dtype=np.int32)
    bcell = np.ascontiguousarray(bcell, dtype=np.int32)
    u = _f64(uniforms)
    nq, ns = u.shape[0], u.shape[1]
    dirs, pdfv = np.zeros((nq, ns, 3)), np.zeros((nq, ns))
    pair = np.zeros((nq, ns), dtype=np.int32)
    valid = np.zeros((nq, ns), dtype=np.uint8)
    rc = L.orc_product_sample(*_product_args(K, mix, Kb, bmix, qpos, qcell, bpar, bcell, F), nq, _p(qpos),
                              _p(qcell), _p(bpar), _p(bcell), _p(F), ns, _p(u), _p(dirs), _p(pdfv), _p(pair),
                              _p(valid))
    if rc:
        raise ValueError("orc_product_sample failed")
    return dirs, pdfv, pair, valid


def product_pdf(K, mix, Kb, bmix, qpos, qcell, bpar, bcell, frames, dirs):
    """The product density at dirs (nq, nd, 3); returns (nq, nd)."""
    L = lib()
    i32, i64, vp = C.c_int32, C.c_int64, C.c_void_p
    L.orc_product_pdf.argtypes = [i32, vp, vp, vp, vp, i32, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, i32, vp, vp]
    qpos, bpar, F = _f64(qpos), _f64(bpar), _f64(frames)
    qcell = np.ascontiguousarray(qcell, dtype=np.int32)
    bcell = np.ascontiguousarray(bcell, dtype=np.int32)
    dirs = _f64(dirs)
    nq, nd = dirs.shape[0], dirs.shape[1]
    out = np.zeros((nq, nd))
    rc = L.orc_product_pdf(*_product_args(K, mix, Kb, bmix, qpos, qcell, bpar, bcell, F), nq, _p(qpos), _p(qcell),
                           _p(bpar), _p(bcell), _p(F), nd, _p(dirs), _p(out))
    if rc:
        raise ValueError("orc_product_pdf failed")
    return out


# --- spatial kD-tree --------------------------------------------------------------------

class _Tree(C.Structure):
    _fields_ = [("max_nodes", C.c_int32), ("max_leaves", C.c_int32), ("counts", C.c_void_p),
                ("axis", C.c_void_p), ("left", C.c_void_p), ("leaf", C.c_void_p), ("split", C.c_void_p),
                ("leaf_node", C.c_void_p), ("lo", C.c_void_p), ("hi", C.c_void_p), ("init", C.c_void_p)]


class Tree:
    """numpy arrays of a kD-tree with room for max_leaves leaves (2 max_leaves - 1 nodes)."""

    def __init__(self, max_leaves):
        n = 2 * max_leaves - 1
        self.counts = np.zeros(2, dtype=np.int32)
        self.axis = np.full(n, -1, dtype=np.int32)
        self.left = np.full(n, -1, dtype=np.int32)
        self.leaf = np.full(n, -1, dtype=np.int32)
        self.split = np.zeros(n)
        self.leaf_node = np.full(max_leaves, -1, dtype=np.int32)
        self.lo = np.zeros((max_leaves, 3))
        self.hi = np.zeros((max_leaves, 3))
        self.init = np.zeros(max_leaves, dtype=np.int32)
        self.max_leaves, self.max_nodes = max_leaves, n

    def c(self):
        return _Tree(self.max_nodes, self.max_leaves, *[_p(a) for a in (
            self.counts, self.axis, self.left, self.leaf, self.split, self.leaf_node, self.lo, self.hi, self.init)])

    @property
    def n_nodes(self):
        return int(self.counts[0])

    @property
    def n_leaves(self):
        return int(self.counts[1])


def tree_init(max_leaves, depth, lo, hi) -> Tree:
    L = lib()
    L.orc_tree_init.argtypes = [C.POINTER(_Tree), C.c_int32, C.c_void_p, C.c_void_p]
    t = Tree(max_leaves)
    ct = t.c()
    if L.orc_tree_init(C.byref(ct), depth, _p(_f64(lo)), _p(_f64(hi))):
        raise ValueError("orc_tree_init failed")
    return t


def init_leaf(K, lo, hi):
    """The initial mixture of a leaf box (pi, mu_dir, mu_pos, cov as flat arrays)."""
    L = lib()
    L.orc_init_leaf.argtypes = [C.c_int32] + [C.c_void_p] * 6
    pi, mud, mux, cov = np.zeros(K), np.zeros(3 * K), np.zeros(3 * K), np.zeros(15 * K)
    L.orc_init_leaf(K, _p(_f64(lo)), _p(_f64(hi)), _p(pi), _p(mud), _p(mux), _p(cov))
    return {"pi": pi, "mu_dir": mud, "mu_pos": mux, "cov": cov}


def tree_refine(t: Tree, samples, c, K, mix, state, min_init=16):
    """Refines t in place with the samples, copies and initialises leaf mixtures in mix /
    state (arrays sized for t.max_leaves cells). Returns (status, sorted samples, offsets
    [n_leaves + 1])."""
    L = lib()
    i32, i64, vp = C.c_int32, C.c_int64, C.c_void_p
    L.orc_tree_refine.argtypes = [C.POINTER(_Tree), vp, i64, i32, i32, i32] + [vp] * 10
    samples = np.ascontiguousarray(samples, dtype=np.float32)
    N = samples.shape[1]
    sorted_ = np.zeros_like(samples)
    offsets = np.zeros(t.max_leaves + 1, dtype=np.int64)
    for key in ("pi", "mu_dir", "mu_pos", "cov"):
        assert mix[key].dtype == np.float64 and mix[key].flags["C_CONTIGUOUS"]
    ct = t.c()
    st = L.orc_tree_refine(C.byref(ct), _p(samples), N, c, min_init, K, _p(mix["pi"]), _p(mix["mu_dir"]),
                           _p(mix["mu_pos"]), _p(mix["cov"]), _p(state["s0"]), _p(state["s2"]), _p(state["sw"]),
                           _p(state["step"]), _p(sorted_), _p(offsets))
    if st < 0:
        raise ValueError("orc_tree_refine failed")
    return st, sorted_, offsets[:t.n_leaves + 1].copy()


# --- counter-based uniforms -------------------------------------------------------

def philox4x32_10(ctr, key):
    L = lib()
    L.orc_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    L.orc_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def draw_uniforms(seed: int, n: int):
    """(n, 3) uniforms of draws 0..n-1 under ``seed`` (the library's device generator)."""
    L = lib()
    L.orc_draw_uniforms.argtypes = [C.c_uint64, C.c_int64, C.c_void_p]
    u = np.zeros((n, 3))
    L.orc_draw_uniforms(seed, n, _p(u))
    return u


def threads_in_use(threads: int) -> int:
    """The thread count the OpenMP build runs with after asking for `threads`."""
    return int(lib_omp().orc_set_threads(int(threads)))
