"""Seeded synthetic workloads for the spatio-directional mixture path.

This module generates inputs only: path-vertex-like samples (direction, position,
Monte Carlo weight) grouped into spatial cells, initial mixtures, query positions and
uniform random numbers. It holds none of the fitting, conditioning or sampling
arithmetic, and both the GPU library's tests and the oracle's tests draw from it.

The paper trains on path vertices of rendered scenes (Sec. 4.2), which are not available;
the stand-in is a set of planted von Mises-Fisher lobes whose mean direction depends on
the position (parallax towards fixed "emitter" points), with heavy-tailed weights and a
fraction of zero-weight (black) vertices. Cell counts follow the shapes of the workloads
described in the accompanying notes (lognormal, geometric, one huge cell).

Layouts:
  samples  float32 [7, N]: dir x, y, z, pos x, y, z, weight (cells are contiguous ranges)
  offsets  int64 [n_cells + 1]
  mixture  float64: pi [C*K], mu_dir [C*K*3], mu_pos [C*K*3], cov [C*K*15] packed lower
           triangle of the 5x5 covariance in (nu_u, nu_v, x, y, z) order.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# inverse CDF of the chi-square distribution with 3 degrees of freedom at 0.9 (App. B)
CHI2_3_INV_090 = 6.251388631170325


def _normalize(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _any_basis(mu):
    """Two unit vectors orthogonal to each row of mu (Gram-Schmidt against an axis)."""
    helper = np.where(np.abs(mu[..., :1]) < 0.9, np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]))
    t1 = _normalize(helper - np.sum(helper * mu, axis=-1, keepdims=True) * mu)
    t2 = np.cross(mu, t1)
    return t1, t2


def sample_vmf(rng, mu, kappa):
    """One von Mises-Fisher draw per row of mu (N,3) with concentrations kappa (N,),
    using the numerically stable inversion of Jakob (2012)."""
    n = mu.shape[0]
    u = rng.random(n)
    w = 1.0 + np.log(u + (1.0 - u) * np.exp(-2.0 * kappa)) / kappa
    w = np.clip(w, -1.0, 1.0)
    phi = 2.0 * np.pi * rng.random(n)
    t1, t2 = _any_basis(mu)
    r = np.sqrt(np.maximum(0.0, 1.0 - w * w))
    return (w[:, None] * mu + r[:, None] * (np.cos(phi)[:, None] * t1 + np.sin(phi)[:, None] * t2))


@dataclass
class Lobes:
    dirs: np.ndarray      # (L, 3) lobe directions seen from the cube centre
    kappa: np.ndarray     # (L,)
    weight: np.ndarray    # (L,) lobe probabilities
    emitters: np.ndarray  # (L, 3) emitter points (parallax source)


def planted_lobes(seed: int, n_lobes: int = 6, min_sep_deg: float = 45.0,
                  kappa_range=(5.0, 200.0)) -> Lobes:
    rng = np.random.default_rng(seed)
    dirs = []
    while len(dirs) < n_lobes:
        v = _normalize(rng.normal(size=3))
        if all(np.degrees(np.arccos(np.clip(v @ d, -1, 1))) >= min_sep_deg for d in dirs):
            dirs.append(v)
    dirs = np.array(dirs)
    kappa = np.exp(rng.uniform(np.log(kappa_range[0]), np.log(kappa_range[1]), n_lobes))
    weight = rng.dirichlet(np.ones(n_lobes))
    dist = rng.uniform(1.5, 3.0, n_lobes)
    emitters = 0.5 + dist[:, None] * dirs
    return Lobes(dirs, kappa, weight, emitters)


def draw_directions(rng, lobes: Lobes, pos, parallax: bool):
    """Directions for positions pos (N,3): a lobe is chosen by its weight, and its mean
    points from the position towards the lobe's emitter when parallax is on."""
    n = pos.shape[0]
    j = rng.choice(len(lobes.kappa), size=n, p=lobes.weight)
    if parallax:
        mu = _normalize(lobes.emitters[j] - pos)
    else:
        mu = lobes.dirs[j]
    return sample_vmf(rng, mu, lobes.kappa[j]), j


def draw_weights(rng, n, sigma=1.5, zero_frac=0.1):
    w = np.exp(sigma * rng.normal(size=n))
    if zero_frac > 0:
        w[rng.random(n) < zero_frac] = 0.0
    return w


# --- cells ------------------------------------------------------------------

@dataclass
class Grid:
    dims: tuple  # cells along x, y, z; the grid spans the unit cube

    @property
    def n_cells(self):
        return int(np.prod(self.dims))

    def boxes(self):
        nx, ny, nz = self.dims
        ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
        lo = np.stack([ix.ravel() / nx, iy.ravel() / ny, iz.ravel() / nz], axis=1)
        size = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
        return lo, np.broadcast_to(size, lo.shape).copy()


def counts_lognormal(rng, n_cells, mu=6.45, sigma=1.0, lo=64, hi=8192):
    return np.clip(np.round(np.exp(mu + sigma * rng.normal(size=n_cells))), lo, hi).astype(np.int64)


def counts_geometric(rng, n_cells, p=1.0 / 1009.0, lo=16, hi=32768):
    return np.clip(lo + rng.geometric(p, size=n_cells) - 1, lo, hi).astype(np.int64)


@dataclass
class Batch:
    samples: np.ndarray   # float32 [7, N]
    offsets: np.ndarray   # int64 [C+1]
    lobe: np.ndarray      # int32 [N] planted lobe of each sample (for recovery checks)


def make_batch(seed: int, counts, box_lo, box_size, lobes: Lobes, parallax=True,
               weight_sigma=1.5, zero_frac=0.1) -> Batch:
    rng = np.random.default_rng(seed)
    counts = np.asarray(counts, dtype=np.int64)
    offsets = np.zeros(counts.size + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    n = int(offsets[-1])
    cell = np.repeat(np.arange(counts.size), counts)
    pos = box_lo[cell] + rng.random((n, 3)) * box_size[cell]
    dirs, lobe = draw_directions(rng, lobes, pos, parallax)
    w = draw_weights(rng, n, weight_sigma, zero_frac)
    s = np.empty((7, n), dtype=np.float32)
    s[0:3] = dirs.T
    s[3:6] = pos.T
    s[6] = w
    return Batch(s, offsets, lobe.astype(np.int32))


# --- initial mixtures (harness side; App. B shapes without surface normals) ---

_CUBE_DIRS = _normalize(np.array([[sx, sy, sz] for sx in (1, -1) for sy in (1, -1) for sz in (1, -1)],
                                 dtype=np.float64))


def _tri(d, e):
    return d * (d + 1) // 2 + e


def initial_mixtures(box_lo, box_size, K: int) -> dict:
    """K/8 spatial means crossed with 8 directions at the cube vertices; directional
    covariance (2 pi / 8) I; isotropic spatial covariance r^2 I / chi2_3^-1(0.9) with
    r = 2 d / (number of spatial means), d the longest side of the cell; pi = 1/K."""
    C = box_lo.shape[0]
    n_dir = min(8, K)
    n_pos = max(1, (K + n_dir - 1) // n_dir)
    centre = box_lo + 0.5 * box_size
    d = box_size.max(axis=1)
    order = np.argsort(-box_size, axis=1, kind="stable")
    mu_pos = np.zeros((C, K, 3))
    mu_dir = np.zeros((C, K, 3))
    for k in range(K):
        s, v = divmod(k, n_dir)
        off = np.zeros((C, 3))
        if n_pos == 2:
            sign = -1.0 if s == 0 else 1.0
            off[np.arange(C), order[:, 0]] = sign * d / 4
        elif n_pos == 4:
            off[np.arange(C), order[:, 0]] = (-1.0 if s % 2 == 0 else 1.0) * d / 4
            off[np.arange(C), order[:, 1]] = (-1.0 if s // 2 == 0 else 1.0) * d / 4
        elif n_pos > 1:
            off[np.arange(C), order[:, 0]] = ((s + 0.5) / n_pos - 0.5) * d
        mu_pos[:, k] = centre + off
        mu_dir[:, k] = _CUBE_DIRS[v]
    r = 2.0 * d / n_pos
    cov = np.zeros((C, K, 15))
    cov[:, :, _tri(0, 0)] = 2.0 * np.pi / 8.0
    cov[:, :, _tri(1, 1)] = 2.0 * np.pi / 8.0
    for a in range(3):
        cov[:, :, _tri(2 + a, 2 + a)] = (r * r / CHI2_3_INV_090)[:, None]
    return {"pi": np.full(C * K, 1.0 / K), "mu_dir": mu_dir.reshape(-1), "mu_pos": mu_pos.reshape(-1),
            "cov": cov.reshape(-1)}


def copy_mix(mix: dict) -> dict:
    return {k: v.copy() for k, v in mix.items()}


# --- queries -----------------------------------------------------------------

def make_queries(seed: int, box_lo, box_size, per_cell: int):
    """per_cell uniform positions in every cell box, sorted by cell. Returns float32
    positions (nq, 3) and int32 cell ids (nq,)."""
    rng = np.random.default_rng(seed)
    C = box_lo.shape[0]
    cell = np.repeat(np.arange(C, dtype=np.int32), per_cell)
    pos = box_lo[cell] + rng.random((cell.size, 3)) * box_size[cell]
    return pos.astype(np.float32), cell


def make_uniforms(seed: int, n: int):
    """Uniform numbers in [0, 1) for n draws, float32 (n, 3)."""
    rng = np.random.default_rng(seed)
    return rng.random((n, 3), dtype=np.float32)


# --- workload presets ------------------------------------------------------

def workload(name: str, seed: int = 1234, scale: float = 1.0):
    """Named workloads. scale < 1 shrinks the cell grid / sample counts for fast tests
    while keeping the count distribution's shape.

    single     one cell = unit cube, N = 16384, K = 16
    cells4k    16^3 cells, counts lognormal(6.45, 1) clipped to [64, 8192], K = 16
    cells16k   32x32x16 cells, counts 16 + Geom(1/1009) - 1 clipped to [16, 32768], K = 16
    huge       one cell, 2^24 samples, K = 32, weights lognormal(0, 2.5), no zeros
    """
    lobes = planted_lobes(seed)
    rng = np.random.default_rng(seed + 1)
    if name == "single":
        grid = Grid((1, 1, 1))
        counts = np.array([max(16, int(round(16384 * scale)))])
        K, wsig, zf = 16, 1.5, 0.1
    elif name == "cells4k":
        side = max(1, int(round(16 * scale ** (1 / 3))))
        grid = Grid((side, side, side))
        counts = counts_lognormal(rng, grid.n_cells)
        K, wsig, zf = 16, 1.5, 0.1
    elif name == "cells16k":
        f = scale ** (1 / 3)
        grid = Grid((max(1, int(round(32 * f))), max(1, int(round(32 * f))), max(1, int(round(16 * f)))))
        counts = counts_geometric(rng, grid.n_cells)
        K, wsig, zf = 16, 1.5, 0.1
    elif name == "huge":
        grid = Grid((1, 1, 1))
        counts = np.array([max(64, int(round((1 << 24) * scale)))])
        K, wsig, zf = 32, 2.5, 0.0
    else:
        raise ValueError(name)
    lo, size = grid.boxes()
    return {"name": name, "grid": grid, "counts": counts, "K": K, "box_lo": lo, "box_size": size,
            "lobes": lobes, "weight_sigma": wsig, "zero_frac": zf, "seed": seed}


def workload_batch(wl: dict, batch_index: int = 0, parallax: bool = True) -> Batch:
    return make_batch(wl["seed"] + 1000 + batch_index, wl["counts"], wl["box_lo"], wl["box_size"],
                      wl["lobes"], parallax=parallax, weight_sigma=wl["weight_sigma"],
                      zero_frac=wl["zero_frac"])


# --- BSDF models and product-sampling queries ----------------------------------------
#
# A BSDF model is a 5-D tangent-space mixture like the radiance mixtures, over (local
# incident direction; outgoing polar angle, outgoing azimuth, roughness): the three
# Euclidean coordinates take the place of the position. Queries carry those three
# inputs and a local-to-world rotation (the shading frame).

BSDF_PAR_LO = np.array([0.0, 0.0, 0.05])
BSDF_PAR_HI = np.array([1.4, 2.0 * np.pi, 0.6])


def random_rotations(rng, n):
    """n rotation matrices (det +1), uniform over SO(3), shape (n, 3, 3)."""
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
                  2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                  2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], 1)
    return R.reshape(n, 3, 3)


def bsdf_mixtures(seed: int, n_models: int, Kb: int, lobe_sd=(0.08, 0.35)) -> dict:
    """Random BSDF models: means in the upper hemisphere, directional standard deviations
    in lobe_sd, inputs spread over [BSDF_PAR_LO, BSDF_PAR_HI], correlated through a random
    lower-triangular factor; Dirichlet(2) weights."""
    rng = np.random.default_rng(seed)
    n = n_models * Kb
    d = rng.normal(size=(n, 3))
    d[:, 2] = np.abs(d[:, 2]) + 0.6
    mu_dir = _normalize(d)
    mu_pos = BSDF_PAR_LO + rng.random((n, 3)) * (BSDF_PAR_HI - BSDF_PAR_LO)
    sd_dir = lobe_sd[0] + rng.random(n) * (lobe_sd[1] - lobe_sd[0])
    diag = np.stack([sd_dir, sd_dir * (0.6 + 0.8 * rng.random(n)), np.full(n, 0.25), np.full(n, 0.8),
                     np.full(n, 0.1)], 1)
    cov = np.zeros((n, 15))
    for i in range(n):
        Lm = np.diag(diag[i])
        for a in range(5):
            for b in range(a):
                Lm[a, b] = 0.3 * rng.uniform(-1, 1) * np.sqrt(diag[i, a] * diag[i, b])
        S = Lm @ Lm.T
        cov[i] = [S[a, b] for a in range(5) for b in range(a + 1)]
    pi = rng.dirichlet(np.full(Kb, 2.0), size=n_models).reshape(-1)
    return {"pi": pi, "mu_dir": mu_dir.reshape(-1), "mu_pos": mu_pos.reshape(-1), "cov": cov.reshape(-1)}


def bsdf_queries(seed: int, nq: int, n_models: int = 1):
    """Per query: the BSDF inputs (float64 [nq, 3]), the model index and a shading frame
    (local-to-world rotation, [nq, 3, 3])."""
    rng = np.random.default_rng(seed)
    bpar = BSDF_PAR_LO + rng.random((nq, 3)) * (BSDF_PAR_HI - BSDF_PAR_LO)
    bcell = rng.integers(0, n_models, nq).astype(np.int32)
    return bpar, bcell, random_rotations(rng, nq)


def ggx_training_batch(seed: int, n: int) -> Batch:
    """Training samples of a BSDF model for an isotropic GGX reflection lobe, drawn the
    way the BSDF's own importance sampler would: outgoing polar angle, azimuth and
    roughness uniform over the input box, a microfacet normal from the GGX distribution
    of normals (D(h) cos(theta_h)), and the mirror of the outgoing direction about it.
    Directions below the surface get weight 0. One cell, float32 [7][n]."""
    rng = np.random.default_rng(seed)
    par = BSDF_PAR_LO + rng.random((n, 3)) * (BSDF_PAR_HI - BSDF_PAR_LO)
    th_o, ph_o, alpha = par.T
    wo = np.stack([np.sin(th_o) * np.cos(ph_o), np.sin(th_o) * np.sin(ph_o), np.cos(th_o)], 1)
    u1, u2 = rng.random(n), rng.random(n)
    tan2 = alpha * alpha * u1 / (1.0 - u1)
    cos_h = 1.0 / np.sqrt(1.0 + tan2)
    sin_h = np.sqrt(np.maximum(0.0, 1.0 - cos_h * cos_h))
    ph_h = 2.0 * np.pi * u2
    h = np.stack([sin_h * np.cos(ph_h), sin_h * np.sin(ph_h), cos_h], 1)
    wi = 2.0 * (wo * h).sum(1, keepdims=True) * h - wo
    wi = _normalize(wi)
    smp = np.zeros((7, n), dtype=np.float32)
    smp[0:3] = wi.T
    smp[3:6] = par.T
    smp[6] = (wi[:, 2] > 0.0).astype(np.float32)
    return Batch(smp, np.array([0, n], dtype=np.int64), np.zeros(n, dtype=np.int32))
