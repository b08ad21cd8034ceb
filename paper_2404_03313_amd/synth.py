"""Seeded synthetic hyperspectral workloads (inputs only; none of the solver's arithmetic).

The paper evaluates on cropped real scenes (Jasper Ridge 100x100x198, Pavia University
120x120x98, Beltsville 100x100x128; Sec. IV-A) normalised to [0, 1] and corrupted by
mixtures of Gaussian noise, salt-and-pepper noise and vertical stripes (Sec. IV-A, noise
cases 1-8). Those scenes are not available here, so this module synthesises scenes of
the same kind: linear mixtures of smooth spectra over piecewise-constant abundance maps.

Observation model (eq. Obsevation_model): v = u_bar + s_bar + t_bar + n.
Layering: clean + Gaussian + stripes first, salt-and-pepper overwrites last, so a
corrupted voxel carries no Gaussian part (this matches the (1 - p_s) factors of the
radius rule eq. RadiusSet). The exact decomposition is returned so that the radii can be
set from the true noise energies: eps = rho*||n_eff||_2, alpha = rho*||s_bar||_1,
beta = rho*||t_bar||_1 with rho = 0.95 (eq. RadiusSet uses the same rho on the expected
energies).

Array layout: C-contiguous (N1, N2, N3) = (rows i, columns j, bands b), band fastest.
Everything is float64 except ``v`` which is also returned rounded to float32 (the
solver's input); ``v64`` is that float32 value widened back, so both solvers see
bit-identical observations.
"""
from __future__ import annotations

import dataclasses
from typing import Dict

import numpy as np


@dataclasses.dataclass(frozen=True)
class HSIConfig:
    n1: int
    n2: int
    n3: int
    endmembers: int = 4
    cells: int = 8
    sigma: float = 0.1
    p_sp: float = 0.05          # salt-and-pepper rate (fraction of voxels)
    p_stripe: float = 0.05      # fraction of columns striped, per band
    stripe_amp: float = 0.3     # stripe offsets ~ U[-amp, amp]
    rho: float = 0.95
    seed: int = 1


# Named workloads (shapes, noise levels, block sizes and iteration counts of the
# measurement plan). "c1" is the small parity case, "c2" the throughput case.
WORKLOADS: Dict[str, dict] = {
    "c1": dict(cfg=HSIConfig(32, 32, 16, endmembers=4, cells=8, sigma=0.1, p_sp=0.05,
                             p_stripe=0.05, seed=1), k=(3, 3), iters=200),
    "c2": dict(cfg=HSIConfig(256, 256, 128, endmembers=12, cells=64, sigma=0.05, p_sp=0.05,
                             p_stripe=0.1, seed=2), k=(4, 4), iters=500),
    # the paper's experimental shape (a 100 x 100 x 198 scene, 10 x 10 windows, stop rule
    # 1e-5) with its Case 8 noise: Gaussian 0.1, salt-and-pepper 0.05, stripes on 5 % of the
    # columns with offsets ~ U[-0.5, 0.5]
    "paper10": dict(cfg=HSIConfig(100, 100, 198, endmembers=8, cells=32, sigma=0.1, p_sp=0.05,
                                  p_stripe=0.05, stripe_amp=0.5, seed=10), k=(10, 10),
                    rel_tol=1e-5),
    # the shapes of the paper's two other scenes of its running-time table, same noise
    "paper10_120x120x98": dict(cfg=HSIConfig(120, 120, 98, endmembers=8, cells=32, sigma=0.1,
                                             p_sp=0.05, p_stripe=0.05, stripe_amp=0.5, seed=11),
                               k=(10, 10), rel_tol=1e-5),
    "paper10_100x100x128": dict(cfg=HSIConfig(100, 100, 128, endmembers=8, cells=32, sigma=0.1,
                                              p_sp=0.05, p_stripe=0.05, stripe_amp=0.5, seed=12),
                                k=(10, 10), rel_tol=1e-5),
    # learned initial estimate: applied to one large scene, compared with the zero start
    "c5": dict(cfg=HSIConfig(512, 512, 191, endmembers=12, cells=128, sigma=0.1, p_sp=0.1,
                             p_stripe=0.1, seed=5), k=(4, 4), rel_tol=1e-4),
}


def batch_configs(count: int = 24, seed: int = 4):
    """The uneven batch: `count` images with N1, N2 ~ U{64..307}, N3 ~ U{32..191}, sigma,
    salt-and-pepper and stripe rates each drawn from {0.05, 0.1}, block 4 x 4 (seeded)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n1, n2 = (int(x) for x in rng.integers(64, 308, size=2))
        n3 = int(rng.integers(32, 192))
        sig, psp, pst = (float(x) for x in rng.choice([0.05, 0.1], size=3))
        out.append(HSIConfig(n1, n2, n3, endmembers=8, cells=32, sigma=sig, p_sp=psp,
                             p_stripe=pst, seed=seed * 1000 + i))
    return out


def _endmembers(rng: np.random.Generator, e: int, n3: int) -> np.ndarray:
    """E smooth spectra, each a sum of three Gaussian bumps over the band index."""
    b = np.arange(n3, dtype=np.float64)
    spec = np.zeros((e, n3))
    for m in range(e):
        for _ in range(3):
            amp = rng.uniform(0.2, 1.0)
            ctr = rng.uniform(0.0, n3 - 1.0)
            wid = rng.uniform(n3 / 20.0, n3 / 5.0)
            spec[m] += amp * np.exp(-0.5 * ((b - ctr) / wid) ** 2)
    return spec


def _abundances(rng: np.random.Generator, n1: int, n2: int, e: int, cells: int) -> np.ndarray:
    """Piecewise-constant Dirichlet(1) abundances on seeded Voronoi cells plus a linear ramp."""
    seeds = np.stack([rng.uniform(0, n1, cells), rng.uniform(0, n2, cells)], axis=1)
    ii, jj = np.meshgrid(np.arange(n1, dtype=np.float64), np.arange(n2, dtype=np.float64),
                         indexing="ij")
    d2 = (ii[..., None] - seeds[:, 0]) ** 2 + (jj[..., None] - seeds[:, 1]) ** 2
    label = np.argmin(d2, axis=-1)
    vec = rng.dirichlet(np.ones(e), size=cells)            # (cells, e)
    ab = vec[label]                                         # (n1, n2, e)
    ci = rng.uniform(-0.2, 0.2, e)
    cj = rng.uniform(-0.2, 0.2, e)
    ramp = ci * (ii[..., None] / max(n1 - 1, 1)) + cj * (jj[..., None] / max(n2 - 1, 1))
    return np.maximum(ab + ramp, 0.0)


def make_hsi(cfg: HSIConfig) -> dict:
    """Return a dict with v (float32), v64, u_true, s_true, t_true, n_eff and radii."""
    rng = np.random.Generator(np.random.PCG64(cfg.seed))
    n1, n2, n3 = cfg.n1, cfg.n2, cfg.n3
    spec = _endmembers(rng, cfg.endmembers, n3)
    ab = _abundances(rng, n1, n2, cfg.endmembers, cfg.cells)
    u = ab @ spec                                           # (n1, n2, n3)
    lo, hi = u.min(), u.max()
    u = (u - lo) / (hi - lo) if hi > lo else np.zeros_like(u)

    n = rng.normal(0.0, cfg.sigma, size=u.shape) if cfg.sigma > 0 else np.zeros_like(u)

    t = np.zeros_like(u)
    ncols = int(round(cfg.p_stripe * n2))
    if ncols > 0:
        for b in range(n3):
            cols = rng.choice(n2, size=ncols, replace=False)
            t[:, cols, b] = rng.uniform(-cfg.stripe_amp, cfg.stripe_amp, size=ncols)[None, :]

    v = u + n + t
    nsp = int(round(cfg.p_sp * u.size))
    mask = np.zeros(u.size, dtype=bool)
    if nsp > 0:
        idx = rng.choice(u.size, size=nsp, replace=False)
        mask[idx] = True
        vals = (rng.uniform(size=nsp) < 0.5).astype(np.float64)
        vflat = v.reshape(-1)
        vflat[idx] = vals
    mask = mask.reshape(u.shape)

    v32 = v.astype(np.float32)
    v64 = v32.astype(np.float64)
    n_eff = np.where(mask, 0.0, n)
    s = v64 - u - t - n_eff                                 # exact remainder (incl. f32 rounding)
    radii = dict(eps=cfg.rho * float(np.linalg.norm(n_eff.ravel())),
                 alpha=cfg.rho * float(np.abs(s).sum()),
                 beta=cfg.rho * float(np.abs(t).sum()))
    # Degenerate noise cases still need strictly positive radii.
    for key in radii:
        if radii[key] <= 0.0:
            radii[key] = 1e-3
    return dict(v=v32, v64=v64, u_true=u, s_true=s, t_true=t, n_eff=n_eff, mask=mask,
                radii=radii, cfg=cfg)


def small_random(n1: int, n2: int, n3: int, seed: int = 0) -> np.ndarray:
    """Plain uniform [0,1) cube for operator-level tests (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 1.0, size=(n1, n2, n3))


def cnn_train_configs(count: int = 2000, seed0: int = 5000, n: int = 64, n3: int = 64):
    """Training scenes for the initial-estimate network: `count` n x n x n3 images with seeds
    seed0, seed0 + 1, ..., sigma, salt-and-pepper and stripe rates each drawn from
    {0.05, 0.1} and 4..12 endmembers (seeded)."""
    rng = np.random.default_rng(seed0)
    out = []
    for i in range(count):
        sig, psp, pst = (float(x) for x in rng.choice([0.05, 0.1], size=3))
        e = int(rng.integers(4, 13))
        out.append(HSIConfig(n, n, n3, endmembers=e, cells=16, sigma=sig, p_sp=psp,
                             p_stripe=pst, seed=seed0 + i))
    return out


CNN_CHANNELS = (1, 32, 32, 32, 32, 1)


def cnn_init(seed: int = 0, last_scale: float = 0.1) -> np.ndarray:
    """Initial parameters of the network (float32 vector in the documented layout: per
    layer weights [27][cout][cin] then cout biases): He-normal weights (std sqrt(2/(27 cin))),
    the last layer scaled by last_scale, zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for l in range(5):
        ci, co = CNN_CHANNELS[l], CNN_CHANNELS[l + 1]
        std = np.sqrt(2.0 / (27 * ci)) * (last_scale if l == 4 else 1.0)
        parts.append(rng.normal(0.0, std, size=27 * co * ci))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def cnn_random_params(seed: int = 0, bias: float = 0.05) -> np.ndarray:
    """Parameters for numerics tests: He-normal weights and N(0, bias) biases, so that every
    layer has active and inactive ReLUs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for l in range(5):
        ci, co = CNN_CHANNELS[l], CNN_CHANNELS[l + 1]
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (27 * ci)), size=27 * co * ci))
        parts.append(rng.normal(0.0, bias, size=co))
    return np.concatenate(parts).astype(np.float32)
