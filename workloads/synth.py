"""Seeded vector generators (numpy PCG64).

Every generator draws i.i.d. points and the caller splits them into
contiguous blocks in the configured size order, which is the random
partition of one dataset into sub-indexes that the paper merges
(Section 3.1, the composition study, and Exp.4).

Distributions:
  gmm       isotropic Gaussian mixture: centres ~ N(0, centre_std^2 I),
            points = centre + sigma * N(0, I), float32.
  sift      SIFT-shaped integers: centre coordinates
            centre_base + centre_scale * |N(0, 1)|, points = centre +
            sigma * N(0, I), rounded half-to-even and clipped to [0, 255].
  gmm_unit  gmm, then each row normalised in float64 and rounded to float32.
  vmf       von Mises-Fisher mixture on the unit sphere: mean directions are
            normalised Gaussians, samples use Wood's (1994) rejection
            sampler for the cosine to the mean direction.
"""

from __future__ import annotations

import numpy as np

from .configs import WorkloadConfig

_CHUNK = 1 << 18


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _normalise_rows(x: np.ndarray) -> np.ndarray:
    x64 = x.astype(np.float64)
    nrm = np.sqrt(np.einsum("ij,ij->i", x64, x64))
    nrm[nrm == 0.0] = 1.0
    return (x64 / nrm[:, None]).astype(np.float32)


def _wood_cosines(rng: np.random.Generator, n: int, dim: int,
                  kappa: float) -> np.ndarray:
    """Cosines w = <x, mu> of vMF(mu, kappa) samples on S^{dim-1}."""
    m1 = dim - 1.0
    b = (-2.0 * kappa + np.sqrt(4.0 * kappa * kappa + m1 * m1)) / m1
    x0 = (1.0 - b) / (1.0 + b)
    c = kappa * x0 + m1 * np.log(1.0 - x0 * x0)
    out = np.empty(n, dtype=np.float64)
    todo = np.arange(n)
    while todo.size:
        z = rng.beta(m1 / 2.0, m1 / 2.0, size=todo.size)
        w = (1.0 - (1.0 + b) * z) / (1.0 - (1.0 - b) * z)
        u = rng.uniform(size=todo.size)
        ok = kappa * w + m1 * np.log(1.0 - x0 * w) - c >= np.log(u)
        out[todo[ok]] = w[ok]
        todo = todo[~ok]
    return out


def _draw(cfg: WorkloadConfig, n: int, seed: int) -> np.ndarray:
    p = cfg.params()
    d = cfg.dim
    rng = _rng(seed)
    # Cluster structure is shared by base and queries: it comes from the
    # data seed, whichever stream draws the points.
    crng = _rng(cfg.seed + 77)
    C = int(p["clusters"])
    if cfg.dist in ("gmm", "gmm_unit"):
        centres = crng.normal(0.0, p["centre_std"], size=(C, d)).astype(np.float32)
    elif cfg.dist == "sift":
        centres = (p["centre_base"] + p["centre_scale"]
                   * np.abs(crng.standard_normal(size=(C, d)))).astype(np.float32)
    elif cfg.dist == "vmf":
        centres = _normalise_rows(crng.standard_normal(size=(C, d)))
    else:
        raise ValueError(f"unknown distribution {cfg.dist!r}")

    labels = rng.integers(0, C, size=n)
    out = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        lab = labels[s:e]
        if cfg.dist in ("gmm", "gmm_unit", "sift"):
            noise = rng.standard_normal(size=(e - s, d), dtype=np.float32)
            blk = centres[lab] + np.float32(p["sigma"]) * noise
            if cfg.dist == "sift":
                blk = np.clip(np.rint(blk), 0.0, 255.0)
            elif cfg.dist == "gmm_unit":
                blk = _normalise_rows(blk)
        else:  # vmf
            mu = centres[lab].astype(np.float64)
            w = _wood_cosines(rng, e - s, d, p["kappa"])
            v = rng.standard_normal(size=(e - s, d))
            v -= np.einsum("ij,ij->i", v, mu)[:, None] * mu
            v /= np.sqrt(np.einsum("ij,ij->i", v, v))[:, None]
            blk = _normalise_rows(w[:, None] * mu
                                  + np.sqrt(1.0 - w * w)[:, None] * v)
        out[s:e] = blk
    return out


def make_vectors(cfg: WorkloadConfig) -> np.ndarray:
    """Base vectors X (n_total x dim, float32, row-major) in global-id order."""
    return _draw(cfg, cfg.n_total, cfg.seed)


def make_queries(cfg: WorkloadConfig, n: int | None = None) -> np.ndarray:
    """Held-out queries from the same distribution (seed + 1000)."""
    return _draw(cfg, cfg.n_queries if n is None else n, cfg.seed + 1000)


def split_sizes(cfg: WorkloadConfig):
    """(offset, n) of every sub-index."""
    return list(zip(cfg.offsets(), cfg.sizes))
