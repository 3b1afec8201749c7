"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers (numpy PCG64 via ``default_rng``); it
holds none of the search method's arithmetic.  Every array is float32
row-major ``[n][D]``.

Workloads (the paper's test rig draws uniform points in the unit hypercube,
Sec. 4; the other distributions stand in for clustered and surface-like data):
  * ``uniform``      -- U[0,1)^D, values are multiples of 2^-24.
  * ``gmm``          -- equal-weight Gaussian mixture, float64 draws cast to
                        float32 (round to nearest), no clipping.
  * ``clustered_lr`` -- 256 clusters with sigma log-uniform in [0.002, 0.05];
                        queries are 90 % mixture, 10 % uniform.
  * ``shells``       -- points on random sphere shells (radius U[0.01, 0.1]),
                        radial noise N(0, 1e-4).
  * ``batched_jobs`` -- metadata for many independent trees of uneven size and
                        dimension.
"""
from __future__ import annotations

import numpy as np


def uniform(n: int, dim: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((n, dim), dtype=np.float32)


def gmm(n: int, dim: int, seed: int, n_centers: int = 64, sigma: float = 0.01,
        center_seed: int = 7) -> np.ndarray:
    centers = np.random.default_rng(center_seed).random((n_centers, dim))
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, n_centers, size=n)
    x = centers[lab] + sigma * rng.standard_normal((n, dim))
    return x.astype(np.float32)


def _lr_mixture(center_seed: int = 7, n_centers: int = 256, dim: int = 3):
    rng = np.random.default_rng(center_seed)
    centers = rng.random((n_centers, dim))
    sig = np.exp(rng.uniform(np.log(0.002), np.log(0.05), size=n_centers))
    return centers, sig


def clustered_lr_points(n: int, seed: int = 0, dim: int = 3) -> np.ndarray:
    centers, sig = _lr_mixture(dim=dim)
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, len(centers), size=n)
    x = centers[lab] + sig[lab, None] * rng.standard_normal((n, dim))
    return x.astype(np.float32)


def clustered_lr_queries(n: int, seed: int = 1, dim: int = 3, frac_mixture: float = 0.9) -> np.ndarray:
    centers, sig = _lr_mixture(dim=dim)
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, len(centers), size=n)
    x = centers[lab] + sig[lab, None] * rng.standard_normal((n, dim))
    uni = rng.random((n, dim))
    pick = rng.random(n) < frac_mixture
    x = np.where(pick[:, None], x, uni)
    return x.astype(np.float32)


def shells(n: int, seed: int, n_shells: int = 1000, center_seed: int = 7) -> np.ndarray:
    crng = np.random.default_rng(center_seed)
    centers = crng.random((n_shells, 3))
    radii = crng.uniform(0.01, 0.1, size=n_shells)
    rng = np.random.default_rng(seed)
    out = np.empty((n, 3), np.float32)
    step = 1 << 22
    for lo in range(0, n, step):
        m = min(step, n - lo)
        lab = rng.integers(0, n_shells, size=m)
        d = rng.standard_normal((m, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        r = radii[lab] + 1e-4 * rng.standard_normal(m)
        out[lo:lo + m] = (centers[lab] + d * r[:, None]).astype(np.float32)
    return out


def batched_jobs(n_jobs: int = 512, seed: int = 42, n_min: int = 1000, n_max: int = 2_000_000):
    """Job metadata: list of dicts {n, dim, dist, k, point_seed, query_seed}."""
    rng = np.random.default_rng(seed)
    ns = np.round(np.exp(rng.uniform(np.log(n_min), np.log(n_max), size=n_jobs))).astype(np.int64)
    dims = rng.choice([2, 3, 4], size=n_jobs)
    dists = rng.choice(["uniform", "gmm"], size=n_jobs)
    ks = rng.choice([1, 8, 32], size=n_jobs)
    return [dict(n=int(ns[t]), dim=int(dims[t]), dist=str(dists[t]), k=int(ks[t]),
                 point_seed=1000 + t, query_seed=2000 + t) for t in range(n_jobs)]


def job_arrays(job: dict):
    """(points, queries) for one batched job; queries come from the same distribution."""
    n, dim = job["n"], job["dim"]
    if job["dist"] == "uniform":
        return uniform(n, dim, job["point_seed"]), uniform(n, dim, job["query_seed"])
    return (gmm(n, dim, job["point_seed"], center_seed=7 + job["point_seed"]),
            gmm(n, dim, job["query_seed"], center_seed=7 + job["point_seed"]))


def training_queries(name: str, n: int = 1 << 20, seed: int = 7) -> np.ndarray:
    """Queries for training the radius model on a named workload: same
    distribution as the workload's queries, a different seed."""
    if name in ("uniform-16k", "uniform-1m"):
        return uniform(n, 3, seed)
    if name == "gmm64-1m":
        return gmm(n, 3, seed)
    if name == "clustered-10m":
        return clustered_lr_queries(n, seed)
    if name == "shells-100m":
        return shells(n, seed)
    raise KeyError(name)


def workload(name: str):
    """(points, queries) for a named workload."""
    if name == "uniform-16k":
        return uniform(16384, 3, 0), uniform(16384, 3, 1)
    if name == "uniform-1m":
        return uniform(1 << 20, 3, 0), uniform(1 << 20, 3, 1)
    if name == "gmm64-1m":
        return gmm(1 << 20, 3, 0), gmm(1 << 20, 3, 1)
    if name == "clustered-10m":
        return clustered_lr_points(10_000_000, 0), clustered_lr_queries(10_000_000, 1)
    if name == "shells-100m":
        return shells(100_000_000, 0), shells(100_000_000, 1)
    if name == "uniform4d-1m-q10m":
        return uniform(1 << 20, 4, 0), uniform(10_000_000, 4, 1)
    raise KeyError(name)
